"""Scale configuration: N = 512^3 strongly clustered particles (1000 halos
hold 50 %), PM grid 1024^3, rungs 0-7 from grid-count density.  The FP32
forward force for the 8 nested rung subsets in one persistent launch, and
the FP32 adjoint with all particles active, are checked on 4096 seeded
receivers (512 per rung) against the FP64 oracle over all N suppliers.

The set holds about 3.7e12 ordered pairs within r_cut (about 2.8e4
neighbours per particle, up to 2e5 in halo cores), so each GPU call runs for
seconds and the generator for about a minute."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload, stratified_by_rung
from workloads.generators import gaussian_weights

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


@pytest.fixture(scope="module")
def scale512():
    print("generating scale512 (N=512^3, 1000 halos, grid-count rungs)", flush=True)
    wl = make_workload("scale512")
    idx = stratified_by_rung(wl.rung, 512, wl.config_id)
    print("generated; sampled receivers per rung:",
          np.bincount(wl.rung[idx], minlength=8).tolist(), flush=True)
    return wl, idx


def test_scale512_batched_fp32(env, scale512):
    torch, p3, ctx = env
    wl, idx = scale512
    thr = list(range(8))
    ctx.set_config(subtiles_per_dim=2, item_target=4096, cluster_size=32, screen=1)
    ctx.set_timing(True)
    try:
        out = ctx.force_batched(to_dev(torch, wl.pos), None, to_dev(torch, wl.rung), thr,
                                box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
        torch.cuda.synchronize()
        st = ctx.stats()
    finally:
        ctx.set_config()
        ctx.set_timing(False)
    print("batched fp32", st, flush=True)
    assert st["receivers"] == sum(int((wl.rung >= k).sum()) for k in thr)
    rows = torch.from_numpy(idx).to(out.device)
    got_all = out[:, rows].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    print("oracle on %d receivers" % idx.size, flush=True)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled")
    print("oracle neighbours: mean %.0f max %d" % (cnt.mean(), cnt.max()), flush=True)
    for k in thr:
        sel = wl.rung[idx] >= k
        e = oracle.errors(got_all[k][sel], ref[sel], absum[sel])
        print("subset", k, int(sel.sum()), e, flush=True)
        assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], (k, e)
        assert np.all(got_all[k][~sel] == 0)


def test_scale512_adjoint_fp32(env, scale512):
    torch, p3, ctx = env
    wl, idx = scale512
    w = gaussian_weights(wl.n, wl.config_id)
    ctx.set_timing(True)
    g = ctx.force_backward(to_dev(torch, wl.pos), None, None, to_dev(torch, w), box=1.0,
                           x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    torch.cuda.synchronize()
    print("adjoint fp32", ctx.stats(), flush=True)
    ctx.set_timing(False)
    got = g[torch.from_numpy(idx).to(g.device)].cpu().numpy()
    del g
    torch.cuda.empty_cache()
    print("oracle VJP on %d rows" % idx.size, flush=True)
    ref = oracle.vjp(wl.pos, None, None, w, 1.0, wl.x_s, wl.r_cut, kidx=idx, method="tiled")
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    row = np.max(np.linalg.norm(got - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    print("rel L2 %.3e  max row %.3e" % (rel, row), flush=True)
    assert rel <= TOL["fp32"] and row <= TOL["fp32"], (rel, row)
