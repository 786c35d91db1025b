"""Rung-batched launch: the nested receiver subsets S_k = {rung >= k} of one
rung-0 step, all at the same positions, in one persistent launch."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload, stratified_by_rung

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


@pytest.mark.parametrize("csize,screen", [(64, 0), (8, 1), (32, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_matches_oracle_and_single_calls(env, prec, csize, screen):
    torch, p3, ctx = env
    print("clustered256 recipe at n_side=48 with rungs", prec, csize, screen, flush=True)
    ctx.set_config(cluster_size=csize, screen=screen)
    try:
        _batched_vs_oracle(env, prec)
    finally:
        ctx.set_config()


def _batched_vs_oracle(env, prec):
    torch, p3, ctx = env
    wl = make_workload("clustered256", n_side=48)
    thr = list(range(8))
    pos, mass, rung = to_dev(torch, wl.pos), to_dev(torch, wl.mass), to_dev(torch, wl.rung)
    out = ctx.force_batched(pos, mass, rung, thr, box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                            precision=prec).cpu().numpy()
    st = ctx.stats()
    sizes = [int((wl.rung >= k).sum()) for k in thr]
    assert st["receivers"] == sum(sizes)
    total = 0
    for k in thr:
        act = (wl.rung >= k).astype(np.uint8)
        ref, cnt, absum = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, active=act)
        total += int(cnt.sum())
        e = oracle.errors(out[k][act == 1], ref[act == 1], absum[act == 1])
        assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], (k, e)
        assert np.all(out[k][act == 0] == 0)
        single = ctx.force(pos, mass, to_dev(torch, act), box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                           precision=prec).cpu().numpy()
        assert np.max(np.abs(single - out[k])) <= 1e-12 * np.max(np.abs(out[k]))
    ctx.force_batched(pos, mass, rung, thr, box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    assert ctx.stats()["interactions"] == total


def test_batched_uneven_thresholds(env):
    """Arbitrary (non-nested, repeated) thresholds and a subset that is empty."""
    torch, p3, ctx = env
    wl = make_workload("clustered256", n_side=32)
    thr = [3, 0, 7, 7, 9]
    out = ctx.force_batched(to_dev(torch, wl.pos), None, to_dev(torch, wl.rung), thr, box=1.0,
                            x_s=wl.x_s, r_cut=wl.r_cut, precision="fp64").cpu().numpy()
    for k, t in enumerate(thr):
        act = (wl.rung >= t).astype(np.uint8)
        ref, cnt, absum = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, active=act)
        if act.sum():
            e = oracle.errors(out[k][act == 1], ref[act == 1], absum[act == 1])
            assert e["e_max_cond"] <= 1e-12
        assert np.all(out[k][act == 0] == 0)


@pytest.fixture(scope="module")
def clustered256():
    print("generating clustered256 (N=256^3, k-NN rungs)", flush=True)
    return make_workload("clustered256")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_clustered256_full(env, clustered256, prec):
    """Full-size N=256^3 clustered set, 8 nested rung subsets in one launch:
    2048 receivers per rung (stratified, seeded; 16384 in all) checked in
    every subset they belong to against the oracle's cell-list sum over all
    N suppliers (pinned against its brute force)."""
    torch, p3, ctx = env
    wl = clustered256
    thr = list(range(8))
    out = ctx.force_batched(to_dev(torch, wl.pos), to_dev(torch, wl.mass), to_dev(torch, wl.rung),
                            thr, box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    torch.cuda.synchronize()
    st = ctx.stats()
    print(prec, st, flush=True)
    assert st["receivers"] == sum(int((wl.rung >= k).sum()) for k in thr)
    idx = stratified_by_rung(wl.rung, 2048, wl.config_id)
    ref, cnt, absum, _ = oracle.force(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled")
    for k in thr:
        sel = wl.rung[idx] >= k
        got = out[k][torch.from_numpy(idx[sel]).to(out.device)].cpu().numpy()
        e = oracle.errors(got, ref[sel], absum[sel])
        print("subset", k, int(sel.sum()), e, flush=True)
        assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], (k, e)
        # rows outside the subset are zero
        off = idx[~sel]
        if off.size:
            assert torch.count_nonzero(out[k][torch.from_numpy(off).to(out.device)]) == 0
    del out
    torch.cuda.empty_cache()
