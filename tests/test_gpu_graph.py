"""The force calls do not wait for the host: after a warm-up call has grown
the workspace, a call can be captured into a HIP graph (stream capture
refuses host synchronisation and allocation), and every replay, with new
positions written eagerly between replays, matches an eager call on the
same positions."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload, sample_indices

pytestmark = pytest.mark.gpu

# graph and eager calls agree to the rounding of their summation order (the
# atomic ranks of the sort can differ between calls, and with them the
# clusters and the FP32 partial sums of the FP32 path)
AGREE = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3


LAYOUTS = [("fp32", dict(cluster_size=32, screen=2)),    # pairs for both partners
           ("fp32", dict(cluster_size=32, screen=1)),
           ("fp64", dict(cluster_size=16, screen=1, item_target=512)),
           ("fp64", dict(cluster_size=32, screen=2))]


@pytest.mark.parametrize("prec, layout", LAYOUTS)
def test_captured_force_replays_match_eager(env, prec, layout):
    torch, p3 = env
    print("graph capture diff64 n_side=32", prec, layout, flush=True)
    wl = make_workload("diff64", n_side=32)
    rng = np.random.default_rng(3)
    pos_sets = [wl.pos] + [np.mod(wl.pos + rng.normal(0.0, 2e-3, wl.pos.shape), 1.0)
                           for _ in range(3)]
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    ctx = p3.Context(0)
    eager = p3.Context(0)
    try:
        ctx.set_config(**layout)
        eager.set_config(**layout)
        pos_buf = to_dev(torch, pos_sets[0])
        out_buf = torch.empty((wl.n, 3), dtype=torch.float64, device="cuda:0")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.force(pos_buf, None, None, out=out_buf, **kw)   # grows the workspace
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            ctx.force(pos_buf, None, None, out=out_buf, **kw)
        torch.cuda.synchronize()
        for k, p in enumerate(pos_sets):
            pos_buf.copy_(torch.from_numpy(p))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            got = out_buf.cpu().numpy()
            ref = eager.force(to_dev(torch, p), None, None, **kw).cpu().numpy()
            scale = np.max(np.abs(ref))
            assert np.max(np.abs(got - ref)) <= AGREE[prec] * scale, k
            st, st_e = ctx.stats(), eager.stats()
            assert st["interactions"] == st_e["interactions"]
            assert st["items"] == st_e["items"] and st["items"] > 0
        idx = sample_indices(wl.n, 200, 5)
        r, _, absum, _ = oracle.force(pos_sets[-1], None, 1.0, wl.x_s, wl.r_cut, recv=idx)
        e = oracle.errors(got[idx], r, absum)
        assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    finally:
        ctx.close()
        eager.close()


def test_captured_batched_replays_match_eager(env):
    torch, p3 = env
    print("graph capture batched clustered256 recipe n_side=32", flush=True)
    wl = make_workload("clustered256", n_side=32)
    thr = list(range(8))
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    ctx = p3.Context(0)
    eager = p3.Context(0)
    try:
        pos_buf, rung = to_dev(torch, wl.pos), to_dev(torch, wl.rung)
        out_buf = torch.empty((8, wl.n, 3), dtype=torch.float64, device="cuda:0")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.force_batched(pos_buf, None, rung, thr, out=out_buf, **kw)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            ctx.force_batched(pos_buf, None, rung, thr, out=out_buf, **kw)
        torch.cuda.synchronize()
        rng = np.random.default_rng(9)
        for k in range(3):
            p = np.mod(wl.pos + rng.normal(0.0, 1e-3, wl.pos.shape), 1.0)
            pos_buf.copy_(torch.from_numpy(p))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            got = out_buf.cpu().numpy()
            ref = eager.force_batched(to_dev(torch, p), None, rung, thr, **kw).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= AGREE["fp32"] * np.max(np.abs(ref)), k
    finally:
        ctx.close()
        eager.close()
