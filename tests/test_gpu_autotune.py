"""The measure-and-keep autotuner (section 2.1.3, "Subtiles": try a finer
subdivision, time it, keep it if faster) through the C ABI: after tuning the
forward, and then the adjoint on its own, both calls run in the stored
layouts and still match the oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload

pytestmark = pytest.mark.gpu

LAYOUT = ("subtiles_per_dim", "item_target", "cluster_size", "screen")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotuned_forward_and_adjoint(prec):
    print("autotune diff64 n_side=32", prec, flush=True)
    torch, p3 = gpu_or_skip()
    ctx = p3.Context(0)
    wl = make_workload("diff64", n_side=32)
    rng = np.random.default_rng(21)
    mass = rng.uniform(0.5, 2.0, wl.n)
    w = rng.standard_normal((wl.n, 3))
    pos, m = to_dev(torch, wl.pos), to_dev(torch, mass)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)

    ctx.autotune(pos, m, None, level=2, **kw)
    acc = ctx.force(pos, m, None, **kw)
    fwd = {k: ctx.stats()[k] for k in LAYOUT}
    ref, cnt, absum = oracle.force_full(wl.pos, mass, 1.0, wl.x_s, wl.r_cut)
    e = oracle.errors(acc.cpu().numpy(), ref, absum)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    assert ctx.stats()["interactions"] == int(cnt.sum())

    # the adjoint takes the forward's layout until it is tuned on its own
    ctx.force_backward(pos, m, None, to_dev(torch, w), **kw)
    assert {k: ctx.stats()[k] for k in LAYOUT} == fwd
    ctx.autotune(pos, m, None, level=1, adjoint=True, **kw)
    g = ctx.force_backward(pos, m, None, to_dev(torch, w), **kw).cpu().numpy()
    adj = {k: ctx.stats()[k] for k in LAYOUT}
    g_ref = oracle.vjp(wl.pos, mass, None, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print("forward layout", fwd, "adjoint layout", adj, "vjp rel", rel, flush=True)
    assert rel <= (1e-12 if prec == "fp64" else 1e-5)
    # tuning the adjoint leaves the forward's layout alone
    ctx.force(pos, m, None, **kw)
    assert {k: ctx.stats()[k] for k in LAYOUT} == fwd
    ctx.close()
