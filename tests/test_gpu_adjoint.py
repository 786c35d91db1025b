"""GPU adjoint (vector-Jacobian product of the short-range force with
respect to positions) vs the oracle's analytic VJP and central finite
differences, through the C ABI and through torch.autograd."""
import numpy as np
import pytest

import oracle
from gpu_common import gpu_or_skip, to_dev
from workloads import make_workload, random_particles, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def gpu_vjp(env, pos, mass, active, w, box, x_s, r_cut, prec):
    torch, p3, ctx = env
    g = ctx.force_backward(to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active),
                           to_dev(torch, w), box=box, x_s=x_s, r_cut=r_cut, precision=prec)
    torch.cuda.synchronize()
    return g.cpu().numpy()


@pytest.mark.parametrize("prec, tol, screen", [("fp64", 1e-12, 1), ("fp32", 1e-5, 1),
                                               ("fp32", 1e-5, 2), ("fp64", 1e-12, 2)])
@pytest.mark.parametrize("frac", [None, 0.3])
def test_vjp_matches_oracle(env, prec, tol, screen, frac):
    """Config with N = 64^3 clustered particles (PM grid 128^3), every row of
    the adjoint against the oracle's analytic VJP, with per-particle masses
    and, once, 30 % of the particles active; in FP32 also with each pair
    evaluated once for both partners (screen 2)."""
    torch, p3, ctx = env
    print("vjp diff64 full", prec, "screen", screen, frac, flush=True)
    wl = make_workload("diff64")
    rng = np.random.default_rng(11)
    mass = rng.uniform(0.5, 2.0, wl.n)
    active = None if frac is None else (rng.random(wl.n) < frac).astype(np.uint8)
    w = rng.standard_normal((wl.n, 3))
    ref = oracle.vjp(wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    ctx.set_config(subtiles_per_dim=1, item_target=4096, cluster_size=32, screen=screen)
    try:
        g = gpu_vjp(env, wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, prec)
        assert ctx.stats()["screen"] == screen
    finally:
        ctx.set_config()
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    row = np.max(np.linalg.norm(g - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    print("rel L2 %.3e  max row %.3e" % (rel, row), flush=True)
    assert rel <= tol and row <= tol
    if active is not None:
        # particles with no active particle within r_cut get exactly zero
        zero = np.linalg.norm(ref, axis=1) == 0
        assert np.all(g[zero] == 0)
    else:
        # translation invariance with every particle active: sum_k grad_k = 0
        # up to the rounding of the path's arithmetic
        bound = {"fp64": 1e-12, "fp32": 1e-6}[prec]
        assert np.all(np.abs(g.sum(axis=0)) <= bound * np.abs(g).sum(axis=0))


@pytest.mark.parametrize("csize,screen", [(8, 1), (16, 1), (32, 1), (64, 1), (16, 0), (32, 0),
                                          (16, 2), (32, 2), (64, 2)])
@pytest.mark.parametrize("prec, tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_vjp_small_clusters(env, prec, tol, csize, screen):
    """The adjoint on small clusters (several copies of a cluster per wave),
    with and without the per-supplier screen (the listed suppliers carry
    their weights), and, in FP32, with each pair evaluated once for both
    partners (screen 2, in FP32 and in FP64), matches the oracle's VJP like
    the default layout does."""
    torch, p3, ctx = env
    print("vjp clustered n_side=24 csize", csize, "screen", screen, prec, flush=True)
    wl = make_workload("diff64", n_side=24)
    rng = np.random.default_rng(12)
    mass = rng.uniform(0.5, 2.0, wl.n)
    active = (rng.random(wl.n) < 0.5).astype(np.uint8)
    w = rng.standard_normal((wl.n, 3))
    ref = oracle.vjp(wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    ctx.set_config(cluster_size=csize, screen=screen)
    try:
        g = gpu_vjp(env, wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, prec)
        st = ctx.stats()
    finally:
        ctx.set_config()
    assert st["cluster_size"] == csize
    assert st["screen"] == screen
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    row = np.max(np.linalg.norm(g - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    assert rel <= tol and row <= tol, (rel, row)


@pytest.mark.parametrize("prec, screen", [("fp64", 1), ("fp32", 1), ("fp32", 2), ("fp64", 2)])
def test_vjp_finite_differences_diff64(env, prec, screen):
    """Config with N = 64^3 clustered particles, Gaussian weights: adjoint vs
    central differences (step 1e-6 L, pair set frozen) on 64 samples."""
    torch, p3, ctx = env
    print("diff64 FD", prec, "screen", screen, flush=True)
    wl = make_workload("diff64")
    ctx.set_config(subtiles_per_dim=1, item_target=4096, cluster_size=32, screen=screen)
    try:
        g = gpu_vjp(env, wl.pos, wl.mass, None, wl.weights, 1.0, wl.x_s, wl.r_cut, prec)
    finally:
        ctx.set_config()
    idx = sample_indices(wl.n, 64, wl.config_id)
    fd, _ = oracle.fd_grad(wl.pos, wl.mass, None, wl.weights, 1.0, wl.x_s, wl.r_cut, idx,
                           h=1e-6, mode="fixed")
    rel = np.linalg.norm(g[idx] - fd, axis=1) / np.linalg.norm(fd, axis=1)
    print("max rel %.3e median %.3e" % (rel.max(), np.median(rel)), flush=True)
    assert rel.max() <= 1e-4
    # translation invariance with every particle active: sum_k grad_k = 0 (to
    # the rounding of the sums: FP64 pair terms, FP32 ones)
    bound = {"fp64": 1e-12, "fp32": 1e-6}[prec]
    assert np.all(np.abs(g.sum(axis=0)) <= bound * np.abs(g).sum(axis=0))


def test_autograd_function(env):
    torch, p3, ctx = env
    pos_np, mass_np, active_np = random_particles(3000, seed=21, active_frac=0.5)
    x_s = 1.25 / 28
    r_cut = 4.5 * x_s
    pos = to_dev(torch, pos_np).requires_grad_(True)
    mass = to_dev(torch, mass_np)
    active = to_dev(torch, active_np)
    w = torch.randn((3000, 3), dtype=torch.float64, device="cuda:0")
    acc = p3.sr_force(pos, mass, active, box=1.0, x_s=x_s, r_cut=r_cut, precision="fp64",
                      context=ctx)
    (acc * w).sum().backward()
    ref = oracle.vjp(pos_np, mass_np, active_np, w.cpu().numpy(), 1.0, x_s, r_cut)
    got = pos.grad.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
