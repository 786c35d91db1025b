"""B-spline softened short-range force on the GPU (section 2.1.1,
eq. bspline_force; the softening bracket of eq. p3m_gravity) against the
FP64 oracle, through the C ABI.  The softening length is eps = 0.03 L/cbrt(N)
(a small fraction of the mean inter-particle distance), eps_B = 2.8 eps; the
clustered sets put many pairs inside eps_B in their halo cores."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload, random_particles, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def eps_for(n):
    return 0.03 / round(n ** (1.0 / 3.0))


def soft_force(env, pos, mass, active, box, x_s, r_cut, prec, eps, **cfg):
    torch, p3, ctx = env
    ctx.set_softening(eps)
    if cfg:
        ctx.set_config(**cfg)
    try:
        acc = ctx.force(to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active), box=box,
                        x_s=x_s, r_cut=r_cut, precision=prec)
        torch.cuda.synchronize()
        return acc.cpu().numpy(), ctx.stats()
    finally:
        ctx.set_softening(0.0)
        ctx.set_config()


@pytest.mark.parametrize("csize,screen", [(64, 0), (32, 1), (8, 1), (16, 0), (16, 2), (32, 2),
                                          (64, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_softened_clustered(env, prec, csize, screen):
    print("softened diff64 n_side=32", prec, csize, screen, flush=True)
    wl = make_workload("diff64", n_side=32)
    eps = eps_for(wl.n)
    ref, cnt, absum = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, eps=eps)
    plain, _, _ = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut)
    # the softening changes the force noticeably on this set
    assert np.max(np.linalg.norm(ref - plain, axis=1) / absum) > 1e-3
    acc, st = soft_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, prec, eps,
                         cluster_size=csize, screen=screen)
    assert abs(st["eps_b"] - 2.8 * eps) <= 1e-15
    # screen 2: each pair once for both partners, in either precision
    assert st["screen"] == screen
    e = oracle.errors(acc, ref, absum)
    print(e, flush=True)
    assert st["interactions"] == int(cnt.sum())
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e


@pytest.mark.parametrize("n", [2, 65, 1000, 4097])
def test_softened_mutual_ragged_masses(env, n):
    """Softened FP32 calls with every particle active take the kernel that
    evaluates each pair once for both partners (screen 2): ragged sets with
    per-particle masses, in the three cluster layouts; n = 2 puts the pair
    well inside eps_B (and close enough for the FP64 separation)."""
    pos, mass, _ = random_particles(n, seed=500 + n, active_frac=1.0)
    if n == 2:
        pos[0] = [0.5, 0.5, 0.5]
        pos[1] = [0.5 + 1e-4, 0.5, 0.5]
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    eps = 0.01
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute", eps=eps)
    for cs in (16, 32, 64):
        acc, st = soft_force(env, pos, mass, None, 1.0, x_s, r_cut, "fp32", eps,
                             cluster_size=cs, screen=2)
        assert st["screen"] == 2
        e = oracle.errors(acc, ref, absum)
        assert st["interactions"] == int(cnt.sum()), (cs, st["interactions"], int(cnt.sum()))
        assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], (cs, e)


@pytest.mark.parametrize("n", [2, 65, 1000, 4097])
def test_softened_ragged_masses_and_mask(env, n):
    pos, mass, active = random_particles(n, seed=300 + n, active_frac=0.6)
    if n == 2:
        pos[:] = [0.5, 0.5, 0.5]
        pos[1] = [0.5 + 1e-4, 0.5, 0.5]        # well inside eps_B
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    eps = 0.01
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active,
                                        method="brute", eps=eps)
    for prec in ("fp64", "fp32"):
        for cs, sc in ((64, 0), (8, 1)):
            acc, st = soft_force(env, pos, mass, active, 1.0, x_s, r_cut, prec, eps,
                                 cluster_size=cs, screen=sc)
            e = oracle.errors(acc, ref, absum)
            assert st["interactions"] == int(cnt.sum())
            assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], (prec, cs, e)
            assert np.all(acc[active == 0] == 0)


@pytest.mark.parametrize("prec, tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_softened_adjoint(env, prec, tol):
    torch, p3, ctx = env
    wl = make_workload("diff64", n_side=24)
    eps = eps_for(wl.n)
    rng = np.random.default_rng(21)
    mass = rng.uniform(0.5, 2.0, wl.n)
    active = (rng.random(wl.n) < 0.6).astype(np.uint8)
    w = rng.standard_normal((wl.n, 3))
    ref = oracle.vjp(wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, method="tiled", eps=eps)
    ctx.set_softening(eps)
    try:
        g = ctx.force_backward(to_dev(torch, wl.pos), to_dev(torch, mass), to_dev(torch, active),
                               to_dev(torch, w), box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                               precision=prec).cpu().numpy()
    finally:
        ctx.set_softening(0.0)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    row = np.max(np.linalg.norm(g - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    print(prec, "rel %.3e row %.3e" % (rel, row), flush=True)
    assert rel <= tol and row <= tol, (rel, row)
    if prec == "fp64":
        # finite differences of the softened loss, pair set fixed (64 samples)
        kidx = sample_indices(wl.n, 64, wl.config_id, salt=3)
        fd, _ = oracle.fd_grad(wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, kidx, h=1e-6,
                               mode="fixed", eps=eps)
        scale = np.max(np.abs(ref[kidx]))
        assert np.max(np.abs(g[kidx] - fd)) <= 1e-4 * scale


def test_softened_batched(env):
    torch, p3, ctx = env
    wl = make_workload("clustered256", n_side=40)
    eps = eps_for(wl.n)
    thr = [0, 2, 5]
    ctx.set_softening(eps)
    ctx.set_config(cluster_size=16, screen=1)
    try:
        out = ctx.force_batched(to_dev(torch, wl.pos), None, to_dev(torch, wl.rung), thr,
                                box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                                precision="fp32").cpu().numpy()
    finally:
        ctx.set_softening(0.0)
        ctx.set_config()
    for k, t in enumerate(thr):
        act = (wl.rung >= t).astype(np.uint8)
        ref, cnt, absum = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, active=act,
                                            eps=eps)
        e = oracle.errors(out[k][act == 1], ref[act == 1], absum[act == 1])
        assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], (t, e)


@pytest.mark.parametrize("prec, screen", [("fp64", 1), ("fp32", 1), ("fp32", 2), ("fp64", 2)])
def test_softened_clustered128_sampled(env, prec, screen):
    """Full N = 128^3 clustered set with softening; 512 seeded receivers
    checked one by one against the oracle over all N."""
    print("softened clustered128", prec, "screen", screen, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    eps = eps_for(wl.n)
    acc, st = soft_force(env, wl.pos, None, None, 1.0, wl.x_s, wl.r_cut, prec, eps,
                         subtiles_per_dim=1, item_target=4096, cluster_size=32, screen=screen)
    assert st["screen"] == screen
    idx = sample_indices(wl.n, 512, wl.config_id)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled", eps=eps)
    e = oracle.errors(acc[idx], ref, absum)
    print(e, st, flush=True)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
