"""The whole P3M acceleration on the GPU (p3m_force: short range plus PM,
eq. p3m_gravity, section 2.1.3, the two halves overlapped on two streams)
through the C ABI: against the oracle's short range plus the PM oracle,
element by element; against the Ewald sum; against the two halves called
one after the other at the clustered 128^3 size; with inputs produced on the
caller's stream just before the call; and over calls that grow and shrink
the workspace."""
import numpy as np
import pytest

import oracle
from gpu_common import gpu_or_skip, to_dev
from oracle import pm_oracle as pm
from workloads import make_workload, random_particles

pytestmark = pytest.mark.gpu

# FP64: the short range sums in a different order than the oracle (1e-11 of
# the largest row), the PM deposit adds with atomics (1e-12)
TOL_FP64 = 2e-11
# the same call twice: only the order of atomic additions differs
TOL_SAME = 1e-12


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def scales(n_grid):
    x_s = 1.25 / n_grid
    return x_s, 4.5 * x_s


def total(env, pos, mass, active, n_grid, precision="fp64"):
    torch, p3, ctx = env
    x_s, r_cut = scales(n_grid)
    acc = ctx.force_total(to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active), box=1.0,
                          x_s=x_s, r_cut=r_cut, n_grid=n_grid, precision=precision)
    torch.cuda.synchronize()
    return acc.cpu().numpy()


def halves(env, pos, mass, active, n_grid, precision="fp64"):
    torch, p3, ctx = env
    x_s, r_cut = scales(n_grid)
    p, m, a = to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active)
    sr = ctx.force(p, m, a, box=1.0, x_s=x_s, r_cut=r_cut, precision=precision)
    lr = ctx.force_long_range(p, m, a, box=1.0, n_grid=n_grid, x_s=x_s)
    torch.cuda.synchronize()
    return sr.cpu().numpy() + lr.cpu().numpy()


@pytest.mark.parametrize("n, n_grid", [(2, 32), (3000, 32), (8000, 64), (20000, 128)])
def test_p3m_force_matches_oracles(env, n, n_grid):
    print("p3m force n=%d grid=%d" % (n, n_grid), flush=True)
    pos, mass, active = random_particles(n, seed=900 + n, active_frac=0.6)
    pos[: n // 4] = (0.4 + 0.02 * np.random.default_rng(n).standard_normal((n // 4, 3))) % 1.0
    x_s, r_cut = scales(n_grid)
    sr = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active)[0]
    lr = pm.pm_force(pos, mass, 1.0, n_grid, x_s, active=active)
    ref = sr + lr
    got = total(env, pos, mass, active, n_grid)
    assert np.all(got[active == 0] == 0.0)
    scale = np.max(np.abs(ref))
    if scale > 0.0:
        err = np.max(np.abs(got - ref)) / scale
        print("max err / max |a| = %.3e" % err, flush=True)
        assert err <= TOL_FP64


def test_p3m_force_matches_ewald(env):
    """The same bar as the oracle's own P3M check: rms 1 %, max 3 %."""
    n_grid = 32
    rng = np.random.default_rng(5)
    n = 4096
    pos = rng.random((n, 3))
    pos[:512] = (0.5 + 0.03 * rng.standard_normal((512, 3))) % 1.0
    mass = rng.uniform(0.5, 2.0, n)
    recv = np.concatenate([np.arange(0, 512, 32), np.arange(512, n, 256)])
    got = total(env, pos, mass, None, n_grid)
    ref = pm.ewald_force(pos, mass, 1.0, recv=recv)
    err = np.linalg.norm(got[recv] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print("P3M vs Ewald: rms %.3e max %.3e" % (np.sqrt(np.mean(err ** 2)), err.max()), flush=True)
    assert np.sqrt(np.mean(err ** 2)) <= 1e-2 and err.max() <= 3e-2


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_p3m_force_equals_halves_clustered128(env, precision):
    """N = 128^3 clustered, PM grid 256^3: the overlapped call against the
    short range and the long range called one after the other."""
    print("p3m clustered128", precision, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    got = total(env, wl.pos, None, None, wl.n_pm, precision)
    ref = halves(env, wl.pos, None, None, wl.n_pm, precision)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("max diff / max |a| = %.3e" % err, flush=True)
    assert err <= TOL_SAME


def test_p3m_force_waits_for_the_callers_stream(env):
    """Positions written on a side stream just before the call: both halves
    must see them (the long range's stream waits for the caller's)."""
    torch, p3, ctx = env
    pos, mass, _ = random_particles(50000, seed=31)
    n_grid = 64
    x_s, r_cut = scales(n_grid)
    want = halves(env, pos, mass, None, n_grid)
    base = to_dev(torch, (pos + 0.5) % 1.0)
    m = to_dev(torch, mass)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(2_000_000)                  # keep the side stream busy first
        p = torch.remainder(base - 0.5, 1.0)         # pos, produced on the side stream
        acc = ctx.force_total(p, m, None, box=1.0, x_s=x_s, r_cut=r_cut, n_grid=n_grid,
                              precision="fp64")
    side.synchronize()
    got = acc.cpu().numpy()
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert err <= TOL_FP64, err


def test_p3m_force_growing_and_shrinking(env):
    for n, n_grid in [(2000, 32), (60000, 64), (700, 32), (0, 32), (30000, 128)]:
        print("p3m sizes n=%d grid=%d" % (n, n_grid), flush=True)
        pos, mass, active = random_particles(n, seed=70 + n, active_frac=0.8)
        got = total(env, pos, mass, active, n_grid)
        assert got.shape == (n, 3)
        if n:
            ref = halves(env, pos, mass, active, n_grid)
            assert np.max(np.abs(got - ref)) <= TOL_SAME * np.max(np.abs(ref))


def test_p3m_force_stats_cover_both_halves(env):
    torch, p3, ctx = env
    pos, mass, _ = random_particles(20000, seed=41)
    ctx.set_timing(True)
    try:
        total(env, pos, mass, None, 64)
        sr, lr = ctx.stats(), ctx.lr_stats()
    finally:
        ctx.set_timing(False)
    assert sr["n"] == 20000 and sr["interactions"] > 0 and sr["ms_pairs"] >= 0
    assert lr["n"] == 20000 and lr["n_grid"] == 64 and lr["ms_total"] >= 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_p3m_force_softened(env, precision):
    """B-spline softening (eps_B = 2.8 eps) applies to the short-range half
    of the whole force; the long-range half is unsoftened."""
    torch, p3, ctx = env
    n, n_grid = 6000, 32
    pos, mass, active = random_particles(n, seed=4242, active_frac=0.7)
    pos[:1500] = (0.6 + 0.01 * np.random.default_rng(1).standard_normal((1500, 3))) % 1.0
    x_s, r_cut = scales(n_grid)
    eps = 0.03 / 18.0
    sr = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active, eps=eps)[0]
    lr = pm.pm_force(pos, mass, 1.0, n_grid, x_s, active=active)
    ctx.set_softening(eps)
    try:
        got = total(env, pos, mass, active, n_grid, precision)
    finally:
        ctx.set_softening(0.0)
    ref = sr + lr
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("softened p3m", precision, "max err / max |a| = %.3e" % err, flush=True)
    assert err <= (TOL_FP64 if precision == "fp64" else 1e-5)
