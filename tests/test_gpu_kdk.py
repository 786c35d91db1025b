"""Rung-hierarchical KDK step on the GPU (p3m_kdk_step, section 2.2.2)
against the KDK oracle driven by the oracle's short-range and PM forces,
through the C ABI: positions, velocities and the final rungs after a
synchronised period, with rung jumps inside it; fixed rungs; short range
only; the FP32 force path; time reversibility with fixed rungs."""
import numpy as np
import pytest

import oracle
from gpu_common import gpu_or_skip, to_dev
from oracle import kdk_oracle as kdk
from oracle import pm_oracle as pm

pytestmark = pytest.mark.gpu

N_GRID = 32
X_S = 1.25 / N_GRID
R_CUT = 4.5 * X_S


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def particles(n=2048, seed=11):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    pos[:600] = (0.5 + 0.02 * rng.standard_normal((600, 3))) % 1.0
    vel = 0.05 * rng.standard_normal((n, 3))
    mass = rng.uniform(0.5, 1.5, n) / n
    return pos, vel, mass


def eps_for(n):
    return 0.03 / round(n ** (1.0 / 3.0))


def oracle_run(pos, vel, mass, dt, n_steps, eps, n_grid=N_GRID, rung=None, fixed=False):
    def sr(p, m):
        return oracle.force_full(p, mass, 1.0, X_S, R_CUT, active=m, eps=eps)[0]

    lr = (lambda p: pm.pm_force(p, mass, 1.0, n_grid, X_S)) if n_grid else None
    return kdk.kdk(pos, vel, 1.0, dt, n_steps, sr, lr, eps=eps, rung=rung, fixed_rungs=fixed)


def gpu_run(env, pos, vel, mass, dt, n_steps, eps, n_grid=N_GRID, rung=None, fixed=False,
            precision="fp64"):
    torch, p3, ctx = env
    p = to_dev(torch, pos)
    v = to_dev(torch, vel)
    r = to_dev(torch, np.zeros(len(pos), np.uint8) if rung is None else rung.astype(np.uint8))
    ctx.kdk_step(p, v, to_dev(torch, mass), r, box=1.0, x_s=X_S, r_cut=R_CUT, n_grid=n_grid,
                 dt=dt, n_steps=n_steps, eps=eps, fixed_rungs=fixed, precision=precision)
    torch.cuda.synchronize()
    return p.cpu().numpy(), v.cpu().numpy(), r.cpu().numpy(), ctx.kdk_stats()


def periodic_diff(a, b):
    d = a - b
    return d - np.round(d)


@pytest.mark.parametrize("n_steps", [1, 2])
def test_kdk_matches_oracle(env, n_steps):
    print("kdk n_steps", n_steps, flush=True)
    pos, vel, mass = particles()
    eps = eps_for(len(pos))
    dt = 3e-3
    xo, vo, ro = oracle_run(pos, vel, mass, dt, n_steps, eps)
    xg, vg, rg, st = gpu_run(env, pos, vel, mass, dt, n_steps, eps)
    print(st, np.bincount(ro, minlength=8), flush=True)
    assert st["highest_rung"] >= 2 and st["substeps"] == n_steps * 2 ** st["highest_rung"]
    assert st["lr_calls"] == n_steps + 1
    dv = np.max(np.abs(vo - vel))
    assert np.max(np.abs(periodic_diff(xg, xo))) <= 1e-11
    assert np.max(np.abs(vg - vo)) <= 1e-9 * dv
    assert np.array_equal(rg, ro)


def test_kdk_rung_jumps_match_oracle(env):
    """A longer step on the same set: the clump collapses, rungs move inside
    the period and the highest final rung is above the starting one."""
    pos, vel, mass = particles(seed=12)
    eps = eps_for(len(pos))
    dt = 1e-2
    xo, vo, ro = oracle_run(pos, vel, mass, dt, 1, eps)
    xg, vg, rg, st = gpu_run(env, pos, vel, mass, dt, 1, eps)
    print(st, np.bincount(ro, minlength=8), flush=True)
    assert ro.max() > st["highest_rung"]
    dv = np.max(np.abs(vo - vel))
    assert np.max(np.abs(periodic_diff(xg, xo))) <= 1e-10
    assert np.max(np.abs(vg - vo)) <= 1e-8 * dv
    assert np.array_equal(rg, ro)


def test_kdk_short_range_only_fixed_rungs(env):
    pos, vel, mass = particles(n=1500, seed=13)
    eps = eps_for(len(pos))
    rung = np.random.default_rng(3).integers(0, 4, len(pos))
    xo, vo, ro = oracle_run(pos, vel, mass, 2e-3, 2, eps, n_grid=0, rung=rung, fixed=True)
    xg, vg, rg, st = gpu_run(env, pos, vel, mass, 2e-3, 2, eps, n_grid=0, rung=rung, fixed=True)
    assert st["lr_calls"] == 0 and st["highest_rung"] == 3
    assert np.array_equal(rg, rung)
    dv = np.max(np.abs(vo - vel))
    assert np.max(np.abs(periodic_diff(xg, xo))) <= 1e-11
    assert np.max(np.abs(vg - vo)) <= 1e-9 * dv


def test_kdk_fp32_forces(env):
    pos, vel, mass = particles(seed=14)
    eps = eps_for(len(pos))
    rung = np.random.default_rng(4).integers(0, 3, len(pos))
    xo, vo, _ = oracle_run(pos, vel, mass, 2e-3, 1, eps, rung=rung, fixed=True)
    xg, vg, _, _ = gpu_run(env, pos, vel, mass, 2e-3, 1, eps, rung=rung, fixed=True,
                           precision="fp32")
    dv = np.max(np.abs(vo - vel))
    assert np.max(np.abs(vg - vo)) <= 1e-5 * dv


def test_kdk_fixed_rungs_reversible(env):
    pos, vel, mass = particles(n=1000, seed=15)
    eps = eps_for(len(pos))
    rung = np.random.default_rng(5).integers(0, 3, len(pos))
    x1, v1, _, _ = gpu_run(env, pos, vel, mass, 2e-3, 2, eps, rung=rung, fixed=True)
    x2, v2, _, _ = gpu_run(env, x1, -v1, mass, 2e-3, 2, eps, rung=rung, fixed=True)
    assert np.max(np.abs(periodic_diff(x2, pos))) <= 1e-11
    assert np.max(np.abs(-v2 - vel)) <= 1e-9 * np.max(np.abs(v1 - vel))


def test_kdk_empty(env):
    torch, p3, ctx = env
    z = torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")
    r = torch.zeros(0, dtype=torch.uint8, device="cuda:0")
    ctx.kdk_step(z, z.clone(), None, r, box=1.0, x_s=X_S, r_cut=R_CUT, n_grid=N_GRID, dt=1e-3,
                 eps=1e-3)
    st = ctx.kdk_stats()
    assert st["n"] == 0 and st["interactions"] == 0


@pytest.mark.parametrize("n_grid", [0, N_GRID])
def test_kdk_free_particle_drifts(env, n_grid):
    """One particle feels no force (no pair; the PM self-force of CIC with an
    antisymmetric difference vanishes), so it coasts: x = x0 + v T, wrapped."""
    pos = np.array([[0.97, 0.5, 0.02]])
    vel = np.array([[0.5, -0.25, -0.75]])
    xg, vg, rg, st = gpu_run(env, pos, vel, np.ones(1), 0.01, 3, 1e-3, n_grid=n_grid)
    assert st["highest_rung"] == 0 and st["substeps"] == 3
    want = (pos + 3 * 0.01 * vel) % 1.0
    assert np.max(np.abs(periodic_diff(xg, want))) <= 1e-12
    assert np.max(np.abs(vg - vel)) <= 1e-9
