"""Pins of the rung-hierarchical KDK oracle (section 2.2.2, the
time-stepping figure and eq. rung), with force fields whose exact answers
are known:
- eq. rung is the smallest rung whose time step keeps the distance
  accelerated from rest, a (dt / 2^l)^2 / 2, within eta eps;
- leapfrog is exact for constant accelerations, whatever the rung of each
  particle: a wrong kick size, a missing half kick or a mis-timed
  long-range kick breaks x = x0 + v0 T + a T^2 / 2;
- with rung jumps every particle's kicks still add up to the whole period;
- with fixed rungs the scheme is time-reversible and second-order;
- with the P3M forces and one common rung, momentum is conserved.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import kdk_oracle as kdk
from oracle import pm_oracle as pm


def test_rung_is_smallest_safe_rung():
    rng = np.random.default_rng(1)
    dt, eta, eps = 0.01, 0.025, 1e-3
    mags = 10.0 ** rng.uniform(-2, 6, 400)
    dirs = rng.standard_normal((400, 3))
    acc = dirs / np.linalg.norm(dirs, axis=1)[:, None] * mags[:, None]
    r = kdk.rung_of(acc, dt, eta, eps, max_rung=30)
    for l, a in zip(r, mags):
        assert 0.5 * a * (dt / 2.0 ** l) ** 2 <= eta * eps * (1 + 1e-12)
        if l > 0:
            assert 0.5 * a * (dt / 2.0 ** (l - 1)) ** 2 > eta * eps
    assert np.all(kdk.rung_of(acc, dt, eta, eps, max_rung=3) == np.minimum(r, 3))
    assert kdk.rung_of(np.zeros((1, 3)), dt, eta, eps, 7)[0] == 0


@pytest.mark.parametrize("n_steps", [1, 3])
@pytest.mark.parametrize("with_lr", [False, True])
def test_constant_fields_are_integrated_exactly(n_steps, with_lr):
    rng = np.random.default_rng(2)
    n = 64
    box = 1e6                                         # no wrap
    x0 = rng.uniform(1e3, 2e3, (n, 3))
    v0 = rng.standard_normal((n, 3))
    g = rng.standard_normal((n, 3))
    h = rng.standard_normal((n, 3)) if with_lr else np.zeros((n, 3))
    rung = rng.integers(0, 4, n)
    dt = 0.125
    x, v, r = kdk.kdk(x0, v0, box, dt, n_steps, lambda p, m: g.copy(),
                      (lambda p: h.copy()) if with_lr else None,
                      rung=rung, fixed_rungs=True)
    T = n_steps * dt
    assert np.allclose(x, x0 + v0 * T + 0.5 * (g + h) * T * T, rtol=0, atol=1e-11)
    assert np.allclose(v, v0 + (g + h) * T, rtol=0, atol=1e-13)
    assert np.array_equal(r, rung)


def test_rung_jumps_keep_the_kicks_whole():
    """A field that grows with distance from the centre (a = -k r^2 r_hat)
    on particles moving outwards and inwards makes them change rung inside
    the period; every particle's kicks must still cover the whole period."""
    rng = np.random.default_rng(3)
    n = 200
    box = 1e3
    c = np.full(3, 500.0)
    x0 = c + rng.standard_normal((n, 3)) * rng.uniform(0.5, 3.0, (n, 1))
    v0 = rng.standard_normal((n, 3)) * 4.0

    def field(p, mask):
        d = p - c
        r = np.linalg.norm(d, axis=1)[:, None]
        return -30.0 * r * d

    log = []
    dt, n_steps = 0.05, 4
    x, v, r = kdk.kdk(x0, v0, box, dt, n_steps, field, None, eta=0.025, eps=0.05,
                      max_rung=6, log=log)
    per = np.zeros(n)
    times = {}
    for i, t, dk in log:
        per[i] += dk
        times.setdefault(i, []).append(t)
    assert np.allclose(per, n_steps * dt, rtol=0, atol=1e-14)
    for ts in times.values():
        assert all(b > a for a, b in zip(ts, ts[1:]))
    # the rungs changed inside the period for some particles: their kick
    # intervals are not all equal
    changed = sum(len(set(np.diff(ts))) > 1 for ts in times.values())
    assert changed > 10, changed


def harmonic(omega2, c):
    return lambda p, m: -omega2[:, None] * (p - c)


def test_fixed_rungs_are_time_reversible():
    rng = np.random.default_rng(4)
    n = 50
    c = np.full(3, 50.0)
    x0 = c + rng.standard_normal((n, 3))
    v0 = rng.standard_normal((n, 3))
    om2 = rng.uniform(0.5, 40.0, n)
    rung = np.clip(np.floor(np.log2(np.sqrt(om2))).astype(int), 0, 3)
    f = harmonic(om2, c)
    x1, v1, _ = kdk.kdk(x0, v0, 100.0, 0.1, 3, f, None, rung=rung, fixed_rungs=True)
    x2, v2, _ = kdk.kdk(x1, -v1, 100.0, 0.1, 3, f, None, rung=rung, fixed_rungs=True)
    assert np.max(np.abs(x2 - x0)) <= 1e-12
    assert np.max(np.abs(-v2 - v0)) <= 1e-12


def test_fixed_rungs_second_order():
    rng = np.random.default_rng(5)
    n = 20
    c = np.full(3, 50.0)
    x0 = c + rng.standard_normal((n, 3))
    v0 = rng.standard_normal((n, 3))
    om2 = rng.uniform(1.0, 16.0, n)
    om = np.sqrt(om2)[:, None]
    rung = rng.integers(0, 3, n)
    T = 1.0

    def err(n_steps):
        x, v, _ = kdk.kdk(x0, v0, 100.0, T / n_steps, n_steps, harmonic(om2, c), None,
                          rung=rung, fixed_rungs=True)
        exact = c + (x0 - c) * np.cos(om * T) + v0 / om * np.sin(om * T)
        return np.max(np.abs(x - exact))

    e1, e2, e3 = err(8), err(16), err(32)
    assert 3.5 < e1 / e2 < 4.5 and 3.5 < e2 / e3 < 4.5, (e1, e2, e3)


def test_p3m_forces_one_rung_conserve_momentum():
    rng = np.random.default_rng(6)
    n = 1000
    n_grid = 32
    x_s = 1.25 / n_grid
    r_cut = 4.5 * x_s
    eps = 0.03 / 10
    pos = rng.random((n, 3))
    pos[:200] = (0.5 + 0.03 * rng.standard_normal((200, 3))) % 1.0
    vel = 0.01 * rng.standard_normal((n, 3))
    mass = rng.uniform(0.5, 2.0, n)

    def sr(p, mask):
        a, _, _ = oracle.force_full(p, mass, 1.0, x_s, r_cut, active=mask, eps=eps)
        return a

    def lr(p):
        return pm.pm_force(p, mass, 1.0, n_grid, x_s)

    x, v, r = kdk.kdk(pos, vel, 1.0, 2e-3, 2, sr, lr, rung=np.ones(n, dtype=int),
                      fixed_rungs=True)
    p0 = (mass[:, None] * vel).sum(axis=0)
    p1 = (mass[:, None] * v).sum(axis=0)
    scale = np.abs(mass[:, None] * (v - vel)).sum()
    assert np.max(np.abs(p1 - p0)) <= 1e-12 * scale
    assert np.max(np.abs(v - vel)) > 0
