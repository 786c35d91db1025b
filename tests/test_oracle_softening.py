"""Pins of the oracle's B-spline softening (section 2.1.1, eq. bspline_shape
and eq. bspline_force; the softening bracket of eq. p3m_gravity).

The force of a softened point mass at distance r is M(<r) / r^2, where M(<r)
is the mass of the softening shape S_B inside radius r.  So for r < eps_B
the bracket |r|_B^-3 - r^-3 equals (M(<r) - 1) / r^3.  The pin integrates the
shape S_B of eq. bspline_shape numerically (scipy quad) and compares with
the oracle's softened-minus-unsoftened pair force: a wrong coefficient,
sign, branch boundary or the x^-3/480 term in |r|_B^-3 fails it.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle


def bspline_shape(r, eps_b):
    """S_B(r) of eq. bspline_shape."""
    x = r / eps_b
    k = 8.0 / (math.pi * eps_b ** 3)
    if x < 0.5:
        return k * (1.0 - 6.0 * x * x * (1.0 - x))
    if x < 1.0:
        return k * 2.0 * (1.0 - x) ** 3
    return 0.0


def mass_shell(a, b, eps_b):
    """4 pi int_a^b s^2 S_B(s) ds."""
    f = lambda s: 4.0 * math.pi * s * s * bspline_shape(s, eps_b)
    pts = [p for p in (0.5 * eps_b,) if a < p < b]
    return quad(f, a, b, points=pts or None, epsabs=0, epsrel=1e-13, limit=200)[0]


def enclosed(r, eps_b):
    return mass_shell(0.0, min(r, eps_b), eps_b)


BOX, X_S, R_CUT, EPS = 1.0, 0.05, 0.2, 0.02   # eps_B = 0.056


def pair_force(r, eps, direction=(0.6, -0.48, 0.64)):
    d = np.asarray(direction) / np.linalg.norm(direction)
    pos = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    pos[1] = pos[0] - r * d            # r_01 = x_0 - x_1 = r d
    acc, cnt, absum, _ = oracle.force(pos, None, BOX, X_S, R_CUT, recv=[0], eps=eps)
    return acc[0], d, pos


def test_shape_is_normalised():
    eps_b = oracle.eps_b_of(EPS)
    assert abs(enclosed(eps_b, eps_b) - 1.0) < 1e-12


@pytest.mark.parametrize("xb", [0.05, 0.2, 0.4, 0.499, 0.501, 0.6, 0.8, 0.97])
def test_softening_bracket_equals_enclosed_mass(xb):
    eps_b = oracle.eps_b_of(EPS)
    r = xb * eps_b
    a_soft, d, pos = pair_force(r, EPS)
    a_plain, _, _ = pair_force(r, 0.0)
    # delta a_0 = -mu (|r|_B^-3 - r^-3) r_01, and |r|_B^-3 r^3 = M(<r), so
    # delta a_0 . d = (1 - M(<r)) / r^2 = (mass of the shape outside r) / r^2
    got = np.dot(a_soft - a_plain, d)
    want = mass_shell(r, eps_b, eps_b) / (r * r)
    # the difference of two forces of size |a| ~ 1/r^2 carries their rounding
    # (the |r|_B^-3 polynomial cancels to a few percent of its terms near
    # x_B = 1): allow 1e-14 |a| on top of 1e-10 relative
    tol = 1e-10 * abs(want) + 1e-14 * np.linalg.norm(a_plain)
    assert abs(got - want) <= tol, (xb, got, want)
    # the correction acts along the separation only
    perp = (a_soft - a_plain) - got * d
    assert np.linalg.norm(perp) <= tol


def test_no_softening_beyond_eps_b():
    eps_b = oracle.eps_b_of(EPS)
    for xb in (1.0, 1.2, 2.5):
        a_soft, _, _ = pair_force(xb * eps_b, EPS)
        a_plain, _, _ = pair_force(xb * eps_b, 0.0)
        assert np.array_equal(a_soft, a_plain)


def test_softened_force_is_finite_at_small_separation():
    # the softened pair force tends to 0 linearly: (|r|_B^-3 + (g-1)/r^3) r
    eps_b = oracle.eps_b_of(EPS)
    for r in (1e-9, 1e-7, 1e-5):
        a, d, _ = pair_force(r, EPS)
        lim = -(32.0 / (3.0 * eps_b ** 3) - 4.0 / (3.0 * math.sqrt(math.pi) * (2 * X_S) ** 3)) * r
        assert abs(np.dot(a, d) - lim) <= 1e-6 * abs(lim), (r, np.dot(a, d), lim)


def test_softened_momentum_conservation():
    rng = np.random.default_rng(7)
    pos = rng.random((400, 3)) * 0.3 + 0.35          # dense blob: many softened pairs
    acc, cnt, absum, _ = oracle.force(pos, None, BOX, X_S, R_CUT, eps=EPS)
    assert np.linalg.norm(acc.sum(axis=0)) <= 1e-12 * absum.sum()


@pytest.mark.parametrize("mode", ["fixed"])
def test_softened_vjp_matches_finite_differences(mode):
    rng = np.random.default_rng(8)
    n = 300
    pos = rng.random((n, 3)) * 0.25 + 0.375
    mass = rng.uniform(0.5, 2.0, n)
    active = (rng.random(n) < 0.7).astype(np.uint8)
    w = rng.standard_normal((n, 3))
    kidx = np.arange(0, n, 7)
    g = oracle.vjp(pos, mass, active, w, BOX, X_S, R_CUT, kidx=kidx, eps=EPS)
    fd, st = oracle.fd_grad(pos, mass, active, w, BOX, X_S, R_CUT, kidx, h=1e-6, mode=mode,
                            eps=EPS)
    scale = np.max(np.abs(g))
    assert np.max(np.abs(g - fd)) <= 1e-5 * scale, np.max(np.abs(g - fd)) / scale
    # and tiled equals brute force
    g2 = oracle.vjp(pos, mass, active, w, BOX, X_S, R_CUT, kidx=kidx, method="tiled", eps=EPS)
    assert np.max(np.abs(g2 - g)) <= 1e-13 * scale
