"""Pins of the oracle's vector-Jacobian product (adjoint of the short-range
force of eq. p3m_gravity with respect to positions).

Facts used, none taken from the oracle itself:
  * the pair Jacobian is minus the Hessian of the split potential
    erfc(r/2x_s)/r, differentiated numerically with mpmath;
  * its trace is minus the Laplacian of that potential, i.e. -4 pi times
    the density of a normalised Gaussian of standard deviation sqrt(2) x_s
    (erf(r/2x_s)/r is that Gaussian's potential), also checked by mpmath;
  * its Newtonian limit is the point-mass tidal tensor (I - 3 r r^T/r^2)/r^3;
  * central finite differences of the oracle's own force sum;
  * translation invariance: sum_k dL/dx_k = 0 when every particle is active.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from workloads import lattice_sites, make_workload, random_particles

mp.mp.dps = 40


@pytest.fixture(autouse=True, scope="module")
def _built(oracle_lib):
    return oracle_lib


def pair_jacobian(rv, x_s, r_cut):
    """Columns of J from one-hot weights on a two-particle system:
    with w_0 = e_b, w_1 = 0, mu = 1: dL/dx_0 = -J(r_01) e_b."""
    x0 = np.array([0.5, 0.5, 0.5])
    pos = np.stack([x0, x0 - np.asarray(rv)])
    rv = pos[0] - pos[1]
    J = np.zeros((3, 3))
    for b in range(3):
        w = np.zeros((2, 3))
        w[0, b] = 1.0
        g = oracle.vjp(pos, None, None, w, 1.0, x_s, r_cut, kidx=[0])
        J[:, b] = -g[0]
    return J, rv


def mp_hessian(rv, x_s):
    xs = mp.mpf(x_s)

    def psi(x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        return mp.erfc(r / (2 * xs)) / r

    pt = [mp.mpf(float(v)) for v in rv]
    H = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            order = [0, 0, 0]
            order[a] += 1
            order[b] += 1
            H[a, b] = float(mp.diff(psi, pt, tuple(order)))
    return H


@pytest.mark.parametrize("r_over_xs", [0.3, 1.0, 2.5, 4.4])
def test_jacobian_is_minus_potential_hessian(r_over_xs):
    x_s = 0.01
    d = np.array([0.36, 0.48, -0.8])
    J, rv = pair_jacobian(d / np.linalg.norm(d) * r_over_xs * x_s, x_s, 4.5 * x_s)
    H = mp_hessian(rv, x_s)
    assert np.max(np.abs(J + H)) <= 1e-12 * np.max(np.abs(H))
    assert np.max(np.abs(J - J.T)) <= 1e-14 * np.max(np.abs(J))


@pytest.mark.parametrize("r_over_xs", [0.5, 1.7, 3.9])
def test_jacobian_trace_is_gaussian_density(r_over_xs):
    x_s = 0.02
    J, rv = pair_jacobian([r_over_xs * x_s, 0.0, 0.0], x_s, 4.5 * x_s)
    r = float(np.linalg.norm(rv))
    sigma = math.sqrt(2.0) * x_s
    gauss = (2 * math.pi * sigma ** 2) ** -1.5 * math.exp(-r * r / (2 * sigma ** 2))
    assert abs(np.trace(J) + 4 * math.pi * gauss) <= 1e-12 * 4 * math.pi * gauss
    # the same Laplacian from mpmath: psi'' + 2 psi'/r for a radial function
    f = lambda t: mp.erfc(t / (2 * mp.mpf(x_s))) / t
    lap = float(mp.diff(f, mp.mpf(r), 2) + 2 * mp.diff(f, mp.mpf(r), 1) / r)
    assert abs(np.trace(J) + lap) <= 1e-12 * abs(lap)


def test_jacobian_newtonian_limit():
    x_s = 0.02
    J, rv = pair_jacobian([1e-6, 2e-6, -1.5e-6], x_s, 4.5 * x_s)
    r = np.linalg.norm(rv)
    n = rv / r
    tidal = (np.eye(3) - 3 * np.outer(n, n)) / r ** 3
    assert np.max(np.abs(J - tidal)) <= 1e-9 * np.max(np.abs(tidal))


def test_vjp_matches_finite_differences():
    pos, mass, active = random_particles(400, seed=31, active_frac=0.5)
    x_s = 0.04
    r_cut = 4.5 * x_s
    w = np.random.default_rng(4).standard_normal((400, 3))
    k = np.arange(0, 400, 7)
    g = oracle.vjp(pos, mass, active, w, 1.0, x_s, r_cut, kidx=k)
    fd, _ = oracle.fd_grad(pos, mass, active, w, 1.0, x_s, r_cut, k, h=1e-6, mode="fixed")
    nz = np.linalg.norm(fd, axis=1) > 0
    assert nz.sum() > 40
    assert np.all(g[~nz] == 0)          # no active particle within reach
    rel = np.linalg.norm(g[nz] - fd[nz], axis=1) / np.linalg.norm(fd[nz], axis=1)
    assert np.max(rel) <= 1e-6


def test_fd_plain_flags_cutoff_straddles():
    """Re-evaluating the pair set flags exactly the samples whose pairs cross
    r_cut within the step; the other samples agree with the frozen set."""
    pos, mass, _ = random_particles(300, seed=8)
    x_s = 0.04
    r_cut = 4.5 * x_s
    w = np.random.default_rng(5).standard_normal((300, 3))
    k = np.arange(300)
    h = 2e-3                                  # large step: some straddles
    fix, _ = oracle.fd_grad(pos, mass, None, w, 1.0, x_s, r_cut, k, h=h, mode="fixed")
    pla, st = oracle.fd_grad(pos, mass, None, w, 1.0, x_s, r_cut, k, h=h, mode="plain")
    assert st.any() and not st.all()
    ok = st == 0
    assert np.array_equal(fix[ok], pla[ok])


def test_vjp_translation_invariance_and_tiled():
    wl = make_workload("diff64", n_side=16)
    w = np.random.default_rng(6).standard_normal((wl.n, 3))
    g = oracle.vjp(wl.pos, wl.mass, None, w, 1.0, wl.x_s, wl.r_cut)
    gt = oracle.vjp(wl.pos, wl.mass, None, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    scale = np.abs(g).sum(axis=0)
    assert np.all(np.abs(g.sum(axis=0)) <= 1e-13 * scale)
    assert np.max(np.abs(g - gt)) <= 1e-14 * np.max(np.abs(g))


def test_vjp_inactive_particles_only_supply():
    """With no active particle the loss is identically zero."""
    pos, mass, _ = random_particles(200, seed=2)
    w = np.ones((200, 3))
    g = oracle.vjp(pos, mass, np.zeros(200, np.uint8), w, 1.0, 0.04, 0.18)
    assert np.all(g == 0)


def test_fd_fixed_on_lattice_sites_with_pairs_on_cutoff():
    """Sites of a 64^3 lattice with r_cut = 4 spacings: hundreds of pairs lie
    exactly on r_cut (excluded: the sum is strict), duplicated sites are
    coincident particles (no contribution).  The frozen pair set of the
    finite differences and the analytic VJP must make the same decisions, so
    they agree to the differences' truncation error on every sample."""
    n_side, k = 64, 4
    pos, ijk = lattice_sites(n_side, 3000, 200, 40, seed=9)
    r_cut = k / n_side
    x_s = r_cut / 4.5
    d = ijk[:, None, :] - ijk[None, :, :]
    d = (d + n_side // 2) % n_side - n_side // 2
    on_cut = ((d * d).sum(axis=2) == k * k).any(axis=1)
    assert on_cut.sum() > 100
    w = np.random.default_rng(10).standard_normal((pos.shape[0], 3))
    kidx = np.flatnonzero(on_cut)[:60]
    g = oracle.vjp(pos, None, None, w, 1.0, x_s, r_cut, kidx=kidx)
    fd, _ = oracle.fd_grad(pos, None, None, w, 1.0, x_s, r_cut, kidx, h=1e-7, mode="fixed")
    nz = np.linalg.norm(fd, axis=1) > 0
    assert np.all(g[~nz] == 0)
    rel = np.linalg.norm(g[nz] - fd[nz], axis=1) / np.linalg.norm(fd[nz], axis=1)
    assert np.max(rel) <= 1e-6


def _pair_split_by_rounding(r_cut, seed):
    """Two particles whose separation d has fma(dz, dz, fma(dy, dy, dx dx))
    below r_cut^2 while the unfused ((dx dx + dy dy) + dz dz) is not (or the
    reverse): the pair's membership depends on the rounding of r^2."""
    rng = np.random.default_rng(seed)
    rc2 = r_cut * r_cut
    for _ in range(200000):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        x0 = rng.uniform(0.3, 0.7, 3)
        x1 = x0 - u * r_cut
        dd = x0 - x1
        fused = oracle.sq_dist(dd[None, :])[0]
        plain = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
        if (fused < rc2) != (plain < rc2):
            return np.stack([x0, x1]), fused < rc2
    raise AssertionError("no pair found")


def test_fd_fixed_pair_set_uses_the_cutoff_rounding():
    """The frozen pair set of the finite differences is decided with the same
    r^2 rounding as the force and the VJP (the fused form), so a pair whose
    membership depends on that rounding is in both sets or in neither."""
    x_s = 0.01
    r_cut = 4.5 * x_s
    pos, inside = _pair_split_by_rounding(r_cut, seed=3)
    w = np.array([[0.3, -1.0, 0.7], [0.5, 0.2, -0.4]])
    g = oracle.vjp(pos, None, None, w, 1.0, x_s, r_cut, kidx=[0, 1])
    fd, _ = oracle.fd_grad(pos, None, None, w, 1.0, x_s, r_cut, [0, 1], h=1e-7, mode="fixed")
    if inside:
        assert np.all(np.linalg.norm(g, axis=1) > 0)
        rel = np.linalg.norm(g - fd, axis=1) / np.linalg.norm(g, axis=1)
        assert np.max(rel) <= 1e-6
    else:
        assert np.all(g == 0) and np.all(fd == 0)
