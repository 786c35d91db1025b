"""Pins of the long-range (PM) oracle and of the Ewald reference (section
2.1.3, the long-range half of eq. p3m_gravity; eq. pm_method, eq. W_CIC,
eq. weight_fourier, eq. symmetric_diff_4; eq. ewald_force with
eq. ewald_parameters).

Each step is pinned by a fact that does not restate its own formula:
- deposit: the cell-centred reading (a particle at a node centre lands on
  one node, one on a node corner on eight), mass conservation;
- readout: exact linear interpolation of a linear field;
- D4: exact derivative of polynomials up to degree 4 and the closed-form
  response (8 sin t - sin 2t) / 6 to a sampled sinusoid;
- the kernel: a uniform density gives no force; the whole PM chain
  conserves momentum exactly and matches the continuum long-range force
  (the reciprocal Ewald sum at the same split scale) to the discretisation
  error of CIC + D4, which a missing or single deconvolution or a 2-point
  difference exceeds several times;
- Ewald: Newton plus the cubic-lattice term -(4 pi / 3) r / L^3 at small
  separation, zero force on a symmetric lattice;
- P3M total (short range from the short-range oracle plus PM) against
  Ewald at the paper's split parameters.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import pm_oracle as pm

BOX = 1.0


def test_deposit_cell_centred_node():
    n = 8
    h = BOX / n
    pos = np.array([[h * 2.5, h * 5.5, h * 7.5]])
    rho = pm.cic_deposit(pos, np.array([3.0]), BOX, n)
    assert rho[2, 5, 7] == 3.0
    assert np.count_nonzero(rho) == 1


def test_deposit_cell_corner_and_wrap():
    n = 8
    h = BOX / n
    pos = np.array([[0.0, h * 3.0, h * 6.0]])     # a node corner on the periodic seam
    rho = pm.cic_deposit(pos, None, BOX, n)
    nz = np.argwhere(rho != 0)
    assert len(nz) == 8
    assert np.allclose(rho[rho != 0], 0.125, rtol=0, atol=1e-15)
    assert set(nz[:, 0]) == {n - 1, 0} and set(nz[:, 1]) == {2, 3} and set(nz[:, 2]) == {5, 6}


def test_deposit_conserves_mass():
    rng = np.random.default_rng(1)
    pos = rng.random((1000, 3))
    mass = rng.uniform(0.5, 2.0, 1000)
    rho = pm.cic_deposit(pos, mass, BOX, 16)
    assert abs(rho.sum() - mass.sum()) <= 1e-12 * mass.sum()
    assert rho.min() >= 0.0


def test_readout_interpolates_linear_field():
    n = 16
    h = BOX / n
    ix = np.arange(n, dtype=np.float64)
    grid = np.broadcast_to(ix[:, None, None] * 2.0 + 1.0, (n, n, n)).copy()
    rng = np.random.default_rng(2)
    # keep x inside [h/2, (n - 1.5) h] so that no weight wraps round
    pos = rng.random((200, 3))
    pos[:, 0] = h * (0.5 + (n - 2.0) * rng.random(200))
    got = pm.cic_readout(grid, pos, BOX)
    want = 2.0 * (pos[:, 0] / h - 0.5) + 1.0
    assert np.max(np.abs(got - want)) <= 1e-12


def test_d4_exact_on_quartic():
    n = 32
    m = np.arange(n, dtype=np.float64)
    p = 0.3 - 1.2 * m + 0.5 * m ** 2 - 0.02 * m ** 3 + 1e-3 * m ** 4
    dp = -1.2 + 1.0 * m - 0.06 * m ** 2 + 4e-3 * m ** 3
    phi = np.broadcast_to(p[:, None, None], (n, 4, 4)).copy()
    got = pm.d4(phi, 0)[2:n - 2, 1, 1]           # interior: no periodic wrap
    assert np.max(np.abs(got - dp[2:n - 2])) <= 1e-9 * np.max(np.abs(dp))


@pytest.mark.parametrize("q", [1, 3, 7])
def test_d4_response_to_sinusoid(q):
    n = 16
    t = 2.0 * math.pi * q / n
    m = np.arange(n)
    phi = np.broadcast_to(np.sin(t * m)[None, None, :], (4, 4, n)).copy()
    got = pm.d4(phi, 2)[0, 0]
    want = (8.0 * math.sin(t) - math.sin(2.0 * t)) / 6.0 * np.cos(t * m)
    assert np.max(np.abs(got - want)) <= 1e-13


def test_uniform_density_has_no_force():
    n = 16
    rho = np.full((n, n, n), 2.5)
    phi = pm.lr_potential(rho, BOX, 1.25 / n)
    assert np.max(np.abs(phi)) <= 1e-12
    # particles at every node centre: the deposit is uniform, the force zero
    h = BOX / n
    c = (np.arange(n) + 0.5) * h
    pos = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    acc = pm.pm_force(pos, None, BOX, n, 1.25 * h)
    assert np.max(np.abs(acc)) <= 1e-9


def test_pm_conserves_momentum_and_no_self_force():
    rng = np.random.default_rng(3)
    n = 16
    pos = rng.random((500, 3))
    pos[:100] = (0.5 + 0.05 * rng.standard_normal((100, 3))) % 1.0
    mass = rng.uniform(0.5, 2.0, 500)
    acc = pm.pm_force(pos, mass, BOX, n, 1.25 / n)
    tot = (mass[:, None] * acc).sum(axis=0)
    assert np.max(np.abs(tot)) <= 1e-12 * np.abs(mass[:, None] * acc).sum()
    one = pm.pm_force(pos[:1], None, BOX, n, 1.25 / n)
    assert np.max(np.abs(one)) <= 1e-10


def _pair_errors(n_grid, r_cells, n_dir, seed):
    h = BOX / n_grid
    x_s = 1.25 * h
    rng = np.random.default_rng(seed)
    errs = []
    for _ in range(n_dir):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        p0 = rng.random(3)
        pos = np.array([p0, (p0 + r_cells * h * d) % BOX])
        a = pm.pm_force(pos, None, BOX, n_grid, x_s)[0]
        ref = pm.ewald_long_range(pos, None, BOX, x_s, recv=[0])[0]
        errs.append(np.linalg.norm(a - ref) / np.linalg.norm(ref))
    return np.array(errs)


@pytest.mark.slow
def test_pm_matches_continuum_long_range():
    # at 3-4 cells the CIC + D4 + double deconvolution scheme is within ~1.5 %
    # of the continuum force on average; with no deconvolution (8 %), a single
    # one (4 %) or the 2-point difference (4.5 %) it is not
    e = np.concatenate([_pair_errors(32, 3.0, 12, 11), _pair_errors(32, 4.0, 12, 12)])
    assert e.mean() <= 0.02, e.mean()
    far = _pair_errors(32, 12.0, 8, 13)
    assert far.max() <= 0.006, far.max()


@pytest.mark.parametrize("r", [0.01, 0.002])
def test_ewald_small_separation(r):
    # periodic images of a cubic lattice add -(4 pi / 3) r / L^3 to Newton at
    # first order; the next term is O(r^3 / L^5)
    d = np.array([0.48, -0.6, 0.64])
    d /= np.linalg.norm(d)
    pos = np.array([[0.3, 0.4, 0.5], [0.3, 0.4, 0.5]])
    pos[1] -= r * d
    a = pm.ewald_force(pos, None, BOX, recv=[0])[0]
    want = -(1.0 / r ** 2 - 4.0 * math.pi / 3.0 * r / BOX ** 3) * d
    assert np.linalg.norm(a - want) <= 1e-8 * np.linalg.norm(want)


def test_ewald_symmetric_lattice_has_no_force():
    g = np.stack(np.meshgrid([0.1, 0.6], [0.2, 0.7], [0.3, 0.8], indexing="ij"), -1).reshape(-1, 3)
    assert np.max(np.abs(pm.ewald_force(g, None, BOX))) <= 1e-10


@pytest.mark.slow
def test_p3m_total_matches_ewald():
    """Short range (oracle, r_cut = 4.5 x_s) plus PM at x_s = 1.25 h against
    Ewald: the P3M force error is set by the PM discretisation near the
    split scale and by the short-range cut (g(4.5 x_s / 2 x_s) = 1.75 % of
    Newton is dropped beyond r_cut)."""
    n_grid = 32
    h = BOX / n_grid
    x_s = 1.25 * h
    r_cut = 4.5 * x_s
    rng = np.random.default_rng(5)
    n = 4096
    pos = rng.random((n, 3))
    pos[:512] = (0.5 + 0.03 * rng.standard_normal((512, 3))) % 1.0
    mass = rng.uniform(0.5, 2.0, n)
    recv = np.concatenate([np.arange(0, 512, 32), np.arange(512, n, 256)])
    a_lr = pm.pm_force(pos, mass, BOX, n_grid, x_s)[recv]
    a_sr, _, _, _ = oracle.force(pos, mass, BOX, x_s, r_cut, recv=recv)
    ref = pm.ewald_force(pos, mass, BOX, recv=recv)
    err = np.linalg.norm(a_lr + a_sr - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.sqrt(np.mean(err ** 2)) <= 1e-2 and err.max() <= 3e-2, (err.mean(), err.max())


@pytest.mark.parametrize("n_grid, r_cells", [(64, 3.0), (128, 8.0)])
def test_long_range_pair_closed_form(n_grid, r_cells):
    """The closed-form continuum long-range pair force (smoothed Newton plus
    the cubic-lattice image term) against the reciprocal Ewald sum at the
    same split scale: they agree to the next image term, about
    8 (r / L)^5 relative (3e-6 at r = 0.047 L, 8e-6 at 0.0625 L)."""
    h = BOX / n_grid
    x_s = 1.25 * h
    d = np.array([0.36, 0.48, -0.8])
    pos = np.array([[0.2, 0.7, 0.4], [0.2, 0.7, 0.4]])
    pos[1] -= r_cells * h * d
    ref = pm.ewald_long_range(pos, None, BOX, x_s, recv=[0])[0]
    got = pm.long_range_pair(pos[0] - pos[1], 1.0, BOX, x_s)
    assert np.linalg.norm(got - ref) <= 2e-5 * np.linalg.norm(ref)
