"""Pins of the CPU oracle against facts that do not come from the oracle.

The paper prints no force values, so the oracle is fixed by:
  * the potential it must be the gradient of (the Ewald split of section
    2.1.1: short-range potential erfc(r/2x_s)/r), differentiated numerically
    with mpmath at high precision;
  * the Newtonian limit r << x_s (eq. force);
  * the strict cut-off and the nearest-image rule (section 2.1.3);
  * symmetries: Newton's third law, inversion symmetry of a lattice,
    translation / permutation / axis-permutation / reflection;
  * the paper's printed rejection fractions for ideal cubic tiles;
  * agreement of brute force with an independent cell-list walk.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from workloads import lattice_sites, make_workload, random_particles

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
mp.mp.dps = 40


@pytest.fixture(autouse=True, scope="module")
def _built(oracle_lib):
    return oracle_lib


def two_body(r_vec, x_s, r_cut, mu1=1.0, box=1.0, base=(0.5, 0.5, 0.5)):
    x0 = np.array(base, dtype=np.float64)
    x1 = x0 - np.asarray(r_vec, dtype=np.float64)
    pos = np.stack([x0, x1])
    acc, cnt, absum, _ = oracle.force(pos, np.array([1.0, mu1]), box, x_s, r_cut)
    return acc[0], int(cnt[0]), pos


def mp_potential_grad(rv, x_s):
    """mpmath gradient of psi(x) = erfc(|x| / (2 x_s)) / |x| at rv."""
    xs = mp.mpf(x_s)

    def psi(x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        return mp.erfc(r / (2 * xs)) / r

    pt = [mp.mpf(float(v)) for v in rv]
    return np.array([float(mp.diff(psi, pt, tuple(int(i == d) for i in range(3))))
                     for d in range(3)])


def mp_potential_hessian(rv, x_s):
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


# --- kernel shape ---------------------------------------------------------

@pytest.mark.parametrize("r_over_xs", [0.05, 0.5, 1.0, 2.0, 3.3, 4.0, 4.49])
def test_force_is_gradient_of_short_range_potential(r_over_xs):
    """a_0 = mu_1 grad_{x0} [erfc(r/2x_s)/r]: the bracket of eq. p3m_gravity
    is the derivative of the split potential G_sr of section 2.1.1."""
    x_s = 0.01
    r_cut = 4.5 * x_s
    direction = np.array([0.48, -0.6, 0.64])
    direction /= np.linalg.norm(direction)
    rv = direction * r_over_xs * x_s
    a0, cnt, pos = two_body(rv, x_s, r_cut, mu1=1.7)
    assert cnt == 1
    ref = 1.7 * mp_potential_grad(pos[0] - pos[1], x_s)
    assert np.max(np.abs(a0 - ref)) <= 1e-13 * np.linalg.norm(ref)


def test_newtonian_limit():
    """For r << x_s the split force tends to the point-mass force of eq. force."""
    x_s = 0.02
    rv = np.array([1e-6, -2e-6, 0.5e-6])
    a0, cnt, pos = two_body(rv, x_s, 4.5 * x_s, mu1=2.5)
    rv = pos[0] - pos[1]                   # the separation actually stored
    r = np.linalg.norm(rv)
    newton = -2.5 * rv / r ** 3
    assert cnt == 1
    # relative deviation is (4 / (3 sqrt(pi))) u^3 with u = r / (2 x_s) ~ 6e-5
    assert np.max(np.abs(a0 - newton)) <= 1e-11 * np.linalg.norm(newton)


def test_cutoff_is_strict_and_hard():
    x_s = 1.25 / 64
    r_cut = 4.5 * x_s                      # 0.087890625, exact in binary
    inside, c_in, _ = two_body([r_cut * (1 - 1e-12), 0, 0], x_s, r_cut)
    outside, c_out, _ = two_body([r_cut * (1 + 1e-12), 0, 0], x_s, r_cut)
    exact, c_eq, pos = two_body([r_cut, 0, 0], x_s, r_cut, base=(0.25, 0.5, 0.5))
    assert (pos[0, 0] - pos[1, 0]) == r_cut   # the separation is exactly r_cut
    assert c_in == 1 and c_out == 0 and c_eq == 0
    assert np.all(outside == 0) and np.all(exact == 0)
    # the force does not taper to zero: its magnitude just inside equals the
    # potential gradient there (a jump at r_cut)
    ref = mp_potential_grad([r_cut * (1 - 1e-12), 0, 0], x_s)
    assert abs(np.linalg.norm(inside) - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(inside) > 1.0


def test_coincident_pair_contributes_nothing():
    pos = np.array([[0.3, 0.3, 0.3], [0.3, 0.3, 0.3], [0.31, 0.3, 0.3]])
    acc, cnt, _, _ = oracle.force(pos, None, 1.0, 0.01, 0.045)
    assert cnt.tolist() == [1, 1, 2]
    assert np.all(np.isfinite(acc))


def lattice_counts(ijk, n_side, r_cut_sites):
    """Accepted partners per particle by integer arithmetic: the minimum-image
    site difference (each component reduced to [-n_side/2, n_side/2)),
    0 < d^2 < r_cut^2, all in lattice units."""
    d = ijk[:, None, :] - ijk[None, :, :]
    d = (d + n_side // 2) % n_side - n_side // 2
    d2 = (d * d).sum(axis=2)
    return ((d2 > 0) & (d2 < r_cut_sites ** 2)).sum(axis=1)


def test_lattice_counts_are_integer_exact():
    """Sites of a 64^3 lattice with r_cut = 4 spacings: many pairs lie exactly
    on the cut-off (strict <, section 2.1.3), duplicated sites are coincident
    distinct particles (no contribution), and a coordinate of exactly 1.0 is
    the same point as 0.0 (nearest image).  The oracle's accepted-pair counts
    must equal the integer count, and every pair's separation is exact."""
    n_side, k = 64, 4
    pos, ijk = lattice_sites(n_side, 3000, 200, 40, seed=7)
    r_cut = k / n_side
    x_s = r_cut / 4.5
    want = lattice_counts(ijk, n_side, k)
    d = ijk[:, None, :] - ijk[None, :, :]
    d = (d + n_side // 2) % n_side - n_side // 2
    assert ((d * d).sum(axis=2) == k * k).sum() > 100     # pairs exactly at r_cut exist
    for method in ("brute", "tiled"):
        acc, cnt, _ = oracle.force_full(pos, None, 1.0, x_s, r_cut, method=method)
        assert np.array_equal(cnt, want), method
        assert np.all(np.isfinite(acc))


def test_minimum_image_across_boundary():
    """The nearest image n' is used (eq. p3m_gravity): a pair split by the
    periodic boundary acts like the same pair in the interior."""
    x_s, r_cut = 0.01, 0.045
    pos_edge = np.array([[0.01, 0.5, 0.999], [0.99, 0.5, 0.002]])
    pos_mid = np.array([[0.51, 0.5, 0.499], [0.49, 0.5, 0.502]])
    a_edge, c_edge, _, _ = oracle.force(pos_edge, None, 1.0, x_s, r_cut)
    a_mid, c_mid, _, _ = oracle.force(pos_mid, None, 1.0, x_s, r_cut)
    assert c_edge.tolist() == [1, 1] and c_mid.tolist() == [1, 1]
    assert np.allclose(a_edge, a_mid, rtol=1e-12, atol=0)
    assert a_edge[0, 0] < 0          # pulled toward the image at x = -0.01


def test_mpmath_pair_sum_tiny():
    """High-precision pair sum for 7 particles near the box corner, each pair
    force taken as the mpmath gradient of the split potential."""
    pos, mass, _ = random_particles(7, seed=11)
    pos = (pos * 0.12 - 0.06) % 1.0             # cluster around the corner (wraps)
    x_s = 0.02
    r_cut = 4.5 * x_s
    acc, cnt, _, _ = oracle.force(pos, mass, 1.0, x_s, r_cut)
    for i in range(7):
        ref = np.zeros(3)
        c = 0
        for j in range(7):
            if j == i:
                continue
            d = pos[i] - pos[j]
            d -= np.rint(d)
            if np.dot(d, d) < r_cut ** 2:
                ref += mass[j] * mp_potential_grad(d, x_s)
                c += 1
        assert cnt[i] == c
        assert np.max(np.abs(acc[i] - ref)) <= 1e-12 * max(np.linalg.norm(ref), 1e-300)


# --- symmetries -------------------------------------------------------------

def test_newtons_third_law_momentum():
    pos, mass, _ = random_particles(3000, seed=5)
    acc, cnt, absum, _ = oracle.force(pos, mass, 1.0, 0.02, 0.09)
    total = (mass[:, None] * acc).sum(axis=0)
    scale = (mass * absum).sum()
    assert np.max(np.abs(total)) <= 1e-14 * scale
    assert cnt.sum() % 2 == 0


def test_lattice_forces_vanish():
    n = 16
    q = (np.arange(n) + 0.5) / n
    pos = np.stack(np.meshgrid(q, q, q, indexing="ij"), axis=-1).reshape(-1, 3)
    x_s = 1.25 / 32
    acc, cnt, absum, _ = oracle.force(pos, None, 1.0, x_s, 4.5 * x_s)
    assert cnt.min() == cnt.max() and cnt[0] > 50
    assert np.max(np.linalg.norm(acc, axis=1) / absum) <= 1e-14


def test_translation_permutation_axis_reflection():
    pos, mass, _ = random_particles(2000, seed=9)
    x_s, r_cut = 0.025, 0.1125
    a, cnt, absum, _ = oracle.force(pos, mass, 1.0, x_s, r_cut)

    shift = np.array([0.3711, -0.125, 0.0625])   # exact in binary for the last two
    a_t, c_t, _, _ = oracle.force((pos + shift) % 1.0, mass, 1.0, x_s, r_cut)
    assert np.array_equal(cnt, c_t)
    assert oracle.errors(a_t, a, absum)["e_max_cond"] <= 1e-11

    perm = np.random.default_rng(3).permutation(pos.shape[0])
    a_p, c_p, _, _ = oracle.force(pos[perm], mass[perm], 1.0, x_s, r_cut)
    assert np.array_equal(c_p, cnt[perm])
    assert oracle.errors(a_p, a[perm], absum[perm])["e_max_cond"] <= 1e-15

    # r^2 = fma(dz, dz, fma(dy, dy, dx dx)) rounds differently once the axes
    # are permuted: agreement to rounding, not to the bit
    axes = [2, 0, 1]
    a_ax, _, _, _ = oracle.force(pos[:, axes], mass, 1.0, x_s, r_cut)
    assert oracle.errors(a_ax, a[:, axes], absum)["e_max_cond"] <= 1e-14

    refl = pos.copy()
    refl[:, 1] = -refl[:, 1]
    a_r, _, _, _ = oracle.force(refl, mass, 1.0, x_s, r_cut)
    expect = a.copy()
    expect[:, 1] = -expect[:, 1]
    assert oracle.errors(a_r, expect, absum)["e_max_cond"] <= 1e-15


def test_active_mask_restricts_receivers_only():
    """Receivers only on active rungs, suppliers always (section 2.2.2)."""
    pos, mass, active = random_particles(3000, seed=21, active_frac=0.2)
    x_s, r_cut = 0.02, 0.09
    a_all, _, _ = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute")
    a_sub, _, _ = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active, method="brute")
    on = active.astype(bool)
    assert np.array_equal(a_sub[on], a_all[on])
    assert np.all(a_sub[~on] == 0)


# --- cell list --------------------------------------------------------------

@pytest.mark.parametrize("which", ["uniform", "clustered"])
def test_brute_equals_tiled(which):
    """The cell-list walk reaches the same sum; only the summation order
    differs (section 2.1.3 / section 3: geometry does not change the force)."""
    if which == "uniform":
        pos, mass, _ = random_particles(6000, seed=2)
        x_s = 1.25 / 40
    else:
        wl = make_workload("diff64", n_side=20)
        pos, mass, x_s = wl.pos, wl.mass * 1.3, wl.x_s
    r_cut = 4.5 * x_s
    a_b, c_b, ab_b, _ = oracle.force(pos, mass, 1.0, x_s, r_cut, method="brute")
    a_t, c_t, ab_t, _ = oracle.force(pos, mass, 1.0, x_s, r_cut, method="tiled")
    assert np.array_equal(c_b, c_t)
    assert oracle.errors(a_t, a_b, ab_b)["e_max_cond"] <= 1e-14
    assert np.allclose(ab_t, ab_b, rtol=1e-14, atol=0)


def _golden_rejections():
    out = {}
    with open(os.path.join(GOLDEN, "rejection_fractions.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def test_rejection_fractions_match_paper():
    """Ideal cubic tiles of side exactly x_r: the cut-off rejects 9/66/91/98 %
    of candidate pairs in same/face/edge/corner tile pairs (section 2.1.3)."""
    golden = _golden_rejections()
    rng = np.random.default_rng(1234)
    pos = rng.random((60000, 3))
    cand, acc = oracle.cell_census(pos, 1.0, 1.0 / 8)
    rejected = 100.0 * (1.0 - acc / cand)
    for kind, got in zip(["same", "face", "edge", "corner"], rejected):
        assert abs(got - golden[kind]) <= 0.6, (kind, got)
