"""Plain FP64 oracle of the long-range (PM) half of P3M gravity and of the
Ewald sum it is checked against.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
imports this module and this module never imports the GPU library.

What is computed (CONCEPT 1.0, section 2.1.3, the long-range half of
eq. p3m_gravity, which runs the PM steps of eq. pm_method with the Poisson
kernel replaced by the long-range kernel of eq. ewald_potential):

  1. particles -> mesh (eq. density_grid_implementation with eq. W_CIC):
     rho_m = sum_j mu_j W(x_m - x_j), grid points cell-centred at
     x_m = h (m + 1/2), h = L / n, periodic;
  2. forward FFT (unnormalised), multiply by
     exp(-x_s^2 k^2) / k^2 * prod_d sinc(h k_d / 2)^-4
     (the long-range kernel and two CIC deconvolutions, eq. weight_fourier),
     k = 2 pi hvec / L with signed integer hvec, k = 0 set to zero;
  3. inverse FFT normalised so that F F^-1 = 1;
  4. the 4-point symmetric difference of eq. symmetric_diff_4 along each axis;
  5. mesh -> particles with the same CIC weights (eq. pm_force), times
     4 pi / h^4 (the prefactor of eq. p3m_gravity with G m folded into mu).

The result is an acceleration, like the short-range oracle: mu_j = G m_j
and a_i = f_i / m_i.  numpy's FFT serves as the transform; every other
step is written out as its definition, without fusion.

The Ewald reference is eq. ewald_force written out: real-space images with
|x_ijn| < 3.6 L and reciprocal vectors with h^2 < 10 at x_s = L / 4
(eq. ewald_parameters).  ewald_long_range is its reciprocal half alone at
an arbitrary split scale, summed until the Gaussian factor is below 1e-17,
which is the continuum quantity the PM steps approximate.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc


def _wrap(pos, box):
    p = np.asarray(pos, dtype=np.float64) % box
    p[p >= box] -= box          # (x % L) can round up to L itself
    return p


def cic_nodes(pos, box, n_grid):
    """Per particle and axis: the lower node index i0 (in [0, n)) and the
    weights (1 - f, f) of nodes i0 and i0 + 1 of eq. W_CIC for cell-centred
    nodes (node m at h (m + 1/2))."""
    h = box / n_grid
    u = _wrap(pos, box) / h - 0.5
    i0 = np.floor(u)
    f = u - i0
    return i0.astype(np.int64) % n_grid, f


def cic_deposit(pos, mass, box, n_grid):
    """rho_m = sum_j mu_j W_CIC(x_m - x_j) on an (n, n, n) grid indexed
    [ix, iy, iz] (eq. density_grid_implementation with the background term
    dropped, as the paper does by zeroing the k = 0 mode)."""
    n = int(pos.shape[0])
    mu = np.ones(n) if mass is None else np.asarray(mass, dtype=np.float64)
    i0, f = cic_nodes(pos, box, n_grid)
    rho = np.zeros((n_grid,) * 3)
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = (i0[:, 0] + cx) % n_grid
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + cy) % n_grid
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + cz) % n_grid
                np.add.at(rho, (ix, iy, iz), mu * wx * wy * wz)
    return rho


def lr_green(n_grid, box, x_s):
    """exp(-x_s^2 k^2) / k^2 / prod_d sinc^4(h k_d / 2) on the FFT grid,
    zero at k = 0 (the long-range kernel of eq. p3m_gravity with its two CIC
    deconvolutions)."""
    hv = np.fft.fftfreq(n_grid, d=1.0 / n_grid)          # signed integers
    k1 = 2.0 * math.pi * hv / box
    kx, ky, kz = k1[:, None, None], k1[None, :, None], k1[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    # sinc(h k / 2) with h k / 2 = pi hv / n; np.sinc(t) = sin(pi t) / (pi t)
    s1 = np.sinc(hv / n_grid)
    w2 = (s1[:, None, None] * s1[None, :, None] * s1[None, None, :]) ** 4
    g = np.zeros_like(k2)
    nz = k2 > 0
    g[nz] = np.exp(-x_s * x_s * k2[nz]) / k2[nz] / w2[nz]
    return g


def lr_potential(rho, box, x_s):
    """F^-1 { G F{rho} } with the normalised inverse (steps 2-3)."""
    n_grid = rho.shape[0]
    return np.real(np.fft.ifftn(lr_green(n_grid, box, x_s) * np.fft.fftn(rho)))


def d4(phi, axis):
    """(phi_{m-2} - 8 phi_{m-1} + 8 phi_{m+1} - phi_{m+2}) / 12 along axis,
    periodic (eq. symmetric_diff_4); per grid unit."""
    return (np.roll(phi, 2, axis) - 8.0 * np.roll(phi, 1, axis)
            + 8.0 * np.roll(phi, -1, axis) - np.roll(phi, -2, axis)) / 12.0


def cic_readout(grid, pos, box):
    """sum_m W_CIC(x_i - x_m) grid_m for every particle (eq. pm_force)."""
    n_grid = grid.shape[0]
    i0, f = cic_nodes(pos, box, n_grid)
    out = np.zeros(pos.shape[0])
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        ix = (i0[:, 0] + cx) % n_grid
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + cy) % n_grid
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + cz) % n_grid
                out += wx * wy * wz * grid[ix, iy, iz]
    return out


def pm_force(pos, mass, box, n_grid, x_s, active=None):
    """Long-range acceleration of every particle (all particles supply;
    rows of inactive receivers are 0), steps 1-5 above."""
    pos = np.asarray(pos, dtype=np.float64)
    h = box / n_grid
    phi = lr_potential(cic_deposit(pos, mass, box, n_grid), box, x_s)
    acc = np.empty((pos.shape[0], 3))
    for d in range(3):
        acc[:, d] = cic_readout(d4(phi, d), pos, box)
    acc *= 4.0 * math.pi / h ** 4
    if active is not None:
        acc[np.asarray(active) == 0] = 0.0
    return acc


def _kvectors(box, h2max=None, hmax=None, x_s=None, tiny=1e-17):
    if hmax is None:
        # exp(-x_s^2 k^2) < tiny beyond |k| = sqrt(-ln tiny) / x_s
        hmax = int(math.ceil(math.sqrt(-math.log(tiny)) / x_s * box / (2.0 * math.pi)))
    r = np.arange(-hmax, hmax + 1)
    hx, hy, hz = np.meshgrid(r, r, r, indexing="ij")
    hv = np.stack([hx.ravel(), hy.ravel(), hz.ravel()], axis=1)
    q = (hv * hv).sum(axis=1)
    keep = q > 0
    if h2max is not None:
        keep &= q < h2max
    else:
        keep &= q <= hmax * hmax
    return 2.0 * math.pi / box * hv[keep].astype(np.float64)


def _reciprocal(pos, mu, box, x_s, kv, recv, chunk=4096):
    """-sum_j mu_j (4 pi / L^3) sum_k exp(-x_s^2 k^2) / k^2 sin(k.(x_i - x_j)) k."""
    k2 = (kv * kv).sum(axis=1)
    c = 4.0 * math.pi / box ** 3 * np.exp(-x_s * x_s * k2) / k2
    out = np.zeros((len(recv), 3))
    for a, i in enumerate(recv):
        acc = np.zeros(3)
        for s in range(0, pos.shape[0], chunk):
            d = pos[i] - pos[s:s + chunk]                        # (m, 3)
            ph = d @ kv.T                                        # (m, K)
            acc -= ((mu[s:s + chunk, None] * np.sin(ph)) @ (c[:, None] * kv)).sum(axis=0)
        out[a] = acc
    return out


def ewald_long_range(pos, mass, box, x_s, recv=None):
    """Reciprocal half of eq. ewald_force at split scale x_s, the sum over
    k taken until exp(-x_s^2 k^2) < 1e-17: the continuum long-range
    acceleration that the PM steps approximate."""
    pos = _wrap(pos, box)
    n = pos.shape[0]
    mu = np.ones(n) if mass is None else np.asarray(mass, dtype=np.float64)
    recv = np.arange(n) if recv is None else np.asarray(recv)
    return _reciprocal(pos, mu, box, x_s, _kvectors(box, x_s=x_s), recv)


def long_range_pair(sep, mu, box, x_s):
    """Continuum long-range acceleration of a particle at separation sep =
    x_i - x_j from a single supplier mu_j, for |sep| much smaller than the
    box: the Gaussian-smoothed Newtonian force -mu (1 - g(u)) sep / r^3
    (erf(r / 2 x_s) / r is the long-range potential of eq. ewald_potential,
    u = r / (2 x_s), g as in the short-range kernel) plus the first-order
    pull of the periodic images of a cubic lattice, +mu (4 pi / 3) sep / L^3;
    the next image term is O(r^3 / L^5), about 8 (r / L)^5 relative."""
    sep = np.asarray(sep, dtype=np.float64)
    r = float(np.linalg.norm(sep))
    u = r / (2.0 * x_s)
    g = math.erfc(u) + 2.0 / math.sqrt(math.pi) * u * math.exp(-u * u)
    return -mu * ((1.0 - g) / r ** 3 - 4.0 * math.pi / (3.0 * box ** 3)) * sep


def ewald_force(pos, mass, box, recv=None):
    """Periodic Newtonian acceleration by eq. ewald_force (no softening)
    with x_s = L / 4, real-space images |x_ijn| < 3.6 L and h^2 < 10
    (eq. ewald_parameters)."""
    pos = _wrap(pos, box)
    n = pos.shape[0]
    mu = np.ones(n) if mass is None else np.asarray(mass, dtype=np.float64)
    recv = np.arange(n) if recv is None else np.asarray(recv)
    x_s = box / 4.0
    r_max = 3.6 * box
    m = int(math.ceil(r_max / box)) + 1
    r = np.arange(-m, m + 1)
    nx, ny, nz = np.meshgrid(r, r, r, indexing="ij")
    images = box * np.stack([nx.ravel(), ny.ravel(), nz.ravel()], axis=1).astype(np.float64)
    # images that can hold a point within r_max of a point of the box
    images = images[np.sqrt((images * images).sum(axis=1)) < r_max + math.sqrt(3.0) * box]
    out = _reciprocal(pos, mu, box, x_s, _kvectors(box, h2max=10, hmax=3), recv)
    c = 1.0 / (math.sqrt(math.pi) * x_s)
    for a, i in enumerate(recv):
        others = np.delete(np.arange(n), i)
        for s0 in range(0, others.size, 256):
            js = others[s0:s0 + 256]
            x = pos[i] - (pos[js, None, :] + images[None, :, :])   # x_ijn, (m, I, 3)
            r2 = (x * x).sum(axis=2)
            sel = r2 < r_max * r_max
            rr = np.sqrt(np.where(sel, r2, 1.0))
            s = erfc(rr / (2.0 * x_s)) / (r2 * rr) + c * np.exp(-r2 / (4.0 * x_s * x_s)) / r2
            s = np.where(sel, s, 0.0) * mu[js, None]
            out[a] -= (s[:, :, None] * x).sum(axis=(0, 1))
    return out
