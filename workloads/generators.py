"""Seeded synthetic particle sets for the short-range P3M pair force.

This module only draws inputs: positions, masses, rungs, loss weights and
sample indices.  It holds none of the pair-force arithmetic, so the CPU
oracle and the GPU library can both be fed from it without sharing any of
the method's code.

The shapes follow the workloads of the paper's P3M setup (section 2.1.3,
eq. p3m_parameters and eq. phi_gridsize_preference): a periodic cube of side
L, a PM grid of n_pm cells per dimension, split scale x_s = 1.25 L/n_pm and
cut-off x_r = 4.5 x_s.  The paper's own initial conditions come from CLASS
and GADGET runs that are not available here; the clustered generator below
stands in for them (a Zel'dovich-displaced lattice plus NFW-like halos).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Seed layout: seed = 1000*config_id + stream, one PCG64 stream per purpose.
STREAM_LATTICE = 0
STREAM_FIELD = 1
STREAM_HALOS = 2
STREAM_WEIGHTS = 3
STREAM_SAMPLES = 4


def rng_for(config_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config_id + stream))


def wrap_unit(x: np.ndarray, box: float = 1.0) -> np.ndarray:
    """Map coordinates into [0, box), making sure no value lands on box."""
    y = np.mod(x, box)
    y[y >= box] = 0.0
    return y


def uniform_positions(n: int, rng: np.random.Generator, box: float = 1.0) -> np.ndarray:
    return wrap_unit(rng.random((n, 3)) * box, box)


def zeldovich_displacement(n_side: int, rms: float, rng: np.random.Generator,
                           spectral_index: float = -2.0) -> np.ndarray:
    """Displacement field psi on an n_side^3 lattice (box = 1).

    A Gaussian density field with P(k) proportional to k^spectral_index is
    drawn as white noise times sqrt(P) with the DC mode removed; the
    displacement is psi(k) = i k delta(k) / k^2, scaled so that the rms of
    |psi| equals `rms`.  Returned as float64 array (n_side^3, 3) in lattice
    (C) order.
    """
    noise = rng.standard_normal((n_side, n_side, n_side))
    dk = np.fft.rfftn(noise)
    del noise
    f = np.fft.fftfreq(n_side, d=1.0 / n_side) * 2.0 * np.pi
    fz = np.fft.rfftfreq(n_side, d=1.0 / n_side) * 2.0 * np.pi
    kx = f[:, None, None]
    ky = f[None, :, None]
    kz = fz[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    amp = k2 ** (spectral_index / 4.0)  # sqrt(P(k)) = k^(n/2)
    dk *= amp
    dk[0, 0, 0] = 0.0
    dk /= k2
    out = np.empty((n_side ** 3, 3), dtype=np.float64)
    for d, kd in enumerate((kx, ky, kz)):
        comp = np.fft.irfftn(1j * kd * dk, s=(n_side, n_side, n_side), axes=(0, 1, 2))
        out[:, d] = comp.reshape(-1)
        del comp
    cur = math.sqrt(float(np.mean(np.sum(out * out, axis=1))))
    out *= rms / cur
    return out


def _nfw_mass_profile(x: np.ndarray) -> np.ndarray:
    return np.log1p(x) - x / (1.0 + x)


def nfw_radii(u: np.ndarray, conc: np.ndarray) -> np.ndarray:
    """Solve mu(x) = u * mu(c) for x in [0, c], mu(x) = ln(1+x) - x/(1+x).

    A tabulated inverse of mu gives the starting point; Newton steps
    (mu'(x) = x / (1+x)^2) then converge to double precision.  Returns x/c,
    the radius in units of the truncation radius R.
    """
    target = u * _nfw_mass_profile(conc)
    t = np.linspace(0.0, 1.0, 8193)
    x_tab = float(conc.max()) * t * t                  # denser near 0, where mu ~ x^2/2
    mu_tab = _nfw_mass_profile(x_tab)
    x = np.interp(target, mu_tab, x_tab)
    for _ in range(4):
        d = x / ((1.0 + x) * (1.0 + x))
        step = np.where(d > 0, (_nfw_mass_profile(x) - target) / np.where(d > 0, d, 1.0), 0.0)
        x = np.clip(x - step, 0.0, conc)
    return x / conc


@dataclass
class Workload:
    name: str
    config_id: int
    n: int
    box: float
    n_pm: int
    x_s: float
    r_cut: float
    pos: np.ndarray                      # (n, 3) float64 in [0, box)
    mass: np.ndarray                     # (n,) float64, G*m
    rung: Optional[np.ndarray] = None    # (n,) uint8
    weights: Optional[np.ndarray] = None  # (n, 3) float64 loss weights
    meta: dict = field(default_factory=dict)

    def active_subset(self, k: int) -> np.ndarray:
        """Receiver mask of the kick at hierarchy depth k: rung >= k."""
        if self.rung is None:
            return np.ones(self.n, dtype=np.uint8)
        return (self.rung >= k).astype(np.uint8)


def p3m_scales(n_pm: int, box: float = 1.0):
    """x_s = 1.25 cell and x_r = 4.5 x_s (paper's default P3M parameters)."""
    h = box / n_pm
    x_s = 1.25 * h
    return x_s, 4.5 * x_s


def clustered_positions(n_side: int, n_pm: int, n_halos: int, halo_frac: float,
                        config_id: int, box: float = 1.0,
                        rms_cells: float = 0.5,
                        r_min_cells: float = 2.0, r_max_cells: float = 20.0,
                        c_min: float = 5.0, c_max: float = 15.0) -> tuple[np.ndarray, dict]:
    """Displaced lattice plus NFW-like halos.

    (i) lattice (q + 1/2) L / n_side displaced by a Zel'dovich field with
    P(k) ~ k^-2 and rms |psi| = rms_cells PM cells; (ii) a seeded subset of
    halo_frac * N particles is moved into n_halos halos with centres uniform
    in the box, truncation radius R log-uniform in [r_min, r_max] cells,
    concentration uniform in [c_min, c_max], particle share proportional to
    R^3 (multinomial) and NFW radial profile truncated at R, isotropic.
    """
    n = n_side ** 3
    h = box / n_pm
    q = (np.arange(n_side, dtype=np.float64) + 0.5) * (box / n_side)
    pos = np.empty((n, 3), dtype=np.float64)
    pos[:, 0] = np.repeat(q, n_side * n_side)
    pos[:, 1] = np.tile(np.repeat(q, n_side), n_side)
    pos[:, 2] = np.tile(q, n_side * n_side)
    psi = zeldovich_displacement(n_side, rms_cells * h, rng_for(config_id, STREAM_FIELD))
    pos += psi * box
    del psi

    rng = rng_for(config_id, STREAM_HALOS)
    centres = rng.random((n_halos, 3)) * box
    radius = h * np.exp(rng.uniform(math.log(r_min_cells), math.log(r_max_cells), n_halos))
    conc = rng.uniform(c_min, c_max, n_halos)
    m_halo = int(round(halo_frac * n))
    chosen = rng.permutation(n)[:m_halo]
    share = radius ** 3
    share = share / share.sum()
    counts = rng.multinomial(m_halo, share)
    owner = np.repeat(np.arange(n_halos), counts)
    u = rng.random(m_halo)
    xr = nfw_radii(u, conc[owner]) * radius[owner]
    dirs = rng.standard_normal((m_halo, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    pos[chosen] = centres[owner] + dirs * xr[:, None]
    pos = wrap_unit(pos, box)
    meta = dict(n_halos=n_halos, halo_frac=halo_frac, halo_counts=counts,
                halo_radius=radius, halo_conc=conc, halo_centres=centres)
    return pos, meta


def knn_rungs(pos: np.ndarray, k: int = 32, box: float = 1.0, max_rung: int = 7,
              exponent_step: float = 1.5, workers: int = -1) -> np.ndarray:
    """Rung from local density: clamp(floor(log2(rho/rho_bar) / 1.5), 0, 7).

    rho/rho_bar is the k-nearest-neighbour estimate k / ((4/3) pi d_k^3 N / L^3)
    with a periodic KD-tree (self excluded).
    """
    from scipy.spatial import cKDTree
    n = pos.shape[0]
    tree = cKDTree(pos, boxsize=box)
    d, _ = tree.query(pos, k=[k + 1], workers=workers)
    dk = d[:, 0]
    ratio = k / ((4.0 / 3.0) * math.pi * dk ** 3 * n / box ** 3)
    rung = np.floor(np.log2(ratio) / exponent_step)
    return np.clip(rung, 0, max_rung).astype(np.uint8)


def grid_rungs(pos: np.ndarray, n_grid: int, box: float = 1.0, max_rung: int = 7,
               exponent_step: float = 1.5) -> np.ndarray:
    """Rung from local density for very large sets: clamp(floor(log2(rho/rho_bar)/1.5), 0, 7)
    with rho/rho_bar estimated from particle counts on an n_grid^3 grid summed
    over the periodic 3x3x3 block of cells around each particle's cell."""
    n = pos.shape[0]
    cell = np.minimum((pos * (n_grid / box)).astype(np.int64), n_grid - 1)
    flat = (cell[:, 0] * n_grid + cell[:, 1]) * n_grid + cell[:, 2]
    del cell
    counts = np.bincount(flat, minlength=n_grid ** 3).astype(np.float32)
    counts = counts.reshape(n_grid, n_grid, n_grid)
    block = counts
    for axis in range(3):
        block = np.roll(block, 1, axis) + block + np.roll(block, -1, axis)
    del counts
    mean = 27.0 * n / float(n_grid) ** 3
    ratio = block.reshape(-1)[flat] / mean
    del block, flat
    rung = np.floor(np.log2(np.maximum(ratio, 1e-30)) / exponent_step)
    return np.clip(rung, 0, max_rung).astype(np.uint8)


def gaussian_weights(n: int, config_id: int) -> np.ndarray:
    return rng_for(config_id, STREAM_WEIGHTS).standard_normal((n, 3))


def sample_indices(n: int, count: int, config_id: int, salt: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(1000 * config_id + STREAM_SAMPLES + 7919 * salt))
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)


def stratified_by_rung(rung: np.ndarray, per_rung: int, config_id: int) -> np.ndarray:
    """Up to per_rung seeded receivers from each rung value present."""
    rng = rng_for(config_id, STREAM_SAMPLES)
    out = []
    for r in range(int(rung.max()) + 1):
        idx = np.nonzero(rung == r)[0]
        if idx.size:
            out.append(rng.choice(idx, size=min(per_rung, idx.size), replace=False))
    return np.sort(np.concatenate(out)).astype(np.int64)
