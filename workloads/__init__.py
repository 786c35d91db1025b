"""Seeded synthetic workloads for the short-range P3M pair force.

Five particle sets, one per measured configuration:

  uniform32        N = 32^3 uniform random, PM grid 64^3, all active
  clustered128     N = 128^3 clustered (200 halos hold 30%), PM grid 256^3
  clustered256     N = 256^3 clustered, PM grid 512^3, rungs 0-7 from density
  diff64           N = 64^3 clustered, PM grid 128^3, Gaussian loss weights
  scale512         N = 512^3, 1000 halos hold 50%, PM grid 1024^3, rungs 0-7 from
                   grid counts

Every set lives in a unit periodic box with G*m = 1, x_s = 1.25 cells and
r_cut = 4.5 x_s.  Nothing here computes forces.
"""
from __future__ import annotations

import numpy as np

from .generators import (Workload, clustered_positions, gaussian_weights, grid_rungs, knn_rungs,
                         p3m_scales, rng_for, sample_indices, stratified_by_rung,
                         uniform_positions, wrap_unit, STREAM_LATTICE)

CONFIGS = {
    "uniform32": dict(config_id=1, n_side=32, n_pm=64, kind="uniform"),
    "clustered128": dict(config_id=2, n_side=128, n_pm=256, kind="clustered",
                         n_halos=200, halo_frac=0.30),
    "clustered256": dict(config_id=3, n_side=256, n_pm=512, kind="clustered",
                         n_halos=200, halo_frac=0.30, rungs=True),
    "diff64": dict(config_id=4, n_side=64, n_pm=128, kind="clustered",
                   n_halos=200, halo_frac=0.30, weights=True),
    "scale512": dict(config_id=5, n_side=512, n_pm=1024, kind="clustered",
                     n_halos=1000, halo_frac=0.50, rungs=True, rung_grid=True),
}


def make_workload(name: str, *, n_side: int | None = None, with_rungs: bool | None = None,
                  n_pm: int | None = None) -> Workload:
    """Build one named workload.  `n_side`/`n_pm` override the size for
    reduced-size variants used by quick tests (same recipe, same seeds)."""
    spec = dict(CONFIGS[name])
    cid = spec["config_id"]
    ns = n_side if n_side is not None else spec["n_side"]
    npm = n_pm if n_pm is not None else (spec["n_pm"] * ns) // spec["n_side"]
    n = ns ** 3
    x_s, r_cut = p3m_scales(npm)
    if spec["kind"] == "uniform":
        pos = uniform_positions(n, rng_for(cid, STREAM_LATTICE))
        meta = {}
    else:
        pos, meta = clustered_positions(ns, npm, spec["n_halos"], spec["halo_frac"], cid)
    mass = np.ones(n, dtype=np.float64)
    wl = Workload(name=name, config_id=cid, n=n, box=1.0, n_pm=npm, x_s=x_s, r_cut=r_cut,
                  pos=pos, mass=mass, meta=meta)
    want_rungs = spec.get("rungs", False) if with_rungs is None else with_rungs
    if want_rungs:
        # k-NN density for the sets up to 256^3; at 512^3 a k-d tree takes too
        # long, so counts on an n_side^3 grid summed over 3x3x3 cells are used
        wl.rung = grid_rungs(pos, n_grid=ns) if spec.get("rung_grid") else knn_rungs(pos)
    if spec.get("weights", False):
        wl.weights = gaussian_weights(n, cid)
    return wl


def random_particles(n: int, seed: int, box: float = 1.0, mass_range=(0.5, 2.0),
                     active_frac: float | None = None):
    """Small generic particle set for unit tests: uniform positions, random
    masses in mass_range and an optional random active mask."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = wrap_unit(rng.random((n, 3)) * box, box)
    mass = rng.uniform(mass_range[0], mass_range[1], n)
    active = None
    if active_frac is not None:
        active = (rng.random(n) < active_frac).astype(np.uint8)
    return pos, mass, active


def lattice_sites(n_side: int, n_sites: int, n_dup: int, n_edge: int, seed: int):
    """Particles on sites of an n_side^3 lattice in the unit box (n_side a
    power of two, so every coordinate and every separation is exact in
    FP64), for tests whose pair distances fall exactly on a cut-off.

    n_sites distinct random sites, then n_dup copies of some of them
    (coincident distinct particles) and n_edge copies with one coordinate
    moved from 0 to exactly 1.0 (the same point of the periodic box).
    Returns (pos, ijk): positions (N, 3) and the integer site indices, with
    1.0 given as index n_side."""
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = rng.choice(n_side ** 3, size=n_sites, replace=False)
    ijk = np.stack([flat // (n_side * n_side), (flat // n_side) % n_side, flat % n_side], axis=1)
    dup = ijk[rng.integers(0, n_sites, n_dup)]
    zero = np.flatnonzero((ijk == 0).any(axis=1))
    edge = ijk[rng.choice(zero, size=min(n_edge, zero.size), replace=False)].copy()
    for row in edge:
        row[rng.choice(np.flatnonzero(row == 0))] = n_side
    ijk = np.concatenate([ijk, dup, edge]).astype(np.int64)
    perm = rng.permutation(ijk.shape[0])
    ijk = ijk[perm]
    return ijk.astype(np.float64) / n_side, ijk


__all__ = ["CONFIGS", "make_workload", "random_particles", "Workload", "sample_indices",
           "stratified_by_rung", "wrap_unit", "p3m_scales", "lattice_sites"]
