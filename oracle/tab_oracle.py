"""Plain oracle of the tabulated short-range kernel shape.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU legs are the only callers.  The GPU library never imports
this module and this module never imports the GPU library.

The paper tabulates the bracket of eq. p3m_gravity in a 1D table indexed by
r^2 between 0 and x_r^2 and reads it by nearest grid point (section 2.1.3,
"Other optimisations"; 2^12 entries by default), noting that a smaller table
with linear interpolation would also do.  Without softening the bracket
g(u)/r^3 diverges at r = 0, so the table here holds its smooth part:

    g(u) / r^3 = r^-3 + H(t) / (2 x_s)^3,   t = u^2,   H(t) = (g(u) - 1) / u^3,

and r^-3 is computed exactly.  Written from that definition, in FP64:

  - the table has n bins on r^2 in [0, r_cut^2); bin k covers
    [k, k + 1) r_cut^2 / n;
  - NGP reads H at the centre of the pair's bin;
  - linear interpolation reads H at the bin's two ends and interpolates at
    the pair's own position x = r^2 n / r_cut^2 inside it (FP64).

The one rule shared with the GPU is which bin a pair falls in: the paper
gives no rounding for the index, and a nearest-grid-point table is
discontinuous at bin edges, so both sides take k = floor(fl32(fl32(r^2) *
fl32(n / r_cut^2))) (capped at n - 1).  Linear interpolation is continuous,
so there the choice only matters at the level of FP64 rounding.  H comes
from erfc and exp (math module), with the Maclaurin series of g - 1 for
u < 0.05 where g - 1 cancels.
"""
from __future__ import annotations

import math

import numpy as np

from . import sq_dist

NGP, LINEAR = 1, 2


def h_exact(t):
    """H(t) = (g(u) - 1) / u^3 with u = sqrt(t), g(u) = erfc(u) + 2u exp(-u^2)/sqrt(pi)."""
    u = math.sqrt(t)
    if u < 0.05:
        # g - 1 = (2/sqrt(pi)) (-2/3 u^3 + 2/5 u^5 - 1/7 u^7 + 1/27 u^9 - ...)
        s = -2.0 / 3.0 + t * (2.0 / 5.0 + t * (-1.0 / 7.0 + t * (1.0 / 27.0)))
        return 2.0 / math.sqrt(math.pi) * s
    g = math.erfc(u) + 2.0 / math.sqrt(math.pi) * u * math.exp(-u * u)
    return (g - 1.0) / (u * u * u)


def bin_index(r2, n, rc2):
    """The pair's bin: floor(fl32(fl32(r^2) * fl32(n / rc2))), at most n - 1."""
    x = np.asarray(r2, dtype=np.float64).astype(np.float32) * np.float32(n / rc2)
    return np.minimum(x.astype(np.int64), n - 1)


def nodes(kind, n, rc2, c2):
    """FP64 values of H the table is made of: NGP the n bin centres, linear
    the n + 1 bin ends."""
    if kind == NGP:
        return np.array([h_exact((k + 0.5) * rc2 / n * c2) for k in range(n)])
    return np.array([h_exact(k * rc2 / n * c2) for k in range(n + 1)])


def shape_h(r2, kind, n, rc2, c2, node_values=None):
    """Tabulated H for squared distances r2 (FP64 everywhere but the bin)."""
    r2 = np.asarray(r2, dtype=np.float64)
    v = nodes(kind, n, rc2, c2) if node_values is None else node_values
    k = bin_index(r2, n, rc2)
    if kind == NGP:
        return v[k]
    f = r2 * (n / rc2) - k
    return v[k] + (v[k + 1] - v[k]) * f


def force(pos, mass, box, x_s, r_cut, recv, kind, n):
    """Short-range acceleration of the receivers `recv` with the tabulated
    shape, brute force over all suppliers (minimum image, r < r_cut, r > 0)."""
    pos = np.asarray(pos, dtype=np.float64)
    m = pos.shape[0]
    mu = np.ones(m) if mass is None else np.asarray(mass, dtype=np.float64)
    rc2 = r_cut * r_cut
    c2 = 1.0 / (4.0 * x_s * x_s)
    c3 = 1.0 / (8.0 * x_s ** 3)
    v = nodes(kind, n, rc2, c2)
    out = np.zeros((len(recv), 3))
    for a, i in enumerate(recv):
        d = pos[i] - pos
        d -= box * np.rint(d / box)
        r2 = sq_dist(d)                       # the cut-off test's rounding
        sel = (r2 < rc2) & (r2 > 0.0)
        r2s, ds, mus = r2[sel], d[sel], mu[sel]
        h = shape_h(r2s, kind, n, rc2, c2, v)
        s = mus * (1.0 / (r2s * np.sqrt(r2s)) + c3 * h)
        out[a] = -(s[:, None] * ds).sum(axis=0)
    return out
