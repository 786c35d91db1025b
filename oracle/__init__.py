"""Python face of the plain FP64 CPU oracle (sr_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
imports this package and this package never imports the GPU library.

All functions take float64 numpy arrays; positions are (n, 3) row-major.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sr_oracle.c")
_LIB = os.path.join(_HERE, "libsr_oracle.so")

CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-msse4.1", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile sr_oracle.c with gcc into libsr_oracle.so (next to it)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    lib.p3o_threads.restype = ctypes.c_int
    lib.p3o_force.argtypes = [_I64, _P, _P, _D, _D, _D, _D, _I64, _P, _P, _P, _P]
    lib.p3o_force.restype = None
    lib.p3o_force_tiled.argtypes = [_I64, _P, _P, _D, _D, _D, _D, _I64, _P, _P, _P, _P]
    lib.p3o_force_tiled.restype = ctypes.c_int
    lib.p3o_cell_census.argtypes = [_I64, _P, _D, _D, _P, _P]
    lib.p3o_cell_census.restype = ctypes.c_int
    lib.p3o_vjp.argtypes = [_I64, _P, _P, _P, _P, _D, _D, _D, _D, _I64, _P, _P]
    lib.p3o_vjp.restype = None
    lib.p3o_vjp_tiled.argtypes = [_I64, _P, _P, _P, _P, _D, _D, _D, _D, _I64, _P, _P]
    lib.p3o_vjp_tiled.restype = ctypes.c_int
    lib.p3o_fd_grad.argtypes = [_I64, _P, _P, _P, _P, _D, _D, _D, _D, _D, ctypes.c_int, _I64,
                                _P, _P, _P]
    lib.p3o_fd_grad.restype = None
    lib.p3o_sq_dist.argtypes = [_I64, _P, _P]
    lib.p3o_sq_dist.restype = None
    _lib = lib
    return lib


def sq_dist(d):
    """r^2 = fma(dz, dz, fma(dy, dy, dx * dx)) for the rows of d (m x 3): the
    rounding every cut-off decision uses (numpy has no fused multiply-add)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(d.shape[0])
    if d.shape[0]:
        _load().p3o_sq_dist(d.shape[0], _ptr(d), _ptr(out))
    return out


# B-spline softening length from the Plummer-equivalent softening length
# (section 2.1.1, below eq. bspline_force: eps_B = 2.8 eps).
BSPLINE_PER_PLUMMER = 2.8


def eps_b_of(eps: float) -> float:
    return BSPLINE_PER_PLUMMER * float(eps)


def threads() -> int:
    """OpenMP threads the oracle runs with (OMP_NUM_THREADS or all cores)."""
    return int(_load().p3o_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(pos, mass, active=None):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    assert pos.ndim == 2 and pos.shape[1] == 3
    mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
    active = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    return pos, mass, active


def _receivers(n, active, recv):
    if recv is not None:
        return np.ascontiguousarray(recv, dtype=np.int64)
    if active is None:
        return np.arange(n, dtype=np.int64)
    return np.nonzero(active)[0].astype(np.int64)


def force(pos, mass, box, x_s, r_cut, recv=None, active=None, method="brute", eps=0.0):
    """Short-range acceleration of receivers.

    Receivers are `recv` (indices) if given, else the particles with a
    nonzero `active` entry, else all.  Returns (acc[n_recv,3], count[n_recv],
    absum[n_recv], recv) where count is the number of accepted pairs and
    absum = sum_j |pair acceleration|.  method "tiled" uses the cell list
    and falls back to brute force when the box holds fewer than 3 cells.
    eps > 0 adds the B-spline softening bracket with eps_B = 2.8 eps.
    """
    pos, mass, active = _prep(pos, mass, active)
    n = pos.shape[0]
    r = _receivers(n, active, recv)
    acc = np.zeros((r.size, 3))
    cnt = np.zeros(r.size, dtype=np.int64)
    absum = np.zeros(r.size)
    lib = _load()
    args = (n, _ptr(pos), _ptr(mass), box, x_s, r_cut, eps_b_of(eps), r.size, _ptr(r), _ptr(acc),
            _ptr(cnt), _ptr(absum))
    if method == "tiled" and lib.p3o_force_tiled(*args) == 0:
        pass
    else:
        lib.p3o_force(*args)
    return acc, cnt, absum, r


def force_full(pos, mass, box, x_s, r_cut, active=None, method="tiled", eps=0.0):
    """acc for every particle (zero rows for inactive ones), count, absum."""
    pos, mass, active = _prep(pos, mass, active)
    n = pos.shape[0]
    acc_r, cnt_r, abs_r, r = force(pos, mass, box, x_s, r_cut, active=active, method=method,
                                   eps=eps)
    acc = np.zeros((n, 3))
    cnt = np.zeros(n, dtype=np.int64)
    absum = np.zeros(n)
    acc[r] = acc_r
    cnt[r] = cnt_r
    absum[r] = abs_r
    return acc, cnt, absum


def cell_census(pos, box, r_cut):
    """(candidates[4], accepted[4]) by neighbour kind: same/face/edge/corner."""
    pos, _, _ = _prep(pos, None)
    c = np.zeros(4, dtype=np.int64)
    a = np.zeros(4, dtype=np.int64)
    if _load().p3o_cell_census(pos.shape[0], _ptr(pos), box, r_cut, _ptr(c), _ptr(a)) != 0:
        raise ValueError("cell census needs at least 3 cells per dimension")
    return c, a


def vjp(pos, mass, active, w, box, x_s, r_cut, kidx=None, method="brute", eps=0.0):
    """dL/dx_k for L = sum_{i active} w_i . a_i at listed k (default all)."""
    pos, mass, active = _prep(pos, mass, active)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = pos.shape[0]
    k = np.arange(n, dtype=np.int64) if kidx is None else np.ascontiguousarray(kidx, np.int64)
    g = np.zeros((k.size, 3))
    lib = _load()
    args = (n, _ptr(pos), _ptr(mass), _ptr(active), _ptr(w), box, x_s, r_cut, eps_b_of(eps), k.size,
            _ptr(k), _ptr(g))
    if method == "tiled" and lib.p3o_vjp_tiled(*args) == 0:
        pass
    else:
        lib.p3o_vjp(*args)
    return g


def fd_grad(pos, mass, active, w, box, x_s, r_cut, kidx, h=1e-6, mode="fixed", eps=0.0):
    """Central finite-difference dL/dx_k; returns (grad[n_k,3], straddle[n_k])."""
    pos, mass, active = _prep(pos, mass, active)
    w = np.ascontiguousarray(w, dtype=np.float64)
    k = np.ascontiguousarray(kidx, dtype=np.int64)
    g = np.zeros((k.size, 3))
    st = np.zeros(k.size, dtype=np.uint8)
    _load().p3o_fd_grad(pos.shape[0], _ptr(pos), _ptr(mass), _ptr(active), _ptr(w), box, x_s,
                        r_cut, eps_b_of(eps), h, 0 if mode == "fixed" else 1, k.size, _ptr(k),
                        _ptr(g), _ptr(st))
    return g, st


def errors(a, ref, absum):
    """Force error measures over receivers.

    e_l2       = ||a - ref||_2 / ||ref||_2 over all components;
    e_max_cond = max_i |a_i - ref_i| / absum_i, the error relative to the
                 sum of pair-force magnitudes (immune to cancellation).  A row
                 with absum_i = 0 has no accepted pair, so its exact value is
                 0: any nonzero |a_i - ref_i| there makes e_max_cond infinite;
    p999       = 99.9th percentile of |a_i - ref_i| / |ref_i| over the rows
                 with ref_i != 0 (numpy's linear interpolation between ranks);
    max_abs    = max_i |a_i - ref_i|.
    """
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    absum = np.asarray(absum, dtype=np.float64)
    assert a.shape == ref.shape and a.ndim == 2 and absum.shape == (a.shape[0],)
    d = np.linalg.norm(a - ref, axis=1)
    nr = np.linalg.norm(ref, axis=1)
    den = np.linalg.norm(ref)
    e_l2 = float(np.linalg.norm(a - ref) / den) if den > 0 else float(np.linalg.norm(a - ref))
    ok = absum > 0
    if np.any(d[~ok] != 0.0):
        e_cond = float("inf")
    else:
        e_cond = float(np.max(d[ok] / absum[ok])) if ok.any() else 0.0
    nz = nr > 0
    p999 = float(np.percentile(d[nz] / nr[nz], 99.9)) if nz.any() else 0.0
    return dict(e_l2=e_l2, e_max_cond=e_cond, p999=p999, max_abs=float(np.max(d, initial=0.0)))
