"""MI355X (gfx950) short-range P3M pair force: Python binding of libp3msr.

Thin ctypes layer over the C ABI declared in include/p3msr.h.  PyTorch only
supplies device memory and the current HIP stream; every step of the force
path runs in the library's HIP kernels.  There is no CPU fallback: if the
library is not built, or no GPU is present, calls raise.

    import paper_2112_01508_amd as p3
    acc = p3.sr_force(pos, mass, active, box=1.0, x_s=x_s, r_cut=r_cut, precision="fp32")

`sr_force` is differentiable with respect to `pos` (torch.autograd): its
backward calls the library's hand-written adjoint kernel.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp3msr.so")

P3M_FP64 = 0
P3M_FP32 = 1
P3M_OK = 0
P3M_EINVAL = -1
P3M_ENOMEM = -2
P3M_EHIP = -3
P3M_EUNSUPPORTED = -4
_CODES = {P3M_EINVAL: "EINVAL", P3M_ENOMEM: "ENOMEM", P3M_EHIP: "EHIP",
          P3M_EUNSUPPORTED: "EUNSUPPORTED"}


class P3MError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("p3msr %s (%d): %s" % (_CODES.get(code, "?"), code, message))
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("receivers", ctypes.c_int64),
                ("interactions", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("clusters", ctypes.c_int64), ("items", ctypes.c_int64),
                ("steps", ctypes.c_int64),
                ("tiles_per_dim", ctypes.c_int32), ("subtiles_per_dim", ctypes.c_int32),
                ("item_target", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ms_build", ctypes.c_float), ("ms_pairs", ctypes.c_float),
                ("ms_total", ctypes.c_float), ("cluster_size", ctypes.c_int32),
                ("screen", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("screened", ctypes.c_int64), ("eps_b", ctypes.c_double),
                ("fp64_steps", ctypes.c_int64), ("ms_sort", ctypes.c_float),
                ("deterministic", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LrStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_grid", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("ms_sort", ctypes.c_float), ("ms_deposit", ctypes.c_float), ("ms_fft_x_fwd", ctypes.c_float),
                ("ms_fft_y_fwd", ctypes.c_float), ("ms_fft_z_conv", ctypes.c_float),
                ("ms_fft_y_inv", ctypes.c_float), ("ms_fft_x_inv", ctypes.c_float),
                ("ms_readout", ctypes.c_float), ("ms_total", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KdkStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("highest_rung", ctypes.c_int32),
                ("substeps", ctypes.c_int32), ("sr_calls", ctypes.c_int32),
                ("lr_calls", ctypes.c_int32), ("ms_total", ctypes.c_float),
                ("pad", ctypes.c_int32), ("interactions", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


P3M_KDK_FIXED_RUNGS = 1
P3M_TUNE_ADJOINT = 4          # p3m_sr_autotune level flag: tune the adjoint
P3M_TUNE_FORCE = 8            # autotune level flag: time even when a cached layout matches

_lib = None
_lib_lock = threading.Lock()
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_I64 = ctypes.c_int64

EXPORTS = {
    "p3m_sr_create": ([ctypes.POINTER(_P), _I], _I),
    "p3m_sr_destroy": ([_P], _I),
    "p3m_sr_last_error": ([], ctypes.c_char_p),
    "p3m_sr_version": ([], ctypes.c_char_p),
    "p3m_sr_force": ([_P, _P, _P, _P, _I64, _D, _D, _D, _I, _P, _P], _I),
    "p3m_sr_force_backward": ([_P, _P, _P, _P, _I64, _D, _D, _D, _I, _P, _P, _P], _I),
    "p3m_sr_force_batched": ([_P, _P, _P, _P, _I64, _I, _P, _D, _D, _D, _I, _P, _P], _I),
    "p3m_sr_autotune": ([_P, _P, _P, _P, _I64, _D, _D, _D, _I, _I, _P, _P], _I),
    "p3m_sr_set_config": ([_P, _I, _I, _I, _I], _I),
    "p3m_sr_set_timing": ([_P, _I], _I),
    "p3m_sr_set_deterministic": ([_P, _I], _I),
    "p3m_sr_set_debug_limits": ([_P, _I64, _I], _I),
    "p3m_sr_set_softening": ([_P, ctypes.c_double], _I),
    "p3m_sr_set_shape": ([_P, _I, _I], _I),
    "p3m_sr_get_stats": ([_P, ctypes.POINTER(Stats)], _I),
    "p3m_lr_force": ([_P, _P, _P, _P, _I64, _D, _I, _D, _P, _P], _I),
    "p3m_lr_get_stats": ([_P, ctypes.POINTER(LrStats)], _I),
    "p3m_force": ([_P, _P, _P, _P, _I64, _D, _D, _D, _I, _I, _P, _P], _I),
    "p3m_sr_force_noalloc": ([_P, _P, _P, _P, _I64, _D, _D, _D, _I, _P, _P], _I),
    "p3m_sr_autotune_batched": ([_P, _P, _P, _P, _I64, _I, _P, _D, _D, _D, _I, _I, _P, _P], _I),
    "p3m_sr_set_tune_cache": ([_P, ctypes.c_char_p], _I),
    "p3m_sr_tune_status": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], _I),
    "p3m_sr_tune_cache_check": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int)], _I),
    "p3m_kdk_step": ([_P, _P, _P, _P, _P, _I64, _D, _D, _D, _I, _D, _I, _D, _D, _I, _I, _I, _P],
                     _I),
    "p3m_kdk_get_stats": ([_P, ctypes.POINTER(KdkStats)], _I),
}


def load_library(path: str = LIB_PATH):
    """Load libp3msr.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError("libp3msr.so is not built (%s); run __graft_entry__.build() or "
                              "python paper_2112_01508_amd/build.py" % path)
        lib = ctypes.CDLL(path)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def tune_cache_check(path):
    """(entries, lines) of an autotuner cache file as a handle would read it
    (p3m_sr_tune_cache_check; needs no GPU)."""
    lib = load_library()
    e, l = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib.p3m_sr_tune_cache_check(os.fsencode(path), ctypes.byref(e), ctypes.byref(l)))
    return e.value, l.value


def _check(rc: int):
    if rc != P3M_OK:
        raise P3MError(rc, load_library().p3m_sr_last_error().decode())


def _prec(precision) -> int:
    if precision in ("fp32", "float32", P3M_FP32):
        return P3M_FP32
    if precision in ("fp64", "float64", P3M_FP64):
        return P3M_FP64
    raise ValueError("precision must be 'fp32' or 'fp64'")


def _dev_ptr(t, dtype, shape_tail, name, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device != device:
        raise ValueError("%s must be a tensor on %s" % (name, device))
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError("%s has shape %s" % (name, tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """One library handle bound to a GPU (not thread-safe)."""

    def __init__(self, device=None):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available: the p3msr path has no CPU fallback")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        h = _P()
        _check(lib.p3m_sr_create(ctypes.byref(h), self.device.index))
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.p3m_sr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling helpers -------------------------------------------------
    def _inputs(self, pos, mass, sel, sel_name):
        pos = _dev_ptr(pos, torch.float64, (3,), "pos", self.device)
        if pos.dim() != 2:
            raise ValueError("pos must be (n, 3)")
        n = pos.shape[0]
        mass = _dev_ptr(mass, torch.float64, (), "mass", self.device)
        if mass is not None and mass.shape[0] != n:
            raise ValueError("mass must have n entries")
        sel = _dev_ptr(sel, torch.uint8, (), sel_name, self.device)
        if sel is not None and sel.shape[0] != n:
            raise ValueError("%s must have n entries" % sel_name)
        return pos, mass, sel, n

    @staticmethod
    def _p(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    def _out(self, out, n):
        """An n x 3 FP64 output on this device: the caller's (checked) or new."""
        if out is None:
            return torch.empty((n, 3), dtype=torch.float64, device=self.device)
        _dev_ptr(out, torch.float64, (3,), "out", self.device)
        if out.shape[0] != n:
            raise ValueError("out must have %d rows (got %d)" % (n, out.shape[0]))
        return out

    # -- entry points ------------------------------------------------------------
    def force(self, pos, mass=None, active=None, *, box, x_s, r_cut, precision="fp32", out=None):
        pos, mass, active, n = self._inputs(pos, mass, active, "active")
        out = self._out(out, n)
        _check(self._lib.p3m_sr_force(self._h, self._p(pos), self._p(mass), self._p(active), n,
                                      float(box), float(x_s), float(r_cut), _prec(precision),
                                      self._p(out), _stream_ptr(self.device)))
        return out

    def force_noalloc(self, pos, mass=None, active=None, *, box, x_s, r_cut, precision="fp32",
                      out=None):
        """p3m_sr_force_noalloc: the force with the library's fixed workspace
        (no device allocation inside the call; n <= 2^18).  `out` (n x 3 FP64
        on the device) is allocated here when not given."""
        pos, mass, active, n = self._inputs(pos, mass, active, "active")
        out = self._out(out, n)
        _check(self._lib.p3m_sr_force_noalloc(self._h, self._p(pos), self._p(mass),
                                              self._p(active), n, float(box), float(x_s),
                                              float(r_cut), _prec(precision), self._p(out),
                                              _stream_ptr(self.device)))
        return out

    def force_backward(self, pos, mass, active, grad_acc, *, box, x_s, r_cut, precision="fp32"):
        pos, mass, active, n = self._inputs(pos, mass, active, "active")
        grad_acc = _dev_ptr(grad_acc.contiguous(), torch.float64, (3,), "grad_acc", self.device)
        out = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        _check(self._lib.p3m_sr_force_backward(self._h, self._p(pos), self._p(mass),
                                               self._p(active), n, float(box), float(x_s),
                                               float(r_cut), _prec(precision), self._p(grad_acc),
                                               self._p(out), _stream_ptr(self.device)))
        return out

    def force_batched(self, pos, mass, rung, min_rung, *, box, x_s, r_cut, precision="fp32",
                      out=None):
        pos, mass, rung, n = self._inputs(pos, mass, rung, "rung")
        thr = bytes(int(v) for v in min_rung)
        n_sub = len(thr)
        if out is None:
            out = torch.empty((n_sub, n, 3), dtype=torch.float64, device=self.device)
        elif (out.device != self.device or out.dtype != torch.float64
              or tuple(out.shape) != (n_sub, n, 3) or not out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 (%d, %d, 3) tensor on %s"
                             % (n_sub, n, self.device))
        buf = ctypes.create_string_buffer(thr, max(n_sub, 1))
        _check(self._lib.p3m_sr_force_batched(self._h, self._p(pos), self._p(mass),
                                              self._p(rung), n, n_sub,
                                              ctypes.cast(buf, ctypes.c_void_p), float(box),
                                              float(x_s), float(r_cut), _prec(precision),
                                              self._p(out), _stream_ptr(self.device)))
        return out

    def autotune_batched(self, pos, mass, rung, min_rung, *, box, x_s, r_cut, precision="fp32",
                         level=1, force=False, out=None):
        """Measure-and-keep tuning of the rung-batched call on these rungs and
        thresholds (see p3m_sr_autotune_batched); `out` (n_sub x n x 3 FP64)
        is optional scratch for the trials."""
        pos, mass, rung, n = self._inputs(pos, mass, rung, "rung")
        thr = bytes(int(v) for v in min_rung)
        n_sub = len(thr)
        if out is None:
            out = torch.empty((n_sub, n, 3), dtype=torch.float64, device=self.device)
        buf = ctypes.create_string_buffer(thr, max(n_sub, 1))
        lvl = int(level) | (P3M_TUNE_FORCE if force else 0)
        _check(self._lib.p3m_sr_autotune_batched(self._h, self._p(pos), self._p(mass),
                                                 self._p(rung), n, n_sub,
                                                 ctypes.cast(buf, ctypes.c_void_p), float(box),
                                                 float(x_s), float(r_cut), _prec(precision), lvl,
                                                 self._p(out), _stream_ptr(self.device)))

    def set_tune_cache(self, path=None):
        """Autotuner cache file (None: the default; "": none), loaded now."""
        p = None if path is None else str(path).encode()
        _check(self._lib.p3m_sr_set_tune_cache(self._h, p))

    def tune_status(self) -> dict:
        """What the last autotune call did: trials timed, cached layout used."""
        t, c = ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.p3m_sr_tune_status(self._h, ctypes.byref(t), ctypes.byref(c)))
        return {"trials": t.value, "from_cache": bool(c.value)}

    def force_long_range(self, pos, mass=None, active=None, *, box, n_grid, x_s, out=None):
        """Long-range (PM) acceleration (n, 3) FP64; see p3m_lr_force."""
        pos, mass, active, n = self._inputs(pos, mass, active, "active")
        out = self._out(out, n)
        _check(self._lib.p3m_lr_force(self._h, self._p(pos), self._p(mass), self._p(active), n,
                                      float(box), int(n_grid), float(x_s), self._p(out),
                                      _stream_ptr(self.device)))
        return out

    def force_total(self, pos, mass=None, active=None, *, box, x_s, r_cut, n_grid,
                    precision="fp32", out=None):
        """Short- plus long-range P3M acceleration (n, 3) FP64, the two halves
        overlapped on two streams; see p3m_force."""
        pos, mass, active, n = self._inputs(pos, mass, active, "active")
        out = self._out(out, n)
        _check(self._lib.p3m_force(self._h, self._p(pos), self._p(mass), self._p(active), n,
                                   float(box), float(x_s), float(r_cut), int(n_grid),
                                   _prec(precision), self._p(out), _stream_ptr(self.device)))
        return out

    def kdk_step(self, pos, vel, mass, rung, *, box, x_s, r_cut, n_grid, dt, n_steps=1,
                 eta=0.025, eps=0.0, max_rung=7, fixed_rungs=False, precision="fp64"):
        """Advance pos, vel (n x 3 FP64, in place) by n_steps steps of dt with
        the rung-hierarchical KDK scheme; rung (n uint8) receives eq. rung at
        the end (or is the fixed input with fixed_rungs).  See p3m_kdk_step."""
        pos, mass, rung, n = self._inputs(pos, mass, rung, "rung")
        vel = _dev_ptr(vel, torch.float64, (3,), "vel", self.device)
        if vel.shape[0] != n:
            raise ValueError("vel must have n rows")
        if rung is None:
            raise ValueError("rung (n uint8) is required")
        _check(self._lib.p3m_kdk_step(self._h, self._p(pos), self._p(vel), self._p(mass),
                                      self._p(rung), n, float(box), float(x_s), float(r_cut),
                                      int(n_grid), float(dt), int(n_steps), float(eta),
                                      float(eps), int(max_rung),
                                      P3M_KDK_FIXED_RUNGS if fixed_rungs else 0,
                                      _prec(precision), _stream_ptr(self.device)))
        return pos, vel, rung

    def kdk_stats(self) -> dict:
        s = KdkStats()
        _check(self._lib.p3m_kdk_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def lr_stats(self) -> dict:
        s = LrStats()
        _check(self._lib.p3m_lr_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def autotune(self, pos, mass=None, active=None, *, box, x_s, r_cut, precision="fp32",
                 level=1, out=None, adjoint=False, force=False):
        """Measure-and-keep tuning of the decomposition for these inputs (of
        the adjoint instead of the forward with adjoint=True); `out` (n x 3
        FP64 on the device) is optional scratch for the trials."""
        pos, mass, active, n = self._inputs(pos, mass, active, "active")
        scratch = self._out(out, n)
        lvl = int(level) | (P3M_TUNE_ADJOINT if adjoint else 0) | (P3M_TUNE_FORCE if force else 0)
        _check(self._lib.p3m_sr_autotune(self._h, self._p(pos), self._p(mass), self._p(active),
                                         n, float(box), float(x_s), float(r_cut),
                                         _prec(precision), lvl, self._p(scratch),
                                         _stream_ptr(self.device)))

    def set_config(self, subtiles_per_dim=0, item_target=0, cluster_size=0, screen=-1):
        """Fix the decomposition (0 / -1 = automatic); see p3m_sr_set_config."""
        _check(self._lib.p3m_sr_set_config(self._h, int(subtiles_per_dim), int(item_target),
                                           int(cluster_size), int(screen)))

    SHAPES = {"poly": 0, "table_ngp": 1, "table_linear": 2}

    def set_shape(self, kind="poly", table_size=0):
        """FP32 forward kernel shape: "poly" (default), "table_ngp" or
        "table_linear" with table_size entries (0 = largest); see
        p3m_sr_set_shape."""
        k = self.SHAPES[kind] if isinstance(kind, str) else int(kind)
        _check(self._lib.p3m_sr_set_shape(self._h, k, int(table_size)))

    def set_softening(self, eps=0.0):
        """B-spline softening with eps_B = 2.8 eps for every following call
        (0 = point particles); see p3m_sr_set_softening."""
        _check(self._lib.p3m_sr_set_softening(self._h, float(eps)))

    def set_timing(self, enable=True):
        _check(self._lib.p3m_sr_set_timing(self._h, 1 if enable else 0))

    def set_deterministic(self, enable=True):
        """Fixed summation order, the same bits call after call; see
        p3m_sr_set_deterministic."""
        _check(self._lib.p3m_sr_set_deterministic(self._h, 1 if enable else 0))

    def set_debug_limits(self, max_workspace_bytes=0, fail_after=-1):
        """Make workspace growth fail with P3M_ENOMEM past a byte cap or after
        fail_after more growths (0 / -1: off); see p3m_sr_set_debug_limits."""
        _check(self._lib.p3m_sr_set_debug_limits(self._h, int(max_workspace_bytes),
                                                 int(fail_after)))

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.p3m_sr_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()


_contexts: dict = {}


def default_context(device=None) -> Context:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    ctx = _contexts.get(dev)
    if ctx is None:
        ctx = Context(dev)
        _contexts[dev] = ctx
    return ctx


class _SRForce(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pos, mass, active, box, x_s, r_cut, precision, ctx):
        acc = ctx.force(pos.detach(), mass, active, box=box, x_s=x_s, r_cut=r_cut,
                        precision=precision)
        fctx.save_for_backward(pos.detach())
        fctx.extra = (mass, active, box, x_s, r_cut, precision, ctx)
        return acc

    @staticmethod
    def backward(fctx, grad_acc):
        (pos,) = fctx.saved_tensors
        mass, active, box, x_s, r_cut, precision, ctx = fctx.extra
        grad_pos = ctx.force_backward(pos, mass, active, grad_acc, box=box, x_s=x_s, r_cut=r_cut,
                                      precision=precision)
        return grad_pos, None, None, None, None, None, None, None


def sr_force(pos, mass=None, active=None, *, box=1.0, x_s, r_cut, precision="fp32",
             context: Context | None = None):
    """Short-range P3M acceleration (n, 3) FP64 of the active particles.

    Differentiable with respect to `pos` for a fixed pair set; `mass` and
    `active` are not differentiated."""
    ctx = context or default_context(pos.device)
    if pos.requires_grad and torch.is_grad_enabled():
        return _SRForce.apply(pos, mass, active, box, x_s, r_cut, precision, ctx)
    return ctx.force(pos, mass, active, box=box, x_s=x_s, r_cut=r_cut, precision=precision)


def sr_force_batched(pos, mass, rung, min_rung, *, box=1.0, x_s, r_cut, precision="fp32",
                     context: Context | None = None):
    """Accelerations (n_sub, n, 3) of the nested rung subsets rung >= min_rung[k]."""
    ctx = context or default_context(pos.device)
    return ctx.force_batched(pos, mass, rung, min_rung, box=box, x_s=x_s, r_cut=r_cut,
                             precision=precision)


def lr_force(pos, mass=None, active=None, *, box=1.0, n_grid, x_s,
             context: Context | None = None):
    """Long-range (PM) P3M acceleration (n, 3) FP64 of the active particles."""
    ctx = context or default_context(pos.device)
    return ctx.force_long_range(pos, mass, active, box=box, n_grid=n_grid, x_s=x_s)


def p3m_force(pos, mass=None, active=None, *, box=1.0, x_s, r_cut, n_grid, precision="fp32",
              context: Context | None = None):
    """The whole P3M acceleration (n, 3) FP64 (short range + PM) of the active particles."""
    ctx = context or default_context(pos.device)
    return ctx.force_total(pos, mass, active, box=box, x_s=x_s, r_cut=r_cut, n_grid=n_grid,
                           precision=precision)


__all__ = ["Context", "P3MError", "Stats", "LrStats", "KdkStats", "lr_force", "p3m_force",
           "P3M_KDK_FIXED_RUNGS", "P3M_TUNE_ADJOINT", "default_context", "load_library", "sr_force",
           "sr_force_batched", "LIB_PATH", "P3M_FP32", "P3M_FP64", "EXPORTS"]
