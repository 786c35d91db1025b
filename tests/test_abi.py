"""The C-ABI library loads and exports every entry point that
include/p3msr.h declares; argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "p3msr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(p3m_(?:(?:sr|lr|kdk)_\w+|force))\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2112_01508_amd as p3
    if not os.path.exists(p3.LIB_PATH):
        from paper_2112_01508_amd import build
        build.build()
    return p3.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["p3m_sr_create", "p3m_sr_destroy", "p3m_sr_force", "p3m_sr_force_backward",
                 "p3m_sr_force_batched", "p3m_sr_autotune", "p3m_sr_get_stats",
                 "p3m_sr_last_error", "p3m_lr_force", "p3m_lr_get_stats", "p3m_kdk_step",
                 "p3m_kdk_get_stats", "p3m_force"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2112_01508_amd as p3
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in p3.EXPORTS, name
    assert lib.p3m_sr_version().decode().startswith("p3msr")


def _force(lib, **kw):
    args = dict(h=None, pos=ctypes.c_void_p(8), mass=None, active=None, n=10, box=1.0,
                x_s=0.01, r_cut=0.045, prec=1, out=ctypes.c_void_p(8), stream=None)
    args.update(kw)
    return lib.p3m_sr_force(args["h"], args["pos"], args["mass"], args["active"], args["n"],
                            args["box"], args["x_s"], args["r_cut"], args["prec"], args["out"],
                            args["stream"])


@pytest.mark.parametrize("kw, msg", [
    (dict(n=-1), "n must be"),
    (dict(box=0.0), "box"),
    (dict(x_s=-1.0), "x_s"),
    (dict(r_cut=0.0), "r_cut"),
    (dict(r_cut=0.6), "box/2"),
    (dict(r_cut=0.34), "3 tiles"),
    (dict(prec=7), "precision"),
    (dict(pos=None), "required"),
    (dict(out=None), "required"),
    (dict(pos=ctypes.c_void_p(12)), "aligned"),
    (dict(), "NULL handle"),
])
def test_invalid_arguments_are_rejected(lib, kw, msg):
    rc = _force(lib, **kw)
    assert rc == -1
    assert msg in lib.p3m_sr_last_error().decode()


def test_batched_and_config_checks(lib):
    assert lib.p3m_sr_force_batched(None, ctypes.c_void_p(8), None, ctypes.c_void_p(8), 10, 0,
                                    None, 1.0, 0.01, 0.045, 1, ctypes.c_void_p(8), None) == -1
    assert "n_sub" in lib.p3m_sr_last_error().decode()
    assert lib.p3m_sr_set_config(None, 2, 0, 0, -1) == -1
    assert "NULL handle" in lib.p3m_sr_last_error().decode()
    for args, msg in (((17, 0, 0, -1), "subtiles"), ((2, 5, 0, -1), "item_target"),
                      ((2, 0, 12, -1), "cluster_size"), ((2, 0, 8, 2), "screen")):
        assert lib.p3m_sr_set_config(None, *args) == -1
        assert msg in lib.p3m_sr_last_error().decode()
    h = ctypes.c_void_p(0)
    # no GPU in the build container: create must fail cleanly, not crash
    if os.environ.get("HIP_VISIBLE_DEVICES", "x") == "":
        assert lib.p3m_sr_create(ctypes.byref(h), 0) != 0


def test_n_too_large_is_unsupported(lib):
    assert _force(lib, n=1 << 31) == -4


@pytest.mark.parametrize("kw, msg", [
    (dict(n=-1), "n must be"),
    (dict(box=0.0), "box"),
    (dict(x_s=0.0), "x_s"),
    (dict(n_grid=48), "power of two"),
    (dict(n_grid=8), "power of two"),
    (dict(n_grid=2048), "power of two"),
    (dict(pos=None), "required"),
    (dict(out=None), "required"),
    (dict(out=ctypes.c_void_p(20)), "aligned"),
    (dict(), "NULL handle"),
])
def test_long_range_invalid_arguments_are_rejected(lib, kw, msg):
    args = dict(h=None, pos=ctypes.c_void_p(8), mass=None, active=None, n=10, box=1.0,
                n_grid=64, x_s=1.25 / 64, out=ctypes.c_void_p(8), stream=None)
    args.update(kw)
    rc = lib.p3m_lr_force(args["h"], args["pos"], args["mass"], args["active"], args["n"],
                          args["box"], args["n_grid"], args["x_s"], args["out"], args["stream"])
    assert rc == -1
    assert msg in lib.p3m_sr_last_error().decode()


@pytest.mark.parametrize("kw, msg", [
    (dict(n=-1), "n must be"),
    (dict(r_cut=0.6), "box/2"),
    (dict(prec=5), "precision"),
    (dict(n_grid=48), "n_grid"),
    (dict(dt=0.0), "dt"),
    (dict(n_steps=0), "n_steps"),
    (dict(n_steps=65), "n_steps"),
    (dict(max_rung=8), "max_rung"),
    (dict(flags=2), "flags"),
    (dict(eps=-1.0), "eps"),
    (dict(eps=0.0), "eq. rung"),
    (dict(eta=0.0), "eq. rung"),
    (dict(vel=None), "required"),
    (dict(rung=None), "required"),
    (dict(vel=ctypes.c_void_p(12)), "aligned"),
    (dict(), "NULL handle"),
])
def test_kdk_invalid_arguments_are_rejected(lib, kw, msg):
    args = dict(h=None, pos=ctypes.c_void_p(8), vel=ctypes.c_void_p(8), mass=None,
                rung=ctypes.c_void_p(8), n=10, box=1.0, x_s=0.01, r_cut=0.045, n_grid=64,
                dt=0.01, n_steps=1, eta=0.025, eps=1e-3, max_rung=7, flags=0, prec=0,
                stream=None)
    args.update(kw)
    rc = lib.p3m_kdk_step(*args.values())
    assert rc == -1
    assert msg in lib.p3m_sr_last_error().decode()


@pytest.mark.parametrize("kw, msg", [
    (dict(n=-1), "n must be"),
    (dict(r_cut=0.6), "box/2"),
    (dict(x_s=0.005), "4.5 x_s"),
    (dict(prec=5), "precision"),
    (dict(n_grid=48), "n_grid"),
    (dict(n_grid=2048), "n_grid"),
    (dict(pos=None), "required"),
    (dict(out=ctypes.c_void_p(20)), "aligned"),
    (dict(), "NULL handle"),
])
def test_p3m_force_invalid_arguments_are_rejected(lib, kw, msg):
    args = dict(h=None, pos=ctypes.c_void_p(8), mass=None, active=None, n=10, box=1.0,
                x_s=0.01, r_cut=0.045, n_grid=64, prec=1, out=ctypes.c_void_p(8), stream=None)
    args.update(kw)
    rc = lib.p3m_force(*args.values())
    assert rc == (-4 if "4.5" in msg else -1)
    assert msg in lib.p3m_sr_last_error().decode()


def test_r_cut_beyond_fitted_range_is_unsupported(lib):
    rc = _force(lib, x_s=0.005, r_cut=0.045)            # 9 x_s
    assert rc == -4
    assert "4.5 x_s" in lib.p3m_sr_last_error().decode()


@pytest.mark.parametrize("kind, size, msg", [(3, 0, "unknown shape"), (1, 100, "power of two"),
                                             (1, 8192, "power of two"), (2, 4096, "power of two"),
                                             (2, 32, "power of two"), (0, 0, "NULL handle"),
                                             (1, 0, "NULL handle")])
def test_shape_arguments(lib, kind, size, msg):
    assert lib.p3m_sr_set_shape(None, kind, size) == -1
    assert msg in lib.p3m_sr_last_error().decode()


@pytest.mark.parametrize("level", [0, 3, 4, 8, 12, -1])
def test_autotune_level_is_checked(lib, level):
    rc = lib.p3m_sr_autotune(None, ctypes.c_void_p(8), None, None, 10, 1.0, 0.01, 0.045, 1,
                             level, ctypes.c_void_p(8), None)
    assert rc == -1
    assert "level" in lib.p3m_sr_last_error().decode()


@pytest.mark.parametrize("level", [0, 3, 4 | 8, -1])
def test_batched_autotune_arguments_are_checked(lib, level):
    thr = ctypes.create_string_buffer(b"\x00\x01", 2)
    rc = lib.p3m_sr_autotune_batched(None, ctypes.c_void_p(8), None, ctypes.c_void_p(8), 10, 2,
                                     ctypes.cast(thr, ctypes.c_void_p), 1.0, 0.01, 0.045, 1,
                                     level, ctypes.c_void_p(8), None)
    assert rc == -1 and "level" in lib.p3m_sr_last_error().decode()
    # subset count, thresholds and pointers are checked before the handle
    rc = lib.p3m_sr_autotune_batched(None, ctypes.c_void_p(8), None, ctypes.c_void_p(8), 10, 0,
                                     ctypes.cast(thr, ctypes.c_void_p), 1.0, 0.01, 0.045, 1, 1,
                                     ctypes.c_void_p(8), None)
    assert rc == -1 and "n_sub" in lib.p3m_sr_last_error().decode()
    rc = lib.p3m_sr_autotune_batched(None, ctypes.c_void_p(8), None, ctypes.c_void_p(8), 10, 2,
                                     None, 1.0, 0.01, 0.045, 1, 1, ctypes.c_void_p(8), None)
    assert rc == -1 and "min_rung" in lib.p3m_sr_last_error().decode()
    rc = lib.p3m_sr_autotune_batched(None, ctypes.c_void_p(9), None, ctypes.c_void_p(8), 10, 2,
                                     ctypes.cast(thr, ctypes.c_void_p), 1.0, 0.01, 0.045, 1, 1,
                                     ctypes.c_void_p(8), None)
    assert rc == -1 and "aligned" in lib.p3m_sr_last_error().decode()


def test_autotune_checks_alignment(lib):
    rc = lib.p3m_sr_autotune(None, ctypes.c_void_p(8), None, None, 10, 1.0, 0.01, 0.045, 1, 1,
                             ctypes.c_void_p(12), None)
    assert rc == -1 and "aligned" in lib.p3m_sr_last_error().decode()


def test_tune_cache_calls_need_a_handle(lib):
    assert lib.p3m_sr_set_tune_cache(None, b"/tmp/x.json") == -1
    t, c = ctypes.c_int(5), ctypes.c_int(5)
    assert lib.p3m_sr_tune_status(None, ctypes.byref(t), ctypes.byref(c)) == -1


def test_noalloc_checks_arguments_before_the_handle(lib):
    out = ctypes.c_void_p(8)
    # n beyond the fixed workspace's limit
    rc = lib.p3m_sr_force_noalloc(None, ctypes.c_void_p(8), None, None, (1 << 18) + 1, 1.0,
                                  0.01, 0.045, 1, out, None)
    assert rc == -4 and "no-alloc" in lib.p3m_sr_last_error().decode()
    rc = lib.p3m_sr_force_noalloc(None, ctypes.c_void_p(8), None, None, 100, 1.0, 0.01, 0.045, 7,
                                  out, None)
    assert rc == -1


def test_deterministic_and_debug_limit_arguments(lib):
    assert lib.p3m_sr_set_deterministic(None, 2) == -1
    assert "0 or 1" in lib.p3m_sr_last_error().decode()
    assert lib.p3m_sr_set_deterministic(None, 1) == -1
    assert "NULL handle" in lib.p3m_sr_last_error().decode()
    assert lib.p3m_sr_set_debug_limits(None, -5, -1) == -1
    assert "max_workspace_bytes" in lib.p3m_sr_last_error().decode()
    assert lib.p3m_sr_set_debug_limits(None, 0, -2) == -1
    assert "fail_after" in lib.p3m_sr_last_error().decode()
    assert lib.p3m_sr_set_debug_limits(None, 1 << 20, 3) == -1
    assert "NULL handle" in lib.p3m_sr_last_error().decode()
