"""Deterministic mode (p3m_sr_set_deterministic): the same bits call after
call for forward, adjoint and rung-batched calls, the same accepted pairs
as the atomic mode, forces within rounding of the atomic mode's and within
the bars of the FP64 oracle; and the debug limits that force P3M_ENOMEM
(p3m_sr_set_debug_limits), after which the handle still works."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def with_duplicates(pos, n_dup, seed):
    """pos with n_dup extra particles placed exactly on existing ones (equal
    cell and fine keys: only the index can order them)."""
    rng = np.random.default_rng(seed)
    src = rng.choice(pos.shape[0], size=n_dup, replace=False)
    return np.concatenate([pos, pos[src]])


def same_bits(a, b):
    return a.dtype == b.dtype and a.shape == b.shape and a.tobytes() == b.tobytes()


LAYOUTS = [dict(item_target=256, cluster_size=32, screen=1),
           dict(item_target=1024, cluster_size=16, screen=0),
           dict(item_target=256, cluster_size=64, screen=1, subtiles_per_dim=2)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forward_bitwise_and_against_atomic_mode(env, prec, layout):
    torch, p3, ctx = env
    print("deterministic forward diff64 n_side=32 + duplicates", prec, layout, flush=True)
    wl = make_workload("diff64", n_side=32)
    pos = with_duplicates(wl.pos, 500, 5)
    d = to_dev(torch, pos)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    ctx.set_config(**layout)
    try:
        ctx.set_deterministic(True)
        runs = []
        for _ in range(3):
            runs.append(ctx.force(d, None, None, **kw).cpu().numpy())
            st = ctx.stats()
        ctx.set_deterministic(False)
        atomic = ctx.force(d, None, None, **kw).cpu().numpy()
        st_a = ctx.stats()
    finally:
        ctx.set_deterministic(False)
        ctx.set_config()
    assert st["deterministic"] == 1 and st_a["deterministic"] == 0
    # the small item target splits clusters into several items
    assert st["items"] > st["clusters"]
    assert st["interactions"] == st_a["interactions"]
    for r in runs[1:]:
        assert same_bits(runs[0], r)
    scale = np.max(np.abs(atomic))
    assert np.max(np.abs(runs[0] - atomic)) <= 1e-12 * scale
    idx = sample_indices(pos.shape[0], 400, 17)
    ref, cnt, absum, _ = oracle.force(pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx)
    e = oracle.errors(runs[0][idx], ref, absum)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e


def test_screen2_runs_as_screen1(env):
    """Layout screen 2 (pairs evaluated for both partners, reactions by
    atomics) is not used in the deterministic mode."""
    torch, p3, ctx = env
    wl = make_workload("diff64", n_side=24)
    d = to_dev(torch, wl.pos)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    ctx.set_config(cluster_size=32, screen=2)
    try:
        ctx.set_deterministic(True)
        a = ctx.force(d, None, None, **kw).cpu().numpy()
        st = ctx.stats()
        b = ctx.force(d, None, None, **kw).cpu().numpy()
    finally:
        ctx.set_deterministic(False)
        ctx.set_config()
    assert st["screen"] == 1 and st["deterministic"] == 1
    assert same_bits(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_bitwise(env, prec):
    torch, p3, ctx = env
    print("deterministic adjoint diff64 n_side=32", prec, flush=True)
    wl = make_workload("diff64", n_side=32)
    rng = np.random.default_rng(8)
    active = (rng.random(wl.n) < 0.6).astype(np.uint8)
    w = rng.standard_normal((wl.n, 3))
    d, a_d, w_d = to_dev(torch, wl.pos), to_dev(torch, active), to_dev(torch, w)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    ctx.set_config(item_target=256)
    try:
        ctx.set_deterministic(True)
        g1 = ctx.force_backward(d, None, a_d, w_d, **kw).cpu().numpy()
        g2 = ctx.force_backward(d, None, a_d, w_d, **kw).cpu().numpy()
        st = ctx.stats()
        ctx.set_deterministic(False)
        ga = ctx.force_backward(d, None, a_d, w_d, **kw).cpu().numpy()
    finally:
        ctx.set_deterministic(False)
        ctx.set_config()
    assert st["deterministic"] == 1 and st["items"] > st["clusters"]
    assert same_bits(g1, g2)
    assert np.max(np.abs(g1 - ga)) <= 1e-12 * np.max(np.abs(ga))
    ref = oracle.vjp(wl.pos, None, active, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    assert np.linalg.norm(g1 - ref) <= {"fp64": 1e-12, "fp32": 1e-5}[prec] * np.linalg.norm(ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_bitwise(env, prec):
    torch, p3, ctx = env
    print("deterministic batched clustered256 recipe n_side=40", prec, flush=True)
    wl = make_workload("clustered256", n_side=40)
    thr = list(range(8))
    pos, rung = to_dev(torch, wl.pos), to_dev(torch, wl.rung)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)
    ctx.set_config(item_target=512)
    try:
        ctx.set_deterministic(True)
        o1 = ctx.force_batched(pos, None, rung, thr, **kw).cpu().numpy()
        o2 = ctx.force_batched(pos, None, rung, thr, **kw).cpu().numpy()
        ctx.set_deterministic(False)
        oa = ctx.force_batched(pos, None, rung, thr, **kw).cpu().numpy()
    finally:
        ctx.set_deterministic(False)
        ctx.set_config()
    assert same_bits(o1, o2)
    assert np.max(np.abs(o1 - oa)) <= 1e-12 * np.max(np.abs(oa))
    for k in (0, 5):
        act = (wl.rung >= k).astype(np.uint8)
        ref, _, absum = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, active=act)
        e = oracle.errors(o1[k][act == 1], ref[act == 1], absum[act == 1])
        assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], (k, e)


def test_clustered128_bitwise_sampled(env):
    """Full-size clustered set (N = 128^3) in the bench's FP32 layout apart
    from screen 2: two deterministic calls agree bit for bit, and sampled
    rows match the oracle."""
    torch, p3, ctx = env
    print("deterministic clustered128 fp32", flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    d = to_dev(torch, wl.pos)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    ctx.set_config(subtiles_per_dim=1, item_target=4096, cluster_size=32, screen=1)
    try:
        ctx.set_deterministic(True)
        a = ctx.force(d, None, None, **kw).cpu().numpy()
        b = ctx.force(d, None, None, **kw).cpu().numpy()
        st = ctx.stats()
    finally:
        ctx.set_deterministic(False)
        ctx.set_config()
    assert st["deterministic"] == 1
    assert same_bits(a, b)
    idx = sample_indices(wl.n, 256, wl.config_id)
    ref, _, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx, method="tiled")
    e = oracle.errors(a[idx], ref, absum)
    assert e["e_max_cond"] <= TOL["fp32"], e


# ---- debug limits -----------------------------------------------------------

def test_debug_byte_limit_forces_enomem(env):
    torch, p3, _ = env
    wl = make_workload("diff64", n_side=32)
    d = to_dev(torch, wl.pos)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp64")
    ref_ctx = p3.Context(0)
    ref = ref_ctx.force(d, None, None, **kw).cpu().numpy()
    ref_ctx.close()
    ctx = p3.Context(0)
    try:
        ctx.set_debug_limits(max_workspace_bytes=1 << 20)
        with pytest.raises(p3.P3MError) as ei:
            ctx.force(d, None, None, **kw)
        assert ei.value.code == p3.P3M_ENOMEM
        ctx.set_debug_limits()
        got = ctx.force(d, None, None, **kw).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    finally:
        ctx.close()


def test_debug_fail_after_each_growth(env):
    """A growth made to fail at each step of a first call's workspace build:
    every call either succeeds or raises P3M_ENOMEM, and the same handle
    gives the normal result once the limit is lifted."""
    torch, p3, _ = env
    wl = make_workload("diff64", n_side=20)
    d = to_dev(torch, wl.pos)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    ref_ctx = p3.Context(0)
    ref = ref_ctx.force(d, None, None, **kw).cpu().numpy()
    ref_ctx.close()
    failed = 0
    for k in range(40):
        ctx = p3.Context(0)
        try:
            ctx.set_debug_limits(fail_after=k)
            try:
                ctx.force(d, None, None, **kw)
                ok = True
            except p3.P3MError as e:
                assert e.code == p3.P3M_ENOMEM, e
                ok = False
                failed += 1
            ctx.set_debug_limits()
            got = ctx.force(d, None, None, **kw).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))
        finally:
            ctx.close()
        if ok:
            break
    assert failed >= 10 and ok
