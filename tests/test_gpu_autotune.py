"""The measure-and-keep autotuner (section 2.1.3, "Subtiles": try a finer
subdivision, time it, keep it if faster) through the C ABI: after tuning the
forward, and then the adjoint on its own, both calls run in the stored
layouts and still match the oracle."""
import json

import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload

pytestmark = pytest.mark.gpu

LAYOUT = ("subtiles_per_dim", "item_target", "cluster_size", "screen")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotuned_forward_and_adjoint(prec):
    print("autotune diff64 n_side=32", prec, flush=True)
    torch, p3 = gpu_or_skip()
    ctx = p3.Context(0)
    wl = make_workload("diff64", n_side=32)
    rng = np.random.default_rng(21)
    mass = rng.uniform(0.5, 2.0, wl.n)
    w = rng.standard_normal((wl.n, 3))
    pos, m = to_dev(torch, wl.pos), to_dev(torch, mass)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision=prec)

    ctx.autotune(pos, m, None, level=2, **kw)
    acc = ctx.force(pos, m, None, **kw)
    fwd = {k: ctx.stats()[k] for k in LAYOUT}
    ref, cnt, absum = oracle.force_full(wl.pos, mass, 1.0, wl.x_s, wl.r_cut)
    e = oracle.errors(acc.cpu().numpy(), ref, absum)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    assert ctx.stats()["interactions"] == int(cnt.sum())

    # the adjoint takes the forward's layout until it is tuned on its own
    # (screen 2 included: the adjoint also pairs once for both partners)
    ctx.force_backward(pos, m, None, to_dev(torch, w), **kw)
    assert {k: ctx.stats()[k] for k in LAYOUT} == fwd
    ctx.autotune(pos, m, None, level=1, adjoint=True, **kw)
    g = ctx.force_backward(pos, m, None, to_dev(torch, w), **kw).cpu().numpy()
    adj = {k: ctx.stats()[k] for k in LAYOUT}
    g_ref = oracle.vjp(wl.pos, mass, None, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print("forward layout", fwd, "adjoint layout", adj, "vjp rel", rel, flush=True)
    assert rel <= (1e-12 if prec == "fp64" else 1e-5)
    # tuning the adjoint leaves the forward's layout alone
    ctx.force(pos, m, None, **kw)
    assert {k: ctx.stats()[k] for k in LAYOUT} == fwd
    ctx.close()


def test_batched_autotune_uses_its_own_subsets(tmp_path):
    """The rung-batched call tuned on its own subsets (8 nested rung
    thresholds of a reduced clustered256 set) runs in the tuned layout and
    still matches the oracle on receivers stratified by rung."""
    torch, p3 = gpu_or_skip()
    ctx = p3.Context(0)
    ctx.set_tune_cache(str(tmp_path / "tune.json"))
    wl = make_workload("clustered256", n_side=64, with_rungs=True)
    thr = list(range(8))
    pos, rung = to_dev(torch, wl.pos), to_dev(torch, wl.rung)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    ctx.autotune_batched(pos, None, rung, thr, **kw)
    st = ctx.tune_status()
    assert st["trials"] > 0 and not st["from_cache"]
    out = ctx.force_batched(pos, None, rung, thr, **kw).cpu().numpy()
    lay = {k: ctx.stats()[k] for k in LAYOUT}
    print("batched layout", lay, flush=True)
    assert lay["screen"] in (0, 1) and lay["item_target"] in (1024, 4096, 16384)
    from workloads import stratified_by_rung
    idx = stratified_by_rung(wl.rung, 64, wl.config_id)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx)
    for k in thr:
        sel = wl.rung[idx] >= k
        got = out[k][idx[sel]]
        e = oracle.errors(got, ref[sel], absum[sel])
        assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], (k, e)
        assert np.all(out[k][wl.rung < k] == 0)
    ctx.close()


def test_cache_persists_across_handles(tmp_path):
    """A second handle reading the same cache file reuses the first one's
    tuned layouts (forward and batched) without timing, and calls run in
    them; P3M_TUNE_FORCE times again."""
    torch, p3 = gpu_or_skip()
    path = str(tmp_path / "tune.json")
    wl = make_workload("diff64", n_side=32, with_rungs=False)
    rung = (np.arange(wl.n) % 4).astype(np.uint8)
    pos, rg = to_dev(torch, wl.pos), to_dev(torch, rung)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    a = p3.Context(0)
    a.set_tune_cache(path)
    a.autotune(pos, None, None, level=1, **kw)
    assert a.tune_status()["trials"] > 0
    a.force(pos, None, None, **kw)
    lay_a = {k: a.stats()[k] for k in LAYOUT}
    a.autotune_batched(pos, None, rg, [0, 1, 2, 3], **kw)
    a.force_batched(pos, None, rg, [0, 1, 2, 3], **kw)
    lay_ab = {k: a.stats()[k] for k in LAYOUT}
    a.close()
    kinds = sorted(e["kind"] for e in json.load(open(path)))
    # the forward and the batched results (and, when the forward's winner
    # pairs once for both partners, the layout kept for the other calls)
    assert kinds in ([0, 2], [0, 2, 3]), kinds
    b = p3.Context(0)
    b.set_tune_cache(path)
    # the loaded layouts apply to calls right away
    b.force(pos, None, None, **kw)
    assert {k: b.stats()[k] for k in LAYOUT} == lay_a
    b.autotune(pos, None, None, level=1, **kw)
    assert b.tune_status() == {"trials": 0, "from_cache": True}
    b.autotune_batched(pos, None, rg, [0, 1, 2, 3], **kw)
    assert b.tune_status() == {"trials": 0, "from_cache": True}
    b.force_batched(pos, None, rg, [0, 1, 2, 3], **kw)
    assert {k: b.stats()[k] for k in LAYOUT} == lay_ab
    # a different particle set of the same size does not match the signature
    other = np.random.default_rng(3).random((wl.n, 3))
    b.autotune(to_dev(torch, other), None, None, level=1, **kw)
    assert b.tune_status()["trials"] > 0
    b.autotune(pos, None, None, level=1, force=True, **kw)
    assert b.tune_status()["trials"] > 0
    b.close()


def test_calls_the_mutual_layout_cannot_serve_take_the_kept_one(tmp_path):
    """On the clustered128 recipe (reduced) the FP32 forward's winner is
    normally the mutual layout (screen 2); the tuner then also keeps the
    fastest of the other layouts (kind 3 in the cache), and calls that cannot
    pair once for both partners (masked, deterministic, softened adjoint) run
    in it, while all-active forward calls, softened or not, keep the winner.
    The masked and deterministic calls still match the oracle."""
    torch, p3 = gpu_or_skip()
    path = str(tmp_path / "tune.json")
    wl = make_workload("clustered128", n_side=64)
    print("autotune plain layout clustered128 n_side=64", flush=True)
    kw = dict(box=1.0, x_s=wl.x_s, r_cut=wl.r_cut, precision="fp32")
    ctx = p3.Context(0)
    try:
        ctx.set_tune_cache(path)
        pos = to_dev(torch, wl.pos)
        ctx.autotune(pos, None, None, level=1, **kw)
        ents = {e["kind"]: e for e in json.load(open(path))}
        win = tuple(ents[0][k] for k in ("ns", "target", "csize", "screen"))
        ctx.force(pos, None, None, **kw)
        lay = lambda: tuple(ctx.stats()[k] for k in LAYOUT)
        assert lay() == win
        print("winner", win, "kinds", sorted(ents), flush=True)
        if win[3] != 2:
            assert 3 not in ents
            pytest.skip("the winner is not the mutual layout on this device")
        plain = tuple(ents[3][k] for k in ("ns", "target", "csize", "screen"))
        assert plain[3] in (0, 1)
        idx = np.arange(0, wl.n, 997)
        ref, _, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx)
        # an active mask
        act = np.zeros(wl.n, dtype=np.uint8)
        act[idx] = 1
        out = ctx.force(pos, None, to_dev(torch, act), **kw).cpu().numpy()
        assert lay() == plain
        e = oracle.errors(out[idx], ref, absum)
        assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], e
        # the deterministic mode
        ctx.set_deterministic(True)
        out = ctx.force(pos, None, None, **kw).cpu().numpy()
        assert lay() == plain
        e = oracle.errors(out[idx], ref, absum)
        assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], e
        ctx.set_deterministic(False)
        # softening: the forward stays on the winner, the adjoint (no
        # softened mutual kernel) takes the kept layout
        ctx.set_softening(1e-4)
        try:
            ctx.force(pos, None, None, **kw)
            assert lay() == win
            ones = torch.ones((wl.n, 3), dtype=torch.float64, device=pos.device)
            ctx.force_backward(pos, None, None, ones, **kw)
            assert lay() == plain
        finally:
            ctx.set_softening(0.0)
        ctx.force(pos, None, None, **kw)
        assert lay() == win
        # a second handle installs both from the cache without timing
        b = p3.Context(0)
        try:
            b.set_tune_cache(path)
            b.autotune(pos, None, None, level=1, **kw)
            assert b.tune_status() == {"trials": 0, "from_cache": True}
            b.force(pos, None, to_dev(torch, act), **kw)
            assert tuple(b.stats()[k] for k in LAYOUT) == plain
        finally:
            b.close()
    finally:
        ctx.close()
