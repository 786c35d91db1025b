"""GPU forward force in FP64 with each pair evaluated once for both partners
(layout screen = 2 on an all-active FP64 call without softening: FP64
offsets from the cluster centre, the reaction sent back along the
wavefront's rows) vs the FP64 CPU oracle, through the C ABI.

Bars as for every FP64 path: e_L2 and e_max_cond <= 1e-12 and the exact
accepted-pair count of the oracle (pairs whose squared distance lies within a
relative 2^-40 of r_cut^2, or closer than a tenth of the receiver's offset
from the cluster centre, are evaluated in the plain form).  The FP64 adjoint
takes the same layout (rows against the oracle's VJP to 1e-12), and so do
softened forward calls; softened FP64 adjoints keep the screened kernel.
"""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from test_gpu_mutual import close_pairs_set
from workloads import lattice_sites, make_workload, random_particles, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def run(env, pos, mass, box, x_s, r_cut, csize, **cfg):
    torch, p3, ctx = env
    ctx.set_config(cluster_size=csize, screen=2, **cfg)
    try:
        acc = ctx.force(to_dev(torch, pos), to_dev(torch, mass), None, box=box, x_s=x_s,
                        r_cut=r_cut, precision="fp64")
        torch.cuda.synchronize()
        st = ctx.stats()
        assert st["screen"] == 2 and st["cluster_size"] == csize
        return acc.cpu().numpy(), st
    finally:
        ctx.set_config()


def check(acc, st, ref, cnt, absum):
    e = oracle.errors(acc, ref, absum)
    assert st["interactions"] == int(cnt.sum()), (st["interactions"], int(cnt.sum()))
    assert e["e_l2"] <= TOL["fp64"] and e["e_max_cond"] <= TOL["fp64"], e
    return e


@pytest.mark.parametrize("csize", [16, 32, 64])
@pytest.mark.parametrize("ns", [1, 2])
@pytest.mark.parametrize("masses", [False, True])
def test_diff64_small_layouts(env, csize, ns, masses):
    print("fp64 mutual diff64 n_side=24 csize", csize, "ns", ns, "masses", masses, flush=True)
    wl = make_workload("diff64", n_side=24)
    mass = np.random.default_rng(5).uniform(0.5, 2.0, wl.n) if masses else None
    ref, cnt, absum = oracle.force_full(wl.pos, mass, 1.0, wl.x_s, wl.r_cut, method="tiled")
    for target in (64, 4096):
        acc, st = run(env, wl.pos, mass, 1.0, wl.x_s, wl.r_cut, csize, subtiles_per_dim=ns,
                      item_target=target)
        check(acc, st, ref, cnt, absum)


@pytest.mark.parametrize("n", [1, 2, 17, 63, 1000])
@pytest.mark.parametrize("csize", [16, 32, 64])
def test_ragged(env, n, csize):
    print("fp64 mutual random n=%d csize=%d" % (n, csize), flush=True)
    pos, mass, _ = random_particles(n, seed=300 + n)
    if n <= 2:
        pos[:] = [0.5, 0.5, 0.5]
        pos[-1] = [0.52, 0.49, 0.5]
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    for m in (mass, None):
        ref, cnt, absum = oracle.force_full(pos, m, 1.0, x_s, r_cut, method="brute")
        acc, st = run(env, pos, m, 1.0, x_s, r_cut, csize)
        check(acc, st, ref, cnt, absum)


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_lattice_pairs_on_the_cutoff(env, csize):
    """Lattice sites with pairs exactly on r_cut (rejected), coincident
    distinct particles and coordinates of exactly 1.0."""
    print("fp64 mutual lattice csize", csize, flush=True)
    n_side, k = 64, 4
    pos, _ = lattice_sites(n_side, 6000, 300, 60, seed=11)
    mass = np.random.default_rng(12).uniform(0.5, 2.0, pos.shape[0])
    r_cut = k / n_side
    x_s = r_cut / 4.5
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute")
    acc, st = run(env, pos, mass, 1.0, x_s, r_cut, csize)
    check(acc, st, ref, cnt, absum)


def test_close_pairs_and_cutoff_band(env):
    print("fp64 mutual close pairs", flush=True)
    pos, x_s, r_cut = close_pairs_set(21)
    ref, cnt, absum = oracle.force_full(pos, None, 1.0, x_s, r_cut, method="brute")
    acc, st = run(env, pos, None, 1.0, x_s, r_cut, 32)
    e = check(acc, st, ref, cnt, absum)
    print(e, "plain-form steps", st["fp64_steps"], flush=True)
    assert st["fp64_steps"] > 0


def test_newtons_third_law(env):
    """Each pair's action and reaction are the same FP64 value."""
    wl = make_workload("diff64", n_side=32)
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, 32)
    tot = np.abs(acc.sum(axis=0))
    assert np.all(tot <= 1e-13 * np.abs(acc).sum(axis=0)), tot


@pytest.mark.parametrize("csize", [16, 32])
def test_clustered128_65536_receivers(env, csize):
    """Full-size N = 128^3 clustered set: 65536 seeded receivers against the
    oracle over all N."""
    print("fp64 mutual clustered128 csize", csize, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, csize, subtiles_per_dim=1,
                  item_target=4096)
    idx = sample_indices(wl.n, 65536, wl.config_id, salt=1)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled")
    e = oracle.errors(acc[idx], ref, absum)
    print(e, "interactions", st["interactions"], flush=True)
    assert e["e_l2"] <= TOL["fp64"] and e["e_max_cond"] <= TOL["fp64"], e
    assert 1.0e9 < st["interactions"] < 2.5e9


def test_clustered128_pair_count_exact(env):
    wl = make_workload("clustered128", with_rungs=False)
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, 16, subtiles_per_dim=1,
                  item_target=4096)
    _, cnt, _ = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, method="tiled")
    assert st["interactions"] == int(cnt.sum())


@pytest.mark.parametrize("csize", [16, 32, 64])
@pytest.mark.parametrize("masses", [False, True])
def test_adjoint_pairs_once(env, csize, masses):
    """The FP64 adjoint in the same layout: every row against the oracle's
    analytic VJP, with half the particles active (activity enters through
    the weights)."""
    torch, p3, ctx = env
    print("fp64 mutual adjoint csize", csize, "masses", masses, flush=True)
    wl = make_workload("diff64", n_side=24)
    rng = np.random.default_rng(13)
    mass = rng.uniform(0.5, 2.0, wl.n) if masses else None
    active = (rng.random(wl.n) < 0.5).astype(np.uint8)
    w = rng.standard_normal((wl.n, 3))
    ref = oracle.vjp(wl.pos, mass, active, w, 1.0, wl.x_s, wl.r_cut, method="tiled")
    ctx.set_config(cluster_size=csize, screen=2)
    try:
        g = ctx.force_backward(to_dev(torch, wl.pos), to_dev(torch, mass), to_dev(torch, active),
                               to_dev(torch, w), box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                               precision="fp64").cpu().numpy()
        st = ctx.stats()
    finally:
        ctx.set_config()
    assert st["screen"] == 2 and st["cluster_size"] == csize
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    row = np.max(np.linalg.norm(g - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1))
    assert rel <= 1e-12 and row <= 1e-12, (rel, row)


@pytest.mark.parametrize("csize", [16, 32])
def test_softened_forward_pairs_once(env, csize):
    """A softened all-active FP64 forward call stays in the layout (pairs
    inside eps_B take the softened factor); a softened FP64 adjoint takes the
    screened kernel."""
    torch, p3, ctx = env
    print("fp64 mutual softened csize", csize, flush=True)
    pos, mass, _ = random_particles(3000, seed=9)
    pos[:40] = 0.5 + 1e-3 * np.random.default_rng(2).standard_normal((40, 3))
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    w = np.random.default_rng(4).standard_normal((3000, 3))
    ctx.set_config(cluster_size=csize, screen=2)
    ctx.set_softening(0.002)
    try:
        acc = ctx.force(to_dev(torch, pos), to_dev(torch, mass), None, box=1.0, x_s=x_s,
                        r_cut=r_cut, precision="fp64").cpu().numpy()
        st = ctx.stats()
        assert st["screen"] == 2
        ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute",
                                            eps=0.002)
        plain, _, _ = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute")
        # the softening changes the force noticeably on this set
        assert np.max(np.linalg.norm(ref - plain, axis=1) / np.maximum(absum, 1e-300)) > 1e-3
        check(acc, st, ref, cnt, absum)
        ctx.force_backward(to_dev(torch, pos), to_dev(torch, mass), None, to_dev(torch, w),
                           box=1.0, x_s=x_s, r_cut=r_cut, precision="fp64")
        assert ctx.stats()["screen"] == 1
    finally:
        ctx.set_softening(0.0)
        ctx.set_config()
