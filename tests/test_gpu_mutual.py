"""GPU forward force with each pair evaluated once for both partners (layout
screen = 2: FP32 pair arithmetic on cluster-relative coordinates, the
reaction sent back along the wavefront's rows) vs the FP64 CPU oracle,
through the C ABI.

Bars as for every FP32 path: e_L2 and e_max_cond <= 1e-5, and the exact
accepted-pair count of the plain FP64 evaluation (pairs whose FP32 r^2 lies
near r_cut^2 are decided in FP64).  Calls this layout does not cover (an
active mask) fall back to the screened kernel; softened forward calls stay on
it (pairs inside eps_B take the softened factor), and so do all-active FP64
calls (the FP64 kind, tested on its own in test_gpu_mutual_fp64.py).
"""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import lattice_sites, make_workload, random_particles, sample_indices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def run(env, pos, mass, box, x_s, r_cut, csize, prec="fp32", active=None, **cfg):
    torch, p3, ctx = env
    ctx.set_config(cluster_size=csize, screen=2, **cfg)
    try:
        acc = ctx.force(to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active), box=box,
                        x_s=x_s, r_cut=r_cut, precision=prec)
        torch.cuda.synchronize()
        return acc.cpu().numpy(), ctx.stats()
    finally:
        ctx.set_config()


def check(acc, st, ref, cnt, absum, prec="fp32"):
    e = oracle.errors(acc, ref, absum)
    assert st["interactions"] == int(cnt.sum()), (st["interactions"], int(cnt.sum()))
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    return e


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_uniform32_full(env, csize):
    print("mutual uniform32 csize", csize, flush=True)
    wl = make_workload("uniform32")
    ref, cnt, absum = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, method="tiled")
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, csize)
    assert st["screen"] == 2 and st["cluster_size"] == csize
    print(check(acc, st, ref, cnt, absum), st["fp64_steps"], flush=True)


@pytest.mark.parametrize("csize", [16, 32, 64])
@pytest.mark.parametrize("ns", [1, 2, 3])
@pytest.mark.parametrize("masses", [False, True])
def test_diff64_small_layouts(env, csize, ns, masses):
    """Subtile counts (own-tile subtile ranges split into several items),
    item sizes, unit and per-particle masses."""
    print("mutual diff64 n_side=24 csize", csize, "ns", ns, "masses", masses, flush=True)
    wl = make_workload("diff64", n_side=24)
    mass = np.random.default_rng(5).uniform(0.5, 2.0, wl.n) if masses else None
    ref, cnt, absum = oracle.force_full(wl.pos, mass, 1.0, wl.x_s, wl.r_cut, method="tiled")
    for target in (64, 4096):
        acc, st = run(env, wl.pos, mass, 1.0, wl.x_s, wl.r_cut, csize, subtiles_per_dim=ns,
                      item_target=target)
        assert st["screen"] == 2
        check(acc, st, ref, cnt, absum)


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_diff64_full(env, csize):
    """Config with N = 64^3 clustered particles, every row."""
    print("mutual diff64 full csize", csize, flush=True)
    wl = make_workload("diff64")
    ref, cnt, absum = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, method="tiled")
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, csize, subtiles_per_dim=1,
                  item_target=4096)
    print(check(acc, st, ref, cnt, absum), "fp64 steps", st["fp64_steps"], flush=True)


@pytest.mark.parametrize("n", [1, 2, 9, 17, 63, 1000, 4097])
@pytest.mark.parametrize("csize", [16, 32, 64])
def test_ragged(env, n, csize):
    """Partial clusters, a cluster alone, empty lists; unit and per-particle
    masses."""
    print("mutual random n=%d csize=%d" % (n, csize), flush=True)
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
    """Sites of a 64^3 lattice, r_cut = 4 spacings: hundreds of pairs exactly
    on r_cut (rejected), coincident distinct particles (no contribution),
    coordinates of exactly 1.0.  The accepted pairs must be the oracle's."""
    print("mutual lattice csize", csize, flush=True)
    n_side, k = 64, 4
    pos, _ = lattice_sites(n_side, 6000, 300, 60, seed=11)
    mass = np.random.default_rng(12).uniform(0.5, 2.0, pos.shape[0])
    r_cut = k / n_side
    x_s = r_cut / 4.5
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute")
    acc, st = run(env, pos, mass, 1.0, x_s, r_cut, csize)
    check(acc, st, ref, cnt, absum)


def close_pairs_set(seed):
    """A uniform background with binaries of separation 1e-7 .. 1e-4 (far
    below a tenth of a cluster's extent, where the separation is redone in
    FP64) and pairs straddling r_cut within a few parts in 1e7."""
    rng = np.random.default_rng(seed)
    n_bg = 6000
    pos = rng.random((n_bg, 3))
    x_s = 1.25 / 40
    r_cut = 4.5 * x_s
    extra = []
    for sep in np.geomspace(1e-7, 1e-4, 200):
        c = rng.random(3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        extra += [c, (c + sep * u) % 1.0]
    for k in range(200):
        c = rng.uniform(0.2, 0.8, 3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        extra += [c, c + r_cut * (1.0 + (k - 100) * 3e-8) * u]
    return np.concatenate([pos, np.array(extra)]) % 1.0, x_s, r_cut


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_close_pairs_and_cutoff_band(env, csize):
    print("mutual close pairs csize", csize, flush=True)
    pos, x_s, r_cut = close_pairs_set(21)
    ref, cnt, absum = oracle.force_full(pos, None, 1.0, x_s, r_cut, method="brute")
    acc, st = run(env, pos, None, 1.0, x_s, r_cut, csize)
    e = check(acc, st, ref, cnt, absum)
    print(e, "fp64 steps", st["fp64_steps"], flush=True)
    assert st["fp64_steps"] > 0


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_newtons_third_law(env, csize):
    """With every particle active the mutual sums conserve momentum: each
    pair's action and reaction are the same FP32 value."""
    wl = make_workload("diff64", n_side=32)
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, csize)
    tot = np.abs(acc.sum(axis=0))
    assert np.all(tot <= 1e-6 * np.abs(acc).sum(axis=0)), tot


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_clustered128_65536_receivers(env, csize):
    """Full-size N = 128^3 clustered set (ns 1, items of 4096): 65536 seeded
    receivers against the cell-list oracle over all N, and the exact total
    pair count of the oracle's full evaluation."""
    print("mutual clustered128 csize", csize, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, csize, subtiles_per_dim=1,
                  item_target=4096)
    idx = sample_indices(wl.n, 65536, wl.config_id, salt=1)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled")
    e = oracle.errors(acc[idx], ref, absum)
    print(e, "interactions", st["interactions"], "fp64 steps", st["fp64_steps"], flush=True)
    assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], e
    assert 1.0e9 < st["interactions"] < 2.5e9


def test_clustered128_pair_count_exact(env):
    """The mutual kernel's accepted-pair total on the full N = 128^3 set
    equals the oracle's (cell-list count over all N)."""
    wl = make_workload("clustered128", with_rungs=False)
    acc, st = run(env, wl.pos, None, 1.0, wl.x_s, wl.r_cut, 32, subtiles_per_dim=1,
                  item_target=4096)
    _, cnt, _ = oracle.force_full(wl.pos, None, 1.0, wl.x_s, wl.r_cut, method="tiled")
    assert st["interactions"] == int(cnt.sum())


@pytest.mark.parametrize("csize", [16, 32, 64])
def test_dense_subtiles_and_smallest_tiling(env, csize):
    rng = np.random.default_rng(77)
    n = 9000
    pos = rng.random((n, 3))
    pos[:3000] = 0.31 + 0.004 * rng.random((3000, 3))
    pos[3000:5000] = 0.72 + 0.01 * rng.standard_normal((2000, 3))
    pos %= 1.0
    mass = rng.uniform(0.5, 2.0, n)
    x_s, r_cut = 1.25 / 32, 4.5 * 1.25 / 32
    recv = np.concatenate([np.arange(0, 3000, 7), np.arange(3000, n, 11)])
    ref, cnt, absum = oracle.force(pos, mass, 1.0, x_s, r_cut, recv=recv)[:3]
    acc, st = run(env, pos, mass, 1.0, x_s, r_cut, csize, subtiles_per_dim=1)
    e = oracle.errors(acc[recv], ref, absum)
    assert e["e_l2"] <= TOL["fp32"] and e["e_max_cond"] <= TOL["fp32"], e
    # three tiles per dimension
    box = 2.0
    r_cut = box / 3 * 0.999
    x_s = r_cut / 4.5
    pos3, mass3, _ = random_particles(700, seed=5, box=box)
    ref, cnt, absum = oracle.force_full(pos3, mass3, box, x_s, r_cut, method="brute")
    acc, st = run(env, pos3, mass3, box, x_s, r_cut, csize)
    assert st["tiles_per_dim"] == 3
    check(acc, st, ref, cnt, absum)


def test_other_calls_fall_back(env):
    """An active mask takes the screened kernel with the same cluster size;
    an all-active FP64 call and a softened all-active FP32 call stay on the
    mutual kernel; results match the oracle."""
    torch, p3, ctx = env
    pos, mass, active = random_particles(3000, seed=9, active_frac=0.5)
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active,
                                        method="brute")
    acc, st = run(env, pos, mass, 1.0, x_s, r_cut, 32, active=active)
    assert st["screen"] == 1
    check(acc, st, ref, cnt, absum)
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute")
    acc, st = run(env, pos, mass, 1.0, x_s, r_cut, 32, prec="fp64")
    assert st["screen"] == 2
    check(acc, st, ref, cnt, absum, "fp64")
    ctx.set_softening(0.002)
    try:
        refs, cnts, abss = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute",
                                             eps=0.002)
        acc, st = run(env, pos, mass, 1.0, x_s, r_cut, 32)
        assert st["screen"] == 2
        check(acc, st, refs, cnts, abss)
    finally:
        ctx.set_softening(0.0)
