"""GPU forward force vs the FP64 CPU oracle, through the C ABI.

Bars: FP64 path e_L2 and e_max_cond <= 1e-12 with the exact accepted-pair
count; FP32 path (FP64 separation / cut-off / accumulation, FP32 kernel
shape) e_L2 and e_max_cond <= 1e-5 with the same pair count (both paths
take the cut-off decision on the same FP64 squared distance).
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


def run_force(env, pos, mass, active, box, x_s, r_cut, prec, **cfg):
    torch, p3, ctx = env
    if cfg:
        ctx.set_config(**cfg)
    try:
        acc = ctx.force(to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active),
                        box=box, x_s=x_s, r_cut=r_cut, precision=prec)
        torch.cuda.synchronize()
        return acc.cpu().numpy(), ctx.stats()
    finally:
        if cfg:
            ctx.set_config()


def check(acc, st, ref, cnt, absum, prec, active=None):
    e = oracle.errors(acc, ref, absum)
    assert st["interactions"] == int(cnt.sum()), (st, int(cnt.sum()))
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    if active is not None:
        assert np.all(acc[active == 0] == 0)
    return e


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform32_full(env, prec):
    print("uniform32 N=32^3", prec, flush=True)
    wl = make_workload("uniform32")
    ref, cnt, absum = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, method="tiled")
    acc, st = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, prec)
    e = check(acc, st, ref, cnt, absum, prec)
    assert st["receivers"] == wl.n and st["tiles_per_dim"] == 11
    print(e, flush=True)


@pytest.mark.parametrize("n", [1, 2, 63, 65, 1000, 4097])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_masses_and_mask(env, n, prec):
    print("random n=%d" % n, prec, flush=True)
    pos, mass, active = random_particles(n, seed=100 + n, active_frac=0.6)
    if n <= 2:
        pos[:] = [0.5, 0.5, 0.5]
        pos[-1] = [0.52, 0.49, 0.5]
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active, method="brute")
    acc, st = run_force(env, pos, mass, active, 1.0, x_s, r_cut, prec)
    check(acc, st, ref, cnt, absum, prec, active)


@pytest.mark.parametrize("ns", [1, 2, 3, 4, 5, 7])
@pytest.mark.parametrize("target", [64, 512, 4096])
def test_decompositions_agree(env, ns, target):
    """Every subtile count and item size gives the oracle's force (section
    2.1.3: the (sub)tiling changes only the summation order)."""
    print("clustered n_side=24 ns=%d target=%d" % (ns, target), flush=True)
    wl = make_workload("diff64", n_side=24)
    ref, cnt, absum = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, method="tiled")
    acc, st = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, "fp64",
                        subtiles_per_dim=ns, item_target=target)
    assert st["subtiles_per_dim"] == ns and st["item_target"] == target
    check(acc, st, ref, cnt, absum, "fp64")


LAYOUTS = [(64, 0), (64, 1), (32, 1), (16, 1), (8, 1), (16, 0), (8, 0)]


@pytest.mark.parametrize("csize,screen", LAYOUTS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_layouts_agree(env, csize, screen, prec):
    """Every cluster size, with and without the per-supplier box screen,
    gives the oracle's force and its exact pair count (the layout changes
    only which lanes evaluate a pair and the FP64 summation order)."""
    print("clustered n_side=24 csize=%d screen=%d" % (csize, screen), prec, flush=True)
    wl = make_workload("diff64", n_side=24)
    ref, cnt, absum = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, method="tiled")
    for ns in (1, 3):
        acc, st = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, prec,
                            subtiles_per_dim=ns, item_target=512, cluster_size=csize,
                            screen=screen)
        assert st["cluster_size"] == csize and st["screen"] == screen
        assert (st["screened"] > 0) == (screen == 1)
        check(acc, st, ref, cnt, absum, prec)


@pytest.mark.parametrize("csize,screen", [(8, 1), (16, 1), (64, 1), (8, 0)])
@pytest.mark.parametrize("n", [1, 2, 9, 63, 1000, 4097])
def test_layouts_ragged_masses_and_mask(env, n, csize, screen):
    """Small and ragged inputs with masses and an active mask on the
    screened / small-cluster layouts (partial clusters, empty lists)."""
    print("random n=%d csize=%d screen=%d" % (n, csize, screen), flush=True)
    pos, mass, active = random_particles(n, seed=200 + n, active_frac=0.6)
    if n <= 2:
        pos[:] = [0.5, 0.5, 0.5]
        pos[-1] = [0.52, 0.49, 0.5]
    x_s = 1.25 / 24
    r_cut = 4.5 * x_s
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active, method="brute")
    for prec in ("fp64", "fp32"):
        acc, st = run_force(env, pos, mass, active, 1.0, x_s, r_cut, prec, cluster_size=csize,
                            screen=screen)
        check(acc, st, ref, cnt, absum, prec, active)
        # unit masses take the specialised kernels
        ref1, cnt1, absum1 = oracle.force_full(pos, np.ones(n), 1.0, x_s, r_cut, active=active,
                                               method="brute")
        torch, p3, ctx = env
        ctx.set_config(cluster_size=csize, screen=screen)
        try:
            acc1 = ctx.force(to_dev(torch, pos), None, to_dev(torch, active), box=1.0, x_s=x_s,
                             r_cut=r_cut, precision=prec)
            torch.cuda.synchronize()
            st1 = ctx.stats()
        finally:
            ctx.set_config()
        check(acc1.cpu().numpy(), st1, ref1, cnt1, absum1, prec, active)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_diff64_clustered_full(env, prec):
    print("diff64 N=64^3 clustered", prec, flush=True)
    wl = make_workload("diff64")
    ref, cnt, absum = oracle.force_full(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, method="tiled")
    acc, st = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, prec)
    print(check(acc, st, ref, cnt, absum, prec), flush=True)


@pytest.mark.parametrize("csize,screen", [(64, 0), (8, 1), (16, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_clustered128_sampled(env, prec, csize, screen):
    """Full-size N=128^3 clustered set in the layouts the autotuner picks
    from; 512 seeded receivers checked one by one against brute force over
    all N."""
    print("clustered128 N=128^3", prec, csize, screen, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    acc, st = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, prec,
                        subtiles_per_dim=2, cluster_size=csize, screen=screen)
    idx = sample_indices(wl.n, 512, wl.config_id)
    ref, cnt, absum, _ = oracle.force(wl.pos, wl.mass, 1.0, wl.x_s, wl.r_cut, recv=idx)
    e = oracle.errors(acc[idx], ref, absum)
    print(e, st, flush=True)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    # total pair count: the ordered-pair total of this set lies near 1.56e9
    assert 1.0e9 < st["interactions"] < 2.5e9


@pytest.mark.parametrize("prec,csize", [("fp32", 32), ("fp64", 32), ("fp64", 16)])
def test_clustered128_65536_receivers(env, prec, csize):
    """Full-size N=128^3 clustered set in the bench's layouts (ns 1, items of
    4096, screened, 32-receiver clusters for FP32 and 16 for FP64): 65536
    seeded receivers against the cell-list oracle over all N."""
    print("clustered128 N=128^3, 65536 receivers", prec, csize, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    acc, st = run_force(env, wl.pos, None, None, 1.0, wl.x_s, wl.r_cut, prec,
                        subtiles_per_dim=1, item_target=4096, cluster_size=csize, screen=1)
    idx = sample_indices(wl.n, 65536, wl.config_id, salt=1)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                      method="tiled")
    e = oracle.errors(acc[idx], ref, absum)
    print(e, flush=True)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e


def test_edge_cases(env):
    torch, p3, ctx = env
    print("edge cases", flush=True)
    # empty input
    empty = torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")
    out = ctx.force(empty, None, None, box=1.0, x_s=0.01, r_cut=0.045)
    assert out.shape == (0, 3)
    # nobody active: output all zero, no interactions
    pos, mass, _ = random_particles(500, seed=3)
    acc, st = run_force(env, pos, mass, np.zeros(500, np.uint8), 1.0, 0.02, 0.09, "fp64")
    assert np.all(acc == 0) and st["interactions"] == 0 and st["receivers"] == 0
    # positions given outside [0, box): same force as the wrapped positions
    shift = np.random.default_rng(1).integers(-3, 4, size=pos.shape).astype(np.float64)
    a0, s0 = run_force(env, pos, mass, None, 1.0, 0.02, 0.09, "fp64")
    a1, s1 = run_force(env, pos + shift, mass, None, 1.0, 0.02, 0.09, "fp64")
    assert s0["interactions"] == s1["interactions"]
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, 0.02, 0.09, method="brute")
    assert oracle.errors(a1, ref, absum)["e_max_cond"] <= 1e-12
    # the smallest legal tiling: 3 tiles per dimension (r_cut just below box/3)
    box = 2.0
    r_cut = box / 3 * 0.999
    x_s = r_cut / 4.5
    pos3, mass3, act3 = random_particles(700, seed=5, box=box, active_frac=0.5)
    ref, cnt, absum = oracle.force_full(pos3, mass3, box, x_s, r_cut, active=act3,
                                        method="brute")
    for prec in ("fp64", "fp32"):
        a, st = run_force(env, pos3, mass3, act3, box, x_s, r_cut, prec)
        assert st["tiles_per_dim"] == 3
        check(a, st, ref, cnt, absum, prec, act3)
    # invalid geometry is rejected with EINVAL and no launch
    with pytest.raises(p3.P3MError) as ei:
        ctx.force(to_dev(torch, pos), None, None, box=1.0, x_s=0.1, r_cut=0.4)
    assert ei.value.code == -1


@pytest.mark.parametrize("csize,screen", [(8, 1), (16, 0), (32, 2), (64, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiny_all_active_sets(env, prec, csize, screen):
    """All-active calls on 1 to 40 particles packed into a few cells (one
    cluster, clusters shorter than a wave's lane group, a single occupied
    subtile): exact pair counts, and rows without a partner exactly 0."""
    x_s, r_cut = 0.01, 0.045
    for n in (1, 2, 5, 40):
        print("tiny all-active n=%d" % n, prec, csize, screen, flush=True)
        rng = np.random.default_rng(100 + n)
        pos = np.mod(0.3 + rng.random((n, 3)) * 0.05, 1.0)
        mass = rng.uniform(0.5, 2.0, n)
        ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, method="brute")
        acc, st = run_force(env, pos, mass, None, 1.0, x_s, r_cut, prec, cluster_size=csize,
                            screen=screen)
        check(acc, st, ref, cnt, absum, prec)
        assert np.all(acc[absum == 0] == 0)


@pytest.mark.parametrize("csize,screen", [(32, 1), (8, 1), (64, 0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lattice_pairs_on_the_cutoff(env, prec, csize, screen):
    """Sites of a 64^3 lattice, r_cut = 4 spacings: hundreds of pairs exactly
    at r_cut (rejected), coincident distinct particles (no contribution) and
    coordinates of exactly 1.0 (the same point as 0.0).  Separations are exact,
    so the accepted-pair count must match the oracle's exactly."""
    print("lattice", prec, csize, screen, flush=True)
    n_side, k = 64, 4
    pos, _ = lattice_sites(n_side, 6000, 300, 60, seed=11)
    rng = np.random.default_rng(12)
    mass = rng.uniform(0.5, 2.0, pos.shape[0])
    active = (rng.random(pos.shape[0]) < 0.6).astype(np.uint8)
    r_cut = k / n_side
    x_s = r_cut / 4.5
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active,
                                        method="brute")
    acc, st = run_force(env, pos, mass, active, 1.0, x_s, r_cut, prec, cluster_size=csize,
                        screen=screen)
    check(acc, st, ref, cnt, absum, prec, active)


def test_repeat_calls_stable(env):
    """Repeated calls reuse the workspace; results agree to rounding (the
    FP64 atomics may add item partial sums in a different order)."""
    wl = make_workload("diff64", n_side=32)
    a0, s0 = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, "fp32")
    a1, s1 = run_force(env, wl.pos, wl.mass, None, 1.0, wl.x_s, wl.r_cut, "fp32")
    assert s0["interactions"] == s1["interactions"]
    assert np.max(np.abs(a0 - a1)) <= 1e-12 * np.max(np.abs(a0))


@pytest.mark.parametrize("csize,screen", [(32, 1), (8, 1), (64, 0)])
@pytest.mark.parametrize("masked", [False, True])
def test_dense_subtiles(env, csize, screen, masked):
    """Subtiles far above 1024 particles (the block-wide fine order), whole
    waves of particles in one cell (grouped cell counts), sparse cells around
    them, with and without an active mask (the flag scan and compaction, or
    the receivers taken in place)."""
    print("dense subtiles csize=%d screen=%d masked=%d" % (csize, screen, masked), flush=True)
    rng = np.random.default_rng(77)
    n = 9000
    pos = rng.random((n, 3))
    pos[:3000] = 0.31 + 0.004 * rng.random((3000, 3))          # one dense subtile
    pos[3000:5000] = 0.72 + 0.01 * rng.standard_normal((2000, 3))
    pos %= 1.0
    mass = rng.uniform(0.5, 2.0, n)
    active = (rng.random(n) < 0.6).astype(np.uint8) if masked else None
    x_s, r_cut = 1.25 / 32, 4.5 * 1.25 / 32
    recv = np.concatenate([np.arange(0, 3000, 7), np.arange(3000, n, 11)])
    if masked:
        recv = recv[active[recv] != 0]
    ref, cnt, absum = oracle.force(pos, mass, 1.0, x_s, r_cut, recv=recv)[:3]
    for prec in ("fp64", "fp32"):
        acc, st = run_force(env, pos, mass, active, 1.0, x_s, r_cut, prec, subtiles_per_dim=1,
                            cluster_size=csize, screen=screen)
        e = oracle.errors(acc[recv], ref, absum)
        assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], (prec, e)
        if masked:
            assert np.all(acc[active == 0] == 0)
        else:
            assert st["receivers"] == n
