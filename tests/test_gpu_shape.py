"""Tabulated FP32 kernel shape on the GPU (p3m_sr_set_shape; section 2.1.3,
"Other optimisations") against the tabulated-shape oracle (the same table
and bin choice, FP64 elsewhere) and, for the stated accuracy, against the
exact FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_common import gpu_or_skip, to_dev
from oracle import tab_oracle as tb
from workloads import make_workload, random_particles, sample_indices

pytestmark = pytest.mark.gpu

KINDS = {"table_ngp": tb.NGP, "table_linear": tb.LINEAR}
# e_L2 against the exact oracle at each choice (the oracle's own figures on
# the diff64 set, with margin for the FP32 rest of the shape)
STATED = {("table_ngp", 4096): 4e-5, ("table_ngp", 1024): 1.5e-4,
          ("table_linear", 2048): 2e-7, ("table_linear", 1024): 3e-7,
          ("table_linear", 256): 4e-6}


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def gpu_force(env, pos, mass, active, x_s, r_cut, kind, size, **cfg):
    torch, p3, ctx = env
    ctx.set_shape(kind, size)
    if cfg:
        ctx.set_config(**cfg)
    try:
        acc = ctx.force(to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active), box=1.0,
                        x_s=x_s, r_cut=r_cut, precision="fp32")
        torch.cuda.synchronize()
        return acc.cpu().numpy(), ctx.stats()
    finally:
        ctx.set_shape("poly")
        ctx.set_config()


@pytest.mark.parametrize("kind, size", sorted(STATED))
@pytest.mark.parametrize("layout", [dict(cluster_size=64, screen=0),
                                    dict(cluster_size=16, screen=1)])
def test_shape_matches_tab_oracle(env, kind, size, layout):
    print("shape", kind, size, layout, flush=True)
    wl = make_workload("diff64", n_side=24)
    idx = sample_indices(wl.n, 600, wl.config_id)
    acc, st = gpu_force(env, wl.pos, None, None, wl.x_s, wl.r_cut, kind, size, **layout)
    assert st["shape"] == {"table_ngp": 1, "table_linear": 2}[kind]
    ref_t = tb.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, idx, KINDS[kind], size)
    ref, cnt, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx)
    assert st["interactions"] == int(oracle.force_full(wl.pos, None, 1.0, wl.x_s,
                                                       wl.r_cut)[1].sum())
    e_t = oracle.errors(acc[idx], ref_t, absum)
    e = oracle.errors(acc[idx], ref, absum)
    print("vs table oracle", e_t, "vs exact", e, flush=True)
    assert e_t["e_max_cond"] <= 2e-6, e_t
    assert e["e_l2"] <= STATED[(kind, size)], e


def test_shape_masses_and_mask(env):
    pos, mass, active = random_particles(3000, seed=71, active_frac=0.5)
    x_s = 1.25 / 48
    r_cut = 4.5 * x_s
    idx = np.nonzero(active)[0][::5]
    acc, st = gpu_force(env, pos, mass, active, x_s, r_cut, "table_linear", 1024)
    ref_t = tb.force(pos, mass, 1.0, x_s, r_cut, idx, tb.LINEAR, 1024)
    _, _, absum, _ = oracle.force(pos, mass, 1.0, x_s, r_cut, recv=idx)
    assert oracle.errors(acc[idx], ref_t, absum)["e_max_cond"] <= 2e-6
    assert np.all(acc[active == 0] == 0.0)


def test_shape_ignored_by_fp64_and_softened_calls(env):
    torch, p3, ctx = env
    wl = make_workload("diff64", n_side=16)
    ctx.set_shape("table_ngp", 4096)
    try:
        ctx.force(to_dev(torch, wl.pos), None, None, box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                  precision="fp64")
        assert ctx.stats()["shape"] == 0
        ctx.set_softening(0.001)
        ctx.force(to_dev(torch, wl.pos), None, None, box=1.0, x_s=wl.x_s, r_cut=wl.r_cut,
                  precision="fp32")
        assert ctx.stats()["shape"] == 0
    finally:
        ctx.set_softening(0.0)
        ctx.set_shape("poly")


@pytest.mark.parametrize("kind", ["table_ngp", "table_linear"])
def test_shape_clustered128_sampled(env, kind):
    print("shape clustered128", kind, flush=True)
    wl = make_workload("clustered128", with_rungs=False)
    size = 4096 if kind == "table_ngp" else 1024
    acc, st = gpu_force(env, wl.pos, None, None, wl.x_s, wl.r_cut, kind, size,
                        subtiles_per_dim=1, item_target=4096, cluster_size=32, screen=1)
    idx = sample_indices(wl.n, 256, wl.config_id)
    ref_t = tb.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, idx, KINDS[kind], size)
    ref, _, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx,
                                    method="tiled")
    e_t = oracle.errors(acc[idx], ref_t, absum)
    print(e_t, oracle.errors(acc[idx], ref, absum), flush=True)
    assert e_t["e_max_cond"] <= 2e-6
