"""The entry point that allocates nothing (p3m_sr_force_noalloc) against the
ordinary one (p3m_sr_force), through the C ABI: two calls in a row, the
second with a smaller input, each matching p3m_sr_force to the FP64 / FP32
bars and the oracle's exact pair count; sizes beyond the fixed workspace are
rejected before any launch."""
import numpy as np
import pytest

import oracle
from gpu_common import TOL, gpu_or_skip, to_dev
from workloads import make_workload, random_particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch, p3 = gpu_or_skip()
    return torch, p3, p3.Context(0)


def both(env, pos, mass, active, x_s, r_cut, prec):
    torch, p3, ctx = env
    args = (to_dev(torch, pos), to_dev(torch, mass), to_dev(torch, active))
    kw = dict(box=1.0, x_s=x_s, r_cut=r_cut, precision=prec)
    a_na = ctx.force_noalloc(*args, **kw)
    torch.cuda.synchronize()
    st_na = ctx.stats()
    a_ref = ctx.force(*args, **kw)
    torch.cuda.synchronize()
    st_ref = ctx.stats()
    return a_na.cpu().numpy(), st_na, a_ref.cpu().numpy(), st_ref


def check(pos, mass, active, x_s, r_cut, prec, got, st, ref_gpu):
    ref, cnt, absum = oracle.force_full(pos, mass, 1.0, x_s, r_cut, active=active)
    assert st["interactions"] == int(cnt.sum())
    e_gpu = oracle.errors(got, ref_gpu, absum)
    assert e_gpu["e_l2"] <= TOL[prec] and e_gpu["e_max_cond"] <= TOL[prec], e_gpu
    e = oracle.errors(got, ref, absum)
    assert e["e_l2"] <= TOL[prec] and e["e_max_cond"] <= TOL[prec], e
    if active is not None:
        assert np.all(got[active == 0] == 0)


@pytest.mark.parametrize("layout", [None, dict(cluster_size=32, screen=2),
                                    dict(cluster_size=16, screen=1, subtiles_per_dim=2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_calls_second_smaller(env, prec, layout):
    torch, p3, ctx = env
    print("no-alloc", prec, layout, flush=True)
    if layout:
        ctx.set_config(**layout)
    try:
        wl = make_workload("diff64", n_side=48)               # 110592 clustered particles
        got, st, ref_gpu, _ = both(env, wl.pos, None, None, wl.x_s, wl.r_cut, prec)
        check(wl.pos, None, None, wl.x_s, wl.r_cut, prec, got, st, ref_gpu)
        pos, mass, active = random_particles(5000, seed=44, active_frac=0.6)
        x_s = 1.25 / 24
        got, st, ref_gpu, _ = both(env, pos, mass, active, x_s, 4.5 * x_s, prec)
        check(pos, mass, active, x_s, 4.5 * x_s, prec, got, st, ref_gpu)
    finally:
        ctx.set_config()


def test_limits_rejected_before_launch(env):
    torch, p3, ctx = env
    n = (1 << 18) + 1
    pos = torch.rand((n, 3), dtype=torch.float64, device="cuda:0")
    out = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(p3.P3MError) as ei:
        ctx.force_noalloc(pos, box=1.0, x_s=0.01, r_cut=0.045, out=out)
    assert ei.value.code == p3.P3M_EUNSUPPORTED
    # a geometry whose fine cells do not fit: 1000^3 tiles
    small = torch.rand((64, 3), dtype=torch.float64, device="cuda:0")
    out2 = torch.full((64, 3), 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(p3.P3MError) as ei:
        ctx.force_noalloc(small, box=1.0, x_s=0.0002, r_cut=0.0009, out=out2)
    assert ei.value.code == p3.P3M_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(out == 7.0) and torch.all(out2 == 7.0)
    # the entry point still works after the rejections
    pos_np, mass_np, _ = random_particles(3000, seed=45)
    got, st, ref_gpu, _ = both(env, pos_np, mass_np, None, 1.25 / 24, 4.5 * 1.25 / 24, "fp64")
    check(pos_np, mass_np, None, 1.25 / 24, 4.5 * 1.25 / 24, "fp64", got, st, ref_gpu)
