"""The seeded generators are deterministic and produce valid inputs."""
import numpy as np

from workloads import make_workload, sample_indices, stratified_by_rung


def test_generators_are_deterministic_and_in_box():
    a = make_workload("diff64", n_side=16)
    b = make_workload("diff64", n_side=16)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.weights, b.weights)
    assert a.pos.min() >= 0.0 and a.pos.max() < 1.0
    assert a.n == 16 ** 3 and a.n_pm == 32
    assert abs(a.x_s - 1.25 / 32) < 1e-18 and abs(a.r_cut - 4.5 * a.x_s) < 1e-18


def test_clustered_rungs_cover_hierarchy():
    wl = make_workload("clustered256", n_side=48)
    hist = np.bincount(wl.rung, minlength=8)
    assert hist[0] == hist.max() and hist.sum() == wl.n
    assert (hist > 0).sum() >= 6
    nested = [int(wl.active_subset(k).sum()) for k in range(8)]
    assert all(nested[k] >= nested[k + 1] for k in range(7))


def test_samples():
    s = sample_indices(1000, 64, 4)
    assert s.size == 64 and np.unique(s).size == 64
    r = np.repeat(np.arange(4, dtype=np.uint8), 50)
    st = stratified_by_rung(r, 10, 3)
    assert st.size == 40 and np.all(np.bincount(r[st]) == 10)
