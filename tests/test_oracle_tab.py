"""Pins of the tabulated-shape oracle (section 2.1.3, "Other
optimisations": the bracket of eq. p3m_gravity in a 1D table on r^2, read
by nearest grid point or, as the paper suggests for smaller tables, by
linear interpolation).

- H(t) = (g(u) - 1) / u^3 has the limit -4 / (3 sqrt(pi)) at u = 0, its
  series and its direct form agree where they meet, and r^-3 + H / (2 x_s)^3
  is the bracket written with erfc and exp;
- the tabulated force converges to the exact one (the short-range oracle)
  at first order in the table size for NGP and at second order for linear
  interpolation: a bin-edge instead of bin-centre NGP value, an index off by
  one or a wrong slope changes those rates;
- the errors at the table sizes the GPU offers are the stated ones.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import tab_oracle as tb
from workloads import make_workload


def test_h_limits_and_series_join():
    assert abs(tb.h_exact(0.0) + 4.0 / (3.0 * math.sqrt(math.pi))) <= 1e-15
    u = 0.05
    g = math.erfc(u) + 2.0 / math.sqrt(math.pi) * u * math.exp(-u * u)
    direct = (g - 1.0) / u ** 3
    assert abs(tb.h_exact(u * u * (1 - 1e-12)) - direct) <= 1e-11
    assert abs(tb.h_exact(u * u) - direct) <= 1e-11


@pytest.mark.parametrize("r", [1e-3, 0.01, 0.03, 0.05])
def test_bracket_identity(r):
    x_s = 0.01
    u = r / (2 * x_s)
    bracket = math.erfc(u) / r ** 3 + math.exp(-u * u) / (math.sqrt(math.pi) * x_s * r * r)
    assert abs(1.0 / r ** 3 + tb.h_exact(u * u) / (2 * x_s) ** 3 - bracket) <= 1e-12 * bracket


@pytest.fixture(scope="module")
def setup():
    wl = make_workload("diff64", n_side=24)
    idx = np.arange(0, wl.n, 37)
    ref, _, absum, _ = oracle.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, recv=idx)
    return wl, idx, ref, absum


def err(setup, kind, n):
    wl, idx, ref, absum = setup
    a = tb.force(wl.pos, None, 1.0, wl.x_s, wl.r_cut, idx, kind, n)
    return oracle.errors(a, ref, absum)["e_l2"]


def test_ngp_converges_at_first_order(setup):
    e = [err(setup, tb.NGP, n) for n in (512, 1024, 2048)]
    assert 1.7 < e[0] / e[1] < 2.3 and 1.7 < e[1] / e[2] < 2.3, e


def test_linear_converges_at_second_order(setup):
    e = [err(setup, tb.LINEAR, n) for n in (64, 128, 256)]
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def test_stated_errors(setup):
    """The errors quoted for the GPU's table choices (e_L2 of the 2^12-entry
    NGP table 2.8e-5; linear interpolation with 1024 entries 1.5e-7)."""
    assert err(setup, tb.NGP, 4096) <= 3.5e-5
    assert err(setup, tb.LINEAR, 1024) <= 2e-7
