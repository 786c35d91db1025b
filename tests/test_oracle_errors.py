"""Pin of the error measures every parity test and the benchmark report
(oracle.errors), on a three-row case worked out by hand.

Rows (reference, computed, sum of pair-force magnitudes):
  0: ref (3, 4, 0)    a (3, 4, 1)      absum 10   |diff| 1    |ref| 5
  1: ref (0, 0, 2)    a (0.3, 0.4, 2)  absum 4    |diff| 0.5  |ref| 2
  2: ref (0, 0, 0)    a (0, 0, 0)      absum 0    (no accepted pair)

  e_l2       = sqrt(1 + 0.25) / sqrt(25 + 4)          = sqrt(1.25 / 29)
  e_max_cond = max(1 / 10, 0.5 / 4)                    = 0.125
  p999       = rows with ref != 0: ratios 0.2 and 0.25; the 99.9th
               percentile sits at rank 0.999 between them: 0.2 + 0.999 * 0.05
  max_abs    = 1
A nonzero computed row where the reference has no partner (absum 0) is an
error no relative measure can express: e_max_cond is then infinite.
"""
import math

import numpy as np

import oracle

REF = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 2.0], [0.0, 0.0, 0.0]])
GOT = np.array([[3.0, 4.0, 1.0], [0.3, 0.4, 2.0], [0.0, 0.0, 0.0]])
ABSUM = np.array([10.0, 4.0, 0.0])


def test_hand_worked_values():
    e = oracle.errors(GOT, REF, ABSUM)
    assert abs(e["e_l2"] - math.sqrt(1.25 / 29.0)) <= 1e-15
    assert abs(e["e_max_cond"] - 0.125) <= 1e-16
    assert abs(e["p999"] - (0.2 + 0.999 * 0.05)) <= 1e-15
    assert e["max_abs"] == 1.0


def test_row_without_partner_must_be_zero():
    got = GOT.copy()
    got[2, 1] = 1e-30
    assert oracle.errors(got, REF, ABSUM)["e_max_cond"] == float("inf")


def test_rows_are_not_transposed_or_swapped():
    """The measures are per row (particle): swapping two computed rows or
    measuring along the wrong axis changes them."""
    e = oracle.errors(GOT[[1, 0, 2]], REF, ABSUM)
    assert e["e_max_cond"] > 0.125
    e0 = oracle.errors(REF, REF, ABSUM)
    assert e0 == dict(e_l2=0.0, e_max_cond=0.0, p999=0.0, max_abs=0.0)
