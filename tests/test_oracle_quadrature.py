"""Pins of the oracle's quadrature (Sec. III.C-D) against the numbers the paper
prints for its worked example (mbar = 5, G1..G6) and its stencil sizes."""
import json
import os

import numpy as np
import pytest
from mpmath import mp, mpf

from oracle import groups, quadrature as quad, lattice
from oracle.polynomials import evaluate_printed

PINS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))
Q5 = PINS["quadrature_m5_G1_G6"]


def test_group_table_cardinalities_and_lengths():
    # Appendix C table: the printed cardinality of each FS set
    for g, (base, card) in groups.GROUPS.items():
        orbit = groups.fs_orbit(base)
        assert len(orbit) == card, g
        assert all(sum(c * c for c in v) == sum(c * c for c in base) for v in orbit)
        assert all(0 <= base[2] <= base[1] <= base[0] <= 6 for _ in [0])
    assert len(groups.GROUPS) == 84


def test_stencil_sizes_match_paper():
    s = PINS["stencil_sizes"]
    size = lambda gs: sum(len(groups.fs_orbit(groups.base_of(g))) for g in gs)
    assert size([1, 2, 3, 4, 5, 6]) == s["second_order_G1_G6"]
    assert size([1, 2, 3, 4, 5, 8, 9, 10, 12, 13, 15]) == s["third_order_G1_G2_G3_G4_G5_G8_G9_G10_G12_G13_G15"]
    assert size([1, 14, 49, 51, 60, 70]) == s["bamps_G1_G14_G49_G51_G60_G70"]
    # pruning one group of the worked example
    assert size([1, 3, 4, 5, 6]) == Q5["n_after_prune_w2"]
    assert size([1, 2, 4, 5, 6]) == Q5["n_after_prune_w3"]


def test_printed_weights_m5():
    w, res = quad.weights(groups.bases_of(Q5["groups"]), Q5["mbar"], mpf("0.398"))
    assert res < mpf(10) ** -35          # the 105 conditions are consistent
    for wi, pi in zip(w, Q5["weights_truncated"]):
        assert 0 <= float(wi) - pi < 1e-10   # printed values are truncated ("...")


def test_pruning_points_m5():
    b = groups.bases_of(Q5["groups"])
    w_lo, _ = quad.weights(b, 5, mpf("0.3965826549"))
    w_hi, _ = quad.weights(b, 5, mpf("0.3984063950"))
    assert abs(w_lo[1]) < 1e-8 and abs(w_hi[2]) < 1e-8
    # and they are zero crossings: the weight changes sign within 1e-9 of the printed v0
    wa, _ = quad.weights(b, 5, mpf("0.3965826549") - mpf("1e-9"))
    wb, _ = quad.weights(b, 5, mpf("0.3965826549") + mpf("1e-9"))
    assert wa[1] * wb[1] < 0


def test_positive_window_m5():
    r = quad.positive_window(groups.bases_of(Q5["groups"]), 5, 0.3955, 0.3995, grid=30)
    assert r is not None
    lo, hi, _ = r
    assert round(float(lo), 4) == Q5["positive_window_rounded"][0]
    assert round(float(hi), 4) == Q5["positive_window_rounded"][1]
    assert abs(float(lo) - Q5["prune_w2_v0"]) < 1e-9
    assert abs(float(hi) - Q5["prune_w3_v0"]) < 1e-9


@pytest.mark.parametrize("gs,mbar,v0", [([1, 2, 3, 4, 5, 6], 5.0, 0.398),
                                        ([1, 5, 11, 13, 17, 21], 1.0, 0.2403918860),
                                        ([1, 14, 49, 51, 60, 70], 0.36, 0.1488231854)])
def test_float64_orthonormality(gs, mbar, v0):
    """sum_i w_i J_l(p_i) J_k(p_i) = delta_lk (eq. ortho1) in float64, all 14x14 pairs,
    and all weights positive at the chosen v0."""
    ps = lattice.build_stencil(groups.bases_of(gs), mbar, v0, mode="full")
    assert min(ps.group_weights) > 0
    J = np.array(evaluate_printed(ps.p, mbar))          # [14, Q]
    G = ps.M.T @ J.T                                    # sum_i w_i J_l J_k
    assert np.abs(G - np.eye(14)).max() < 1e-12
    assert abs(ps.M[:, 0].sum() - 1.0) < 1e-14           # sum_i w_i = 1
