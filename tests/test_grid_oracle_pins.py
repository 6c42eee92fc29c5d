"""Pins of the semi-adaptive grid oracle: quadrature exactness of the three-part
rule, node counts from the densities, and the refinement rule on an integrand
whose peak is known."""
import numpy as np
import pytest

from oracle import grid_oracle as G
from paper_2407_14633_amd import workload as W


def test_three_part_rule_is_exact_for_polynomials():
    E, w = G.three_part_grid(-0.5, 0.7, -0.1, 0.2, (20, 40, 10), 0.0259)
    for deg in range(6):
        exact = (0.7 ** (deg + 1) - (-0.5) ** (deg + 1)) / (deg + 1)
        assert np.sum(w * E ** deg) == pytest.approx(exact, rel=1e-12, abs=1e-14)


def test_node_counts_follow_densities():
    kT = 0.02
    E, w = G.three_part_grid(0.0, 1.0, 0.3, 0.5, (10, 50, 5), kT)
    n = [int(np.ceil(10 * 0.3 / kT)), int(np.ceil(50 * 0.2 / kT)), int(np.ceil(5 * 0.5 / kT))]
    assert len(E) == sum(n)
    assert np.all((E[: n[0]] > 0) & (E[: n[0]] < 0.3))
    assert np.all((E[n[0]: n[0] + n[1]] > 0.3) & (E[n[0]: n[0] + n[1]] < 0.5))


def test_refinement_follows_the_peak():
    # Lorentzian integrand centred at 0.1 eV: the refined upper limit is E_s + b kT with
    # E_s the probe node nearest the peak, the lower limit moves down by a kT
    bias = W.Bias(0.15, -0.15)
    kT = bias.kT_L
    p = W.Problem("g", W.zigzag_cnt(8, 4), np.zeros(32), 0.0, 0.0, bias,
                  W.EnergyGrid(np.zeros(0, complex), np.zeros(0, complex), np.zeros(0), np.zeros(0)))
    peak = 0.1
    f = lambda E: 1.0 / ((E - peak) ** 2 + 1e-4)
    E_r, w_r, (l1, l2, Es) = G.semi_adaptive_grid(p, -0.2, 0.05, 3.0, 1.0, (5, 40, 5), integrand=f)
    E_p, _ = G.three_part_grid(*G.window(bias), -0.2, 0.05, (5, 40, 5), kT)
    assert Es == E_p[np.argmin(np.abs(E_p - peak))]
    assert l1 == pytest.approx(-0.2 - 3 * kT, abs=1e-15) and l2 == pytest.approx(Es + kT, abs=1e-15)
    assert np.sum(w_r) == pytest.approx(G.window(bias)[1] - G.window(bias)[0], rel=1e-13)
