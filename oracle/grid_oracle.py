"""Plain CPU oracle for the semi-adaptive real-axis grid.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

The paper's semi-adaptive scheme (Section 3.3, discussion of integration points),
in its order:
1. the window [E_min, E_max] (Eq. 4) is split at E_l1 < E_l2 into three parts,
   each integrated by Gauss-Legendre with a user density of nodes per kT;
2. from guesses of E_l1 and E_l2, the integrand f_L A_L + f_R A_R at the centre
   of the channel is evaluated on that grid and its peak E_s located;
3. the limits are refined as E_l1 <- E_l1 - a kT and E_l2 <- E_s + b kT
   (a = 3, b = 1 typically) and the grid is rebuilt with the same densities.
Readings: "the centre of the channel" is ring N // 2 (its atoms summed); kT and
the Fermi functions are those of the left lead for f_L and the right lead for
f_R; a part's node count is ceil(density x width / kT_min), at least one; the
refined limits are clipped to [E_min, E_max] and kept ordered.

Pins: ``tests/test_grid_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np

from . import negf_oracle as O


def window(bias, tail=14.0):
    return (min(bias.mu_L, bias.mu_R) - tail * min(bias.kT_L, bias.kT_R),
            max(bias.mu_L, bias.mu_R) + tail * max(bias.kT_L, bias.kT_R))


def three_part_grid(E_min, E_max, E_l1, E_l2, density, kT):
    """Gauss-Legendre nodes/weights on [E_min, E_l1], [E_l1, E_l2], [E_l2, E_max]."""
    E, w = [], []
    for lo, hi, dens in ((E_min, E_l1, density[0]), (E_l1, E_l2, density[1]), (E_l2, E_max, density[2])):
        if hi <= lo:
            continue
        n = max(1, int(np.ceil(dens * (hi - lo) / kT - 1e-9)))
        x, ww = np.polynomial.legendre.leggauss(n)
        E.append(0.5 * (hi + lo) + 0.5 * (hi - lo) * x)
        w.append(0.5 * (hi - lo) * ww)
    return np.concatenate(E), np.concatenate(w)


def centre_integrand(prob, E_r):
    """f_L A_L + f_R A_R summed over the atoms of ring N // 2, at every node."""
    N, b = prob.device.n_rings, prob.device.b
    jc = N // 2
    fL = O.fermi(E_r, prob.bias.mu_L, prob.bias.kT_L)
    fR = O.fermi(E_r, prob.bias.mu_R, prob.bias.kT_R)
    out = np.zeros(len(E_r))
    for k, E in enumerate(E_r):
        AL, AR, _, _ = O.energy_point_real(prob, E)
        out[k] = np.sum(fL[k] * AL[jc * b:(jc + 1) * b] + fR[k] * AR[jc * b:(jc + 1) * b])
    return out


def semi_adaptive_grid(prob, E_l1, E_l2, a, b, density, integrand=None):
    """Returns (E_r, w_r, (E_l1', E_l2', E_s)) after one refinement from the guesses."""
    bias = prob.bias
    kT = min(bias.kT_L, bias.kT_R)
    E_min, E_max = window(bias)
    E_l1, E_l2 = min(max(E_l1, E_min), E_max), min(max(E_l2, E_min), E_max)
    E_p, _ = three_part_grid(E_min, E_max, E_l1, E_l2, density, kT)
    f = (integrand or (lambda E: centre_integrand(prob, E)))(E_p)
    E_s = float(E_p[int(np.argmax(f))])
    n1 = min(max(E_l1 - a * kT, E_min), E_max)
    n2 = min(max(E_s + b * kT, n1), E_max)
    E_r, w_r = three_part_grid(E_min, E_max, n1, n2, density, kT)
    return E_r, w_r, (n1, n2, E_s)
