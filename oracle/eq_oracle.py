"""Plain CPU oracle for the equilibrium density, the neutral reference density and
the zero-bias conductance.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

What it computes (paper Section 2.2.1, the text after Eq. 4, and Eq. 6):

* ``equilibrium_charge``: with equal electrochemical potentials the whole
  density comes from the contour.  The upper contour runs from E_b to
  E_u = mu + f kT (no real-axis window); the closed path made of that arc and
  the real segment encloses the poles z_k = mu + i (2k+1) pi kT of the Fermi
  function, whose residue is -kT, so
      int_{E_b}^{E_u} G F dE = int_arc G F dz - 2 pi i kT sum_k G(z_k),
  and charge_i = -(g_s/pi) Im of that (the electron-count form of Eq. 4).
* ``neutral_charge``: the reference density rho_0 with E_l = E_u = 0, i.e. the
  zero-temperature occupation up to E = 0: the arc from E_b to 0 with F = 1.
* ``zero_bias_conductance``: Eq. 6, G = G_0 int T(E) (-dF/dE) dE with
  G_0 = g_s e^2/h, on real-axis nodes E_r with weights w_r.

Pins: ``tests/test_eq_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np

from . import negf_oracle as O


def fermi_poles(mu, kT, n):
    """The first n poles of F(z - mu; kT) in the upper half plane."""
    k = np.arange(n)
    return mu + 1j * (2 * k + 1) * np.pi * kT


def minus_fermi_derivative(E, mu, kT):
    """-dF/dE = 1 / (4 kT cosh^2((E - mu) / 2kT)), overflow-safe."""
    x = 0.5 * (np.asarray(E, np.float64) - mu) / kT
    return 1.0 / (4.0 * kT * np.cosh(np.clip(x, -350.0, 350.0)) ** 2)


def _contour_diag(prob, z):
    return np.array([O.energy_point_contour(prob, zz) for zz in np.atleast_1d(z)])


def equilibrium_charge(prob, mu, kT, z_arc, w_arc, n_poles):
    """charge_i (electrons per atom incl. spin) at equilibrium (mu, kT) from the arc
    nodes/weights (E_b -> mu + f kT) and the n_poles enclosed Fermi poles."""
    acc = np.zeros(prob.U.shape[0], np.complex128)
    if len(z_arc):
        acc += ((w_arc * O.fermi_complex(z_arc, mu, kT))[:, None] * _contour_diag(prob, z_arc)).sum(axis=0)
    if n_poles:
        acc += (-2j * np.pi * kT) * _contour_diag(prob, fermi_poles(mu, kT, n_poles)).sum(axis=0)
    return -(prob.g_s / np.pi) * np.imag(acc)


def neutral_charge(prob, z_arc, w_arc):
    """rho_0 per atom: the arc E_b -> 0 with no Fermi factor."""
    acc = (w_arc[:, None] * _contour_diag(prob, z_arc)).sum(axis=0)
    return -(prob.g_s / np.pi) * np.imag(acc)


def zero_bias_conductance(prob, mu, kT, E_r, w_r):
    """Eq. 6 in A/V: G_0 sum_r w_r T(E_r) (-dF/dE)(E_r), G_0 = g_s e^2/h."""
    T = np.array([O.energy_point_real(prob, E)[2] for E in E_r])
    return prob.g_s * O.G0_PER_SPIN * float(np.sum(w_r * T * minus_fermi_derivative(E_r, mu, kT)))
