"""Plain CPU oracle for the self-consistent bias point (NEGF + electrostatics).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

What it computes (paper Section 2.3 and Algorithm 3, with the electrostatics
reduced to one dimension along the tube axis):

* ``poisson_rings``: the per-ring electrostatic potential phi from the per-ring
  electron count rho by the finite-difference equation stated in
  ``paper_2407_14633_amd.workload.Electrostatics`` (a banded solve); the
  electron potential energy is U_j = -phi_j on every atom of ring j.
* ``Broyden``: Broyden's modified second method as listed in Algorithm 3,
  step by step on the vector rho (f = rho_in - rho_out; Delta f; the relative
  norm eps = |f/(rho_in + rho_out)|; d = |Delta f|^2; the m-th row of V^T and
  column of W; s = W V^T f; rho_in <- rho_in - zeta f - s).  Readings: the loop
  runs while eps_max >= tol; the printed "eta" of the W update is the Broyden
  fraction zeta; a history of H stored columns restarts the method (m <- 0)
  once m would exceed H.
* ``potential_residual``: phi(rho_out) - phi(rho_in), the change of the
  electrostatic potential that the output charge implies; by linearity it solves
  the Poisson operator with zero boundary values and right-hand side e f / dz.
  Its maximum (V, i.e. eV for one electron) is the alternative stopping norm
  (norm = 1) that states the tolerance as a potential.
* ``self_consistent``: the loop rho_in -> Poisson -> U -> NEGF (the FP64
  oracle of ``negf_oracle``) -> rho_out -> Broyden, from rho_in = n_ref, or from
  a given starting charge (a warm start from a neighbouring bias point, as the
  paper does along an I-V sweep, Section 3.3).  With
  a semi-adaptive grid (Section 3.3), the real-axis nodes are rebuilt by
  ``grid_oracle.semi_adaptive_grid`` at the current potential before NEGF pass
  1, 1 + refresh, 1 + 2 refresh, ... (reading: "refreshed every so many
  iterations" counts NEGF passes, the first rebuild before the first solve).

Pins: ``tests/test_sc_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from . import negf_oracle as O

E_CHARGE = 1.602176634e-19   # C


def poisson_rings(rho, elec):
    """phi (V) per ring for electron counts rho (Electrostatics finite-difference form)."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    k = elec.eps_1d / elec.dz ** 2            # F/m, axial stiffness
    ab = np.zeros((3, N))
    ab[0, 1:] = -k                            # super-diagonal
    ab[1, :] = 2.0 * k + elec.c_gate          # diagonal
    ab[2, :-1] = -k                           # sub-diagonal
    rhs = elec.c_gate * elec.V_GS - E_CHARGE * (rho - elec.n_ref) / elec.dz
    rhs[0] += k * 0.0                         # source: phi_{-1} = 0
    rhs[-1] += k * elec.V_DS                  # drain:  phi_N = V_DS
    return solve_banded((1, 1), ab, rhs)


def potential_residual(f, elec):
    """phi(rho_in - f) - phi(rho_in) for f = rho_in - rho_out: the tridiagonal Poisson
    operator of ``poisson_rings`` with zero boundary values applied to e f / dz."""
    f = np.asarray(f, np.float64)
    N = f.shape[0]
    k = elec.eps_1d / elec.dz ** 2
    ab = np.zeros((3, N))
    ab[0, 1:] = -k
    ab[1, :] = 2.0 * k + elec.c_gate
    ab[2, :-1] = -k
    return solve_banded((1, 1), ab, E_CHARGE * f / elec.dz)


def ring_potential(phi, b):
    """Per-atom electron potential energy (eV) from the ring potential (V)."""
    return -np.repeat(np.asarray(phi, np.float64), b)


class Broyden:
    """Algorithm 3 on a vector of length n (history H columns, fraction zeta)."""

    def __init__(self, rho0, zeta, history):
        n = len(rho0)
        self.zeta, self.H = float(zeta), int(history)
        self.rho_in = np.array(rho0, np.float64)
        self.rho_in_old = np.zeros(n)
        self.f_old = np.zeros(n)
        self.s = np.zeros(n)
        self.Vt = np.zeros((self.H + 1, n))   # rows 1..H used
        self.W = np.zeros((self.H + 1, n))    # W[j] is column j
        self.m = 0

    def step(self, rho_out):
        """One pass of the loop body after the NEGF solve.  Returns (eps_max, converged-input)."""
        rho_in = self.rho_in
        f = rho_in - rho_out                                  # step 2
        df = f - self.f_old                                   # step 3
        eps = np.abs(f / (rho_in + rho_out))                  # step 4
        eps_max = float(np.max(eps))                          # steps 5, 7
        d = float(np.sum(df * df))                            # steps 6, 8
        return eps_max, f, df, d

    def update(self, f, df, d):
        """Steps 9-18 for the current m, then m <- m + 1."""
        if self.m > self.H:                                   # history exhausted: restart
            self.m = 0
            self.s = np.zeros_like(self.s)
        m = self.m
        if m > 0:
            if m > 1:
                k = np.array([self.Vt[j] @ df for j in range(1, m)])      # step 9
                self.s = sum(self.W[j] * k[j - 1] for j in range(1, m))   # step 11
            self.Vt[m] = df / d                                           # step 12
            self.W[m] = -self.zeta * df + self.rho_in - self.rho_in_old - self.s   # step 13
            k = np.array([self.Vt[j] @ f for j in range(1, m + 1)])       # step 14
            self.s = sum(self.W[j] * k[j - 1] for j in range(1, m + 1))   # step 16
        self.rho_in_old = self.rho_in.copy()                              # step 17
        self.rho_in = self.rho_in_old - self.zeta * f - self.s            # step 18
        self.f_old = f
        self.m += 1


def ring_counts(charge, b):
    """Electrons per ring from the per-atom charge."""
    return np.asarray(charge, np.float64).reshape(-1, b).sum(axis=1)


def negf_problem(req, U):
    """The NEGF input of one loop pass: the request's device and grid at potential U."""
    from paper_2407_14633_amd.workload import Problem
    return Problem(req.name, req.device, U, req.U_left, req.U_right, req.bias, req.grid,
                   req.eta, req.decim_tol, req.decim_max_iter, req.g_s)


def self_consistent(req, solve=None):
    """Runs the loop from rho_in = n_ref.  Returns dict(U, phi, rho, charge, current,
    iterations, eps_max, converged, history of eps_max, n_r of the last grid)."""
    from dataclasses import replace

    from . import grid_oracle as G
    solve = solve or (lambda p: O.solve(p))
    b = req.device.b
    br = Broyden(req.elec.n_ref if req.rho_init is None else req.rho_init, req.zeta, req.history)
    trace = []
    out = None
    grid = req.grid
    for it in range(1, req.max_iter + 1):
        phi = poisson_rings(br.rho_in, req.elec)                # step 1: electrostatics
        U = ring_potential(phi, b)
        if req.grid_density is not None and (it - 1) % (req.grid_refresh or 50) == 0:
            probe = negf_problem(req, U)
            E_r, w_r, _ = G.semi_adaptive_grid(probe, req.grid_limits[0], req.grid_limits[1], req.grid_a,
                                               req.grid_b, req.grid_density)
            grid = type(req.grid)(req.grid.z_c, req.grid.w_c, E_r, w_r)
        res = solve(negf_problem(replace(req, grid=grid), U))   # step 1: NEGF
        rho_out = ring_counts(res["charge"], b)
        eps_max, f, df, d = br.step(rho_out)
        if req.norm == 1:
            eps_max = float(np.max(np.abs(potential_residual(f, req.elec))))
        trace.append(eps_max)
        out = dict(U=U, phi=phi, rho=rho_out, rho_in=br.rho_in.copy(), charge=res["charge"],
                   current=res["current"], iterations=it, eps_max=eps_max, converged=eps_max < req.tol,
                   trace=trace, n_r=grid.n_r)
        if eps_max < req.tol:
            break
        br.update(f, df, d)
    return out
