"""Pins of the self-consistency oracle (electrostatics, Broyden, loop) to closed forms.

Each check is independent of the oracle's own formulas: discrete closed-form
solutions of the Poisson recurrence, finite termination of Broyden's method on
a linear fixed-point problem, plain linear mixing when no history is kept, and
the gate-dominated limit where the loop must stop after one secant step.
"""
import numpy as np
import pytest

from oracle import negf_oracle as O
from oracle import sc_oracle as S
from paper_2407_14633_amd import workload as W


def _elec(N, k_over_c=1.0, V_DS=0.0, V_GS=0.0, c_gate=1e-10, dz=1e-10, n_ref=None):
    eps_1d = k_over_c * c_gate * dz ** 2
    return W.Electrostatics(dz, eps_1d, c_gate, np.full(N, 4.0) if n_ref is None else n_ref, V_DS, V_GS)


@pytest.mark.parametrize("V_DS,V_GS,k_over_c", [(0.3, 0.0, 1.0), (0.0, -0.4, 2.5), (0.6, 0.5, 40.0)])
def test_poisson_neutral_closed_form(V_DS, V_GS, k_over_c):
    # psi_j = phi_j - V_GS solves psi_{j+1} - (2 + c/k) psi_j + psi_{j-1} = 0, so
    # psi_j = A r^j + B r^-j with r + 1/r = 2 + c/k, psi_{-1} = -V_GS, psi_N = V_DS - V_GS.
    N = 37
    e = _elec(N, k_over_c, V_DS, V_GS)
    phi = S.poisson_rings(e.n_ref, e)
    q = 2.0 + 1.0 / k_over_c
    r = 0.5 * (q - np.sqrt(q * q - 4.0))
    M = np.array([[r ** -1, r ** 1], [r ** N, r ** -N]])
    A, B = np.linalg.solve(M, [-V_GS, V_DS - V_GS])
    j = np.arange(N)
    ref = V_GS + A * r ** j + B * r ** (-j)
    assert np.max(np.abs(phi - ref)) < 1e-12


def test_poisson_point_charge_response():
    # one extra electron on ring j0 of a long neutral tube with grounded ends and gate:
    # psi_j = C r^|j-j0|, C (2k(1-r) + c) = -e/dz  (ends at r^50 ~ 1e-21 of the peak)
    N, j0 = 101, 50
    e = _elec(N, 1.0)
    rho = e.n_ref.copy()
    rho[j0] += 1.0
    phi = S.poisson_rings(rho, e)
    k, c = e.eps_1d / e.dz ** 2, e.c_gate
    q = 2.0 + c / k
    r = 0.5 * (q - np.sqrt(q * q - 4.0))
    C = (-S.E_CHARGE / e.dz) / (2.0 * k * (1.0 - r) + c)
    ref = C * r ** np.abs(np.arange(N) - j0)
    assert np.max(np.abs(phi - ref)) < 1e-12 * np.max(np.abs(ref))
    assert phi[j0] < 0   # an extra electron lowers the electrostatic potential


def test_ring_potential_sign_and_layout():
    U = S.ring_potential(np.array([0.1, -0.2]), 3)
    assert np.array_equal(U, [-0.1, -0.1, -0.1, 0.2, 0.2, 0.2])


def _linear_problem(n=6, seed=3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = np.linspace(-3.0, 0.5, n)
    A = Q @ np.diag(lam) @ Q.T
    c = rng.normal(size=n) + 5.0
    return A, c, np.linalg.solve(np.eye(n) - A, c)


def test_broyden_terminates_on_linear_problem():
    # Broyden's methods reach the fixed point of an affine map in at most 2n+1 passes
    n = 6
    A, c, rho_star = _linear_problem(n)
    br = S.Broyden(np.full(n, 5.0), 0.3, history=4 * n)
    for it in range(1, 2 * n + 2):
        eps, f, df, d = br.step(A @ br.rho_in + c)
        if eps < 1e-13:
            break
        br.update(f, df, d)
    assert it <= 2 * n + 1
    assert np.max(np.abs(br.rho_in - rho_star)) < 1e-11


def test_broyden_without_history_is_linear_mixing():
    n = 5
    A, c, _ = _linear_problem(n, seed=8)
    br = S.Broyden(np.full(n, 5.0), 0.2, history=0)
    rho = np.full(n, 5.0)
    for _ in range(7):
        out = A @ br.rho_in + c
        eps, f, df, d = br.step(out)
        br.update(f, df, d)
        # history 0 restarts every pass: rho <- rho - zeta (rho - rho_out)
        rho = rho - 0.2 * (rho - (A @ rho + c))
        assert np.max(np.abs(br.rho_in - rho)) < 1e-12


def test_broyden_relative_norm():
    br = S.Broyden(np.array([2.0, 4.0]), 0.1, 8)
    eps, f, df, d = br.step(np.array([1.0, 4.5]))
    assert eps == pytest.approx(max(1.0 / 3.0, 0.5 / 8.5), rel=1e-15)
    assert np.array_equal(f, [1.0, -0.5]) and d == pytest.approx(1.25, rel=1e-15)


def test_gate_dominated_loop_stops_after_one_secant_step():
    # with the gate clamping phi to V_GS, rho_out does not depend on rho_in; the plain
    # mixing pass and one secant pass then land exactly on rho_out (third pass converged)
    req = W.sc_request(8, 6, V_DS=0.0, V_GS=0.2, n_c=8, n_r=12, tol=1e-9, zeta=0.3)
    req.elec.c_gate *= 1e9
    req.elec.eps_1d *= 1e-9
    res = S.self_consistent(req)
    assert res["converged"] and res["iterations"] == 3
    assert np.allclose(res["phi"], 0.2, atol=1e-9)
    ref = O.solve(S.negf_problem(req, np.full(6 * 8, -0.2)))
    assert np.max(np.abs(res["charge"] - ref["charge"])) < 1e-7


def test_potential_residual_is_the_poisson_difference():
    # phi(rho_out) - phi(rho_in) from two full solves (gate and drain terms included)
    # equals the homogeneous solve on f = rho_in - rho_out
    N = 41
    e = _elec(N, 3.0, V_DS=0.4, V_GS=-0.2)
    rng = np.random.default_rng(11)
    rho_in = e.n_ref + rng.normal(0, 0.05, N)
    rho_out = e.n_ref + rng.normal(0, 0.05, N)
    ref = S.poisson_rings(rho_out, e) - S.poisson_rings(rho_in, e)
    got = S.potential_residual(rho_in - rho_out, e)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_potential_residual_point_charge_closed_form():
    # one electron fewer on ring j0 (f = e_j0): psi_j = C r^|j-j0| with
    # C (2k(1-r) + c) = +e/dz, the potential rises where the electron left
    N, j0 = 101, 50
    e = _elec(N, 1.0)
    f = np.zeros(N)
    f[j0] = 1.0
    got = S.potential_residual(f, e)
    k, c = e.eps_1d / e.dz ** 2, e.c_gate
    q = 2.0 + c / k
    r = 0.5 * (q - np.sqrt(q * q - 4.0))
    C = (S.E_CHARGE / e.dz) / (2.0 * k * (1.0 - r) + c)
    ref = C * r ** np.abs(np.arange(N) - j0)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_grid_rebuild_happens_before_the_first_pass():
    # a semi-adaptive request whose only rebuild is the first one equals the
    # fixed-grid request on the grid built at the first potential by hand
    from dataclasses import replace

    from oracle import grid_oracle as G
    req = W.sc_request(8, 12, 0.3, 0.2, n_c=8, n_r=0, tol=1e-7, max_iter=4, grid_density=(1.0, 4.0, 2.0),
                       grid_limits=(-0.25, 0.05), grid_refresh=1000)
    U0 = S.ring_potential(S.poisson_rings(req.elec.n_ref, req.elec), req.device.b)
    E_r, w_r, _ = G.semi_adaptive_grid(S.negf_problem(req, U0), -0.25, 0.05, 3.0, 1.0, (1.0, 4.0, 2.0))
    fixed = replace(req, grid=W.EnergyGrid(req.grid.z_c, req.grid.w_c, E_r, w_r), grid_density=None)
    a, b = S.self_consistent(req), S.self_consistent(fixed)
    assert a["n_r"] == len(E_r) and a["iterations"] == b["iterations"]
    assert np.array_equal(a["U"], b["U"]) and a["trace"] == b["trace"]


def test_warm_start_from_the_fixed_point_stops_at_once():
    # starting from the converged rho_in reproduces that pass exactly: one pass, same U
    from dataclasses import replace
    req = W.sc_request(8, 12, 0.3, 0.2, n_c=8, n_r=12, tol=1e-8)
    cold = S.self_consistent(req)
    assert cold["converged"] and cold["iterations"] > 1
    warm = S.self_consistent(replace(req, rho_init=cold["rho_in"]))
    assert warm["iterations"] == 1 and warm["converged"]
    assert np.array_equal(warm["U"], cold["U"]) and warm["eps_max"] == cold["eps_max"]
