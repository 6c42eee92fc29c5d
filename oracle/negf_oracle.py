"""Plain CPU FP64 oracle for the per-energy NEGF solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library: it is written directly from the paper's equations with
numpy / scipy (LAPACK) primitives in complex128, slowly and without any
blocking, fusion or reordering beyond what the definitions state.

What it computes, per energy node z (paper Section 2.2.1):

* Lead self-energies (Eq. 2): Sigma_l = tau_l g_l tau_l^H, with the surface
  Green's function g_l obtained by Sancho-Rubio iterative layer doubling
  (Section 2.2.2 names decimation as the default procedure).  The lead's
  principal layer is assembled densely from its ring description.
* M(z) = z I - H - diag(U) - Sigma_L - Sigma_R, block tridiagonal (Eq. 2).
* Real-axis nodes z = E + i eta: the two lead block columns of G = M^{-1} by a
  banded LU solve (the plain definition), giving the diagonals of
  A_l = G Gamma_l G^H (Eq. 3) and T_LR = Tr[Gamma_L G Gamma_R G^H] (Eq. 5).
* Contour nodes: the diagonal blocks of G^R from the two-sided recursion
  of Algorithms 1-2 (x from the right, y from the left, G_TT = (a-x-y)^{-1}),
  with the paper's block vectors rewritten in blocks of M (see below).
* The weighted energy sums of Eq. 4 (charge) and the Landauer current.

Readings taken where the paper is ambiguous (each is listed in the design doc):
  - blocks are those of M: a_j = M_jj, up_j = M_{j,j+1} = -H_{j,j+1},
    lo_j = M_{j+1,j} = -H_{j+1,j}; Algorithm 2's recursions hold in this form;
  - the x recursion runs backward from N-2, the y recursion forward from 1;
  - charge is an electron count per atom including spin (g_s = 2);
  - the contour integrand uses the analytic complex Fermi function of the
    lowest chemical potential; the current uses T_LR.

Parity pins for every function live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

E_CHARGE = 1.602176634e-19     # C (exact, SI 2019)
H_PLANCK = 6.62607015e-34      # J s (exact, SI 2019)
G0_PER_SPIN = E_CHARGE ** 2 / H_PLANCK   # e^2/h in A/V


class OracleNoConvergence(RuntimeError):
    pass


# ---------------------------------------------------------------- leads ----
def lead_principal_layer(period, h_diag, h_up, U_lead):
    """Dense (h00, h01) of a lead's principal layer of `period` rings.

    h00 is block tridiagonal over the rings of one cell (on-site blocks plus the
    lead potential on the diagonal); h01 couples the last ring of a cell to the
    first ring of the next cell, so only its (period-1, 0) block is non-zero.
    """
    h_diag = np.asarray(h_diag, np.complex128)
    h_up = np.asarray(h_up, np.complex128)
    b = h_diag.shape[1]
    m = period * b
    h00 = np.zeros((m, m), np.complex128)
    h01 = np.zeros((m, m), np.complex128)
    for r in range(period):
        s = slice(r * b, (r + 1) * b)
        h00[s, s] = h_diag[r] + U_lead * np.eye(b)
        if r + 1 < period:
            s1 = slice((r + 1) * b, (r + 2) * b)
            h00[s, s1] = h_up[r]
            h00[s1, s] = h_up[r].conj().T
    h01[(period - 1) * b:, :b] = h_up[period - 1]
    return h00, h01


def surface_green(h00, h01, z, tol=1e-12, max_iter=64):
    """Sancho-Rubio layer doubling for the surface Green's function.

    eps_s <- h00, eps <- h00, alpha <- h01, beta <- h01^H; repeat
    g = (z - eps)^{-1}; eps_s += alpha g beta; eps += alpha g beta + beta g alpha;
    alpha <- alpha g alpha; beta <- beta g beta; until max|alpha|, max|beta| < tol.
    Returns (g_s = (z - eps_s)^{-1}, number of doubling steps).
    """
    m = h00.shape[0]
    eye = np.eye(m)
    eps_s = h00.copy()
    eps = h00.copy()
    alpha = h01.copy()
    beta = h01.conj().T.copy()
    for it in range(1, max_iter + 1):
        g = np.linalg.inv(z * eye - eps)
        agb = alpha @ g @ beta
        bga = beta @ g @ alpha
        eps_s = eps_s + agb
        eps = eps + agb + bga
        alpha = alpha @ g @ alpha
        beta = beta @ g @ beta
        if np.max(np.abs(alpha)) < tol and np.max(np.abs(beta)) < tol:
            return np.linalg.inv(z * eye - eps_s), it
    raise OracleNoConvergence(f"decimation did not converge in {max_iter} steps at z={z}")


def self_energy(lead, U_lead, z, tol=1e-12, max_iter=64):
    """Sigma = tau g_s[ring 0] tau^H (Eq. 2, tau = H_{device edge, lead ring 0})."""
    h00, h01 = lead_principal_layer(lead.period, lead.h_diag, lead.h_up, U_lead)
    gs, it = surface_green(h00, h01, z, tol, max_iter)
    b = lead.tau.shape[0]
    tau = np.asarray(lead.tau, np.complex128)
    return tau @ gs[:b, :b] @ tau.conj().T, it


def broadening(sigma):
    """Gamma = i (Sigma - Sigma^H)."""
    return 1j * (sigma - sigma.conj().T)


# --------------------------------------------------------------- device ----
def matrix_blocks(dev, U, z, sig_L, sig_R):
    """Blocks of M = z I - H - diag(U) - Sigma_L - Sigma_R."""
    N, b = dev.h_diag.shape[0], dev.h_diag.shape[1]
    Ub = np.asarray(U, np.float64).reshape(N, b)
    a = np.empty((N, b, b), np.complex128)
    for j in range(N):
        a[j] = z * np.eye(b) - dev.h_diag[j] - np.diag(Ub[j])
    a[0] -= sig_L
    a[N - 1] -= sig_R
    up = -np.asarray(dev.h_up, np.complex128)
    lo = -np.conj(np.transpose(np.asarray(dev.h_up, np.complex128), (0, 2, 1)))
    return a, up, lo


def dense_matrix(a, up, lo):
    """The full M from its blocks (small systems only)."""
    N, b = a.shape[0], a.shape[1]
    M = np.zeros((N * b, N * b), np.complex128)
    for j in range(N):
        M[j * b:(j + 1) * b, j * b:(j + 1) * b] = a[j]
        if j + 1 < N:
            M[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = up[j]
            M[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = lo[j]
    return M


def banded_solve(a, up, lo, rhs):
    """Solve M X = rhs with LAPACK's banded LU (partial pivoting), bandwidth 2b-1."""
    N, b = a.shape[0], a.shape[1]
    n = N * b
    kl = ku = 2 * b - 1
    ab = np.zeros((kl + ku + 1, n), np.complex128)

    def put(i0, j0, blk):
        ii, jj = np.meshgrid(np.arange(b) + i0, np.arange(b) + j0, indexing="ij")
        ab[ku + ii - jj, jj] = blk

    for j in range(N):
        put(j * b, j * b, a[j])
        if j + 1 < N:
            put(j * b, (j + 1) * b, up[j])
            put((j + 1) * b, j * b, lo[j])
    return solve_banded((kl, ku), ab, rhs)


def lead_columns(a, up, lo):
    """Block columns 0 and N-1 of G = M^{-1}: returns (G[:,0], G[:,N-1]) as (N,b,b) each."""
    N, b = a.shape[0], a.shape[1]
    rhs = np.zeros((N * b, 2 * b), np.complex128)
    rhs[:b, :b] = np.eye(b)
    rhs[(N - 1) * b:, b:] = np.eye(b)
    X = banded_solve(a, up, lo, rhs)
    return X[:, :b].reshape(N, b, b), X[:, b:].reshape(N, b, b)


def diag_block_plain(a, up, lo, n):
    """G_nn by a banded solve against the unit vectors of block n (plain definition)."""
    N, b = a.shape[0], a.shape[1]
    rhs = np.zeros((N * b, b), np.complex128)
    rhs[n * b:(n + 1) * b, :] = np.eye(b)
    X = banded_solve(a, up, lo, rhs)
    return X[n * b:(n + 1) * b, :]


def diag_blocks_two_sided(a, up, lo):
    """All G_nn from the left/right connected recursions (Algorithms 1-2).

    y_0 = 0,    y_n = lo_{n-1} (a_{n-1} - y_{n-1})^{-1} up_{n-1}       (n = 1..N-1)
    x_{N-1} = 0, x_n = up_n (a_{n+1} - x_{n+1})^{-1} lo_n              (n = N-2..0)
    G_nn = (a_n - x_n - y_n)^{-1}.
    """
    N, b = a.shape[0], a.shape[1]
    y = np.zeros((N, b, b), np.complex128)
    x = np.zeros((N, b, b), np.complex128)
    for n in range(1, N):
        y_tilde = np.linalg.inv(a[n - 1] - y[n - 1]) @ up[n - 1]
        y[n] = lo[n - 1] @ y_tilde
    for n in range(N - 2, -1, -1):
        x_tilde = np.linalg.inv(a[n + 1] - x[n + 1]) @ lo[n]
        x[n] = up[n] @ x_tilde
    G = np.empty((N, b, b), np.complex128)
    for n in range(N):
        G[n] = np.linalg.inv(a[n] - x[n] - y[n])
    return G


def spectral_diag(Gcol, gamma):
    """diag(G_{n,k} Gamma G_{n,k}^H) for every block n, flattened to (N*b,)."""
    return np.real(np.einsum("nij,jk,nik->ni", Gcol, gamma, Gcol.conj())).reshape(-1)


def transmission(G0N, gam_L, gam_R):
    """T_LR = Tr[Gamma_L G_{0,N-1} Gamma_R G_{0,N-1}^H] (Eq. 5)."""
    return float(np.real(np.trace(gam_L @ G0N @ gam_R @ G0N.conj().T)))


# ----------------------------------------------------------- occupations ----
def fermi(E, mu, kT):
    """Real Fermi function 1/(1+exp((E-mu)/kT)), overflow-safe and to full
    relative precision on both sides (exp(-x)/(1+exp(-x)) for x > 0)."""
    x = (np.asarray(E, np.float64) - mu) / kT
    e = np.exp(-np.abs(x))
    return np.where(x > 0, e, 1.0) / (1.0 + e)


def fermi_difference(E, mu_L, kT_L, mu_R, kT_R):
    """f_L(E) - f_R(E) of Eq. 5 without cancellation.

    With x_l = (E - mu_l)/kT_l the identity
        f(x_L) - f(x_R) = -expm1(x_L - x_R) f(x_L) f(-x_R)
    holds exactly (f(-x) = 1 - f(x)); every factor is computed to full relative
    precision, where the plain difference of two Fermi factors close to 1 (E far
    below both levels, where in-band transmissions are of order one) loses all
    but a few digits.  Beyond |x_L - x_R| > 700 the factors are far apart and the
    plain difference is used.
    """
    E = np.asarray(E, np.float64)
    xL = (E - mu_L) / kT_L
    xR = (E - mu_R) / kT_R
    d = xL - xR
    far = np.abs(d) > 700.0
    dd = np.where(far, 0.0, d)
    out = -np.expm1(dd) * fermi(E, mu_L, kT_L) * fermi(-E, -mu_R, kT_R)
    return np.where(far, fermi(E, mu_L, kT_L) - fermi(E, mu_R, kT_R), out)


def fermi_complex(z, mu, kT):
    """Analytic continuation 1/(1+exp((z-mu)/kT)) for complex z, overflow-safe."""
    u = (np.asarray(z, np.complex128) - mu) / kT
    out = np.empty_like(u)
    pos = u.real > 0
    e = np.exp(-u[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(u[~pos]))
    return out


# ----------------------------------------------------------------- solve ----
def energy_point_real(prob, E):
    """Per-energy real-axis quantities: (A_L diag, A_R diag, T_LR, decim iters)."""
    z = E + 1j * prob.eta
    sL, itL = self_energy(prob.device.left, prob.U_left, z, prob.decim_tol, prob.decim_max_iter)
    sR, itR = self_energy(prob.device.right, prob.U_right, z, prob.decim_tol, prob.decim_max_iter)
    a, up, lo = matrix_blocks(prob.device, prob.U, z, sL, sR)
    G0, GN = lead_columns(a, up, lo)
    gL, gR = broadening(sL), broadening(sR)
    return spectral_diag(G0, gL), spectral_diag(GN, gR), transmission(GN[0], gL, gR), (itL, itR)


def energy_point_contour(prob, z):
    """Per-energy contour quantity: diag G^R(z), flattened to (N*b,)."""
    sL, _ = self_energy(prob.device.left, prob.U_left, z, prob.decim_tol, prob.decim_max_iter)
    sR, _ = self_energy(prob.device.right, prob.U_right, z, prob.decim_tol, prob.decim_max_iter)
    a, up, lo = matrix_blocks(prob.device, prob.U, z, sL, sR)
    G = diag_blocks_two_sided(a, up, lo)
    return np.einsum("nii->ni", G).reshape(-1).copy()


def reduce_energies(prob, gr_diag, AL, AR, T):
    """Eq. 4 charge (electrons per atom incl. spin) and the Landauer current (A).

    charge_i = g_s [ -(1/pi) sum_c Im(w_c F_min(z_c) G^R_ii(z_c))
                     + (1/2pi) sum_r w_r (f_L A_L,ii + f_R A_R,ii) ]
    current  = g_s (e^2/h) sum_r w_r T_LR(E_r) (f_L - f_R)
    """
    b = prob.bias
    g = prob.grid
    mu_min, kT_min = min(b.mu_L, b.mu_R), min(b.kT_L, b.kT_R)
    nb = prob.U.shape[0]
    charge = np.zeros(nb)
    if g.n_c:
        coef = g.w_c * fermi_complex(g.z_c, mu_min, kT_min)
        charge += -(1.0 / np.pi) * np.imag(coef[:, None] * gr_diag).sum(axis=0)
    current = 0.0
    if g.n_r:
        fL = fermi(g.E_r, b.mu_L, b.kT_L)
        fR = fermi(g.E_r, b.mu_R, b.kT_R)
        charge += (1.0 / (2 * np.pi)) * ((g.w_r * fL)[:, None] * AL + (g.w_r * fR)[:, None] * AR).sum(axis=0)
        dF = fermi_difference(g.E_r, b.mu_L, b.kT_L, b.mu_R, b.kT_R)
        current = prob.g_s * G0_PER_SPIN * float(np.sum(g.w_r * T * dF))
    return prob.g_s * charge, current


def solve(prob, details=False):
    """Full oracle solve of a Problem: returns dict(charge, T, current[, per-energy arrays])."""
    g = prob.grid
    nb = prob.U.shape[0]
    gr = np.zeros((g.n_c, nb), np.complex128)
    for c in range(g.n_c):
        gr[c] = energy_point_contour(prob, g.z_c[c])
    AL = np.zeros((g.n_r, nb))
    AR = np.zeros((g.n_r, nb))
    T = np.zeros(g.n_r)
    iters = np.zeros((g.n_r, 2), np.int64)
    for r in range(g.n_r):
        AL[r], AR[r], T[r], iters[r] = energy_point_real(prob, g.E_r[r])
    charge, current = reduce_energies(prob, gr, AL, AR, T)
    out = dict(charge=charge, T=T, current=current)
    if details:
        out.update(gr_diag=gr, AL=AL, AR=AR, decim_iters=iters)
    return out
