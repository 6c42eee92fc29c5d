"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module builds *inputs only*: tight-binding ring blocks of zigzag carbon
nanotubes, lead descriptions, on-site potential profiles, quadrature nodes and
weights for the energy integrals, and bias points.  It holds none of the
Green's-function arithmetic (no inversion, no self-energy, no Fermi factor);
both the CPU oracle and the HIP library receive the arrays built here.

Conventions
-----------
* A device has ``N`` rings of ``b`` atoms; atom ``i`` of ring ``j`` has flat
  index ``j*b + i``.  ``h_diag[j]`` is the on-site block ``H_{j,j}`` (potential
  excluded), ``h_up[j] = H_{j,j+1}``; ``H_{j+1,j} = h_up[j]^H``.
* A lead is a semi-infinite, periodic continuation of the ring chain, listed
  *outward* from the device: lead ring 0 touches the device, ring 1 is next,
  and so on.  ``period`` rings form one unit cell; ``h_diag[r]`` is the block of
  lead ring r, ``h_up[r] = H_{ring r, ring r+1}`` (for r = period-1 it couples
  to ring 0 of the next cell), and ``tau = H_{device edge ring, lead ring 0}``.
* Zigzag (n,0) nanotube (the paper's material, Section 3.1: (17,0) tube with a
  2.5 eV nearest-neighbour coupling): rings carry no intra-ring bond, and ring
  couplings alternate between a two-bond block ``t (I + S^T)`` and a one-bond
  block ``t I``, ``S`` being the cyclic shift of the ring.  Ring ``j``'s outgoing
  coupling is the two-bond one for even ``j``.
* Energies are in eV.  Quadrature weights include the Jacobian ``dE/dx``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

T_CC = -2.5          # nearest-neighbour pz coupling (eV), Section 3.1
KT_300K = 0.0259     # kT at room temperature (eV)
FERMI_TAIL = 14.0    # f1 = f2 = 14, Eq. 4


# --------------------------------------------------------------------------
# Containers
# --------------------------------------------------------------------------
@dataclass
class Lead:
    period: int
    h_diag: np.ndarray        # (period, b, b) complex128
    h_up: np.ndarray          # (period, b, b) complex128
    tau: np.ndarray           # (b, b) complex128


@dataclass
class Device:
    h_diag: np.ndarray        # (N, b, b) complex128
    h_up: np.ndarray          # (N-1, b, b) complex128
    left: Lead
    right: Lead

    @property
    def n_rings(self) -> int:
        return self.h_diag.shape[0]

    @property
    def b(self) -> int:
        return self.h_diag.shape[1]


@dataclass
class Bias:
    mu_L: float
    mu_R: float
    kT_L: float = KT_300K
    kT_R: float = KT_300K


@dataclass
class EnergyGrid:
    z_c: np.ndarray           # (n_c,) complex contour nodes
    w_c: np.ndarray           # (n_c,) complex weights (dz Jacobian x Gauss weight)
    E_r: np.ndarray           # (n_r,) real-axis nodes
    w_r: np.ndarray           # (n_r,) real weights

    @property
    def n_c(self) -> int:
        return int(self.z_c.shape[0])

    @property
    def n_r(self) -> int:
        return int(self.E_r.shape[0])


@dataclass
class Problem:
    """One complete solve: device, potential, bias, energy grid, options."""
    name: str
    device: Device
    U: np.ndarray             # (N*b,) per-atom potential energy (eV)
    U_left: float
    U_right: float
    bias: Bias
    grid: EnergyGrid
    eta: float = 1e-6
    decim_tol: float = 1e-12
    decim_max_iter: int = 64
    g_s: float = 2.0
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# Zigzag nanotube Hamiltonian blocks
# --------------------------------------------------------------------------
def ring_shift(n: int) -> np.ndarray:
    """Cyclic shift S with S[i, (i+1) mod n] = 1."""
    S = np.zeros((n, n))
    S[np.arange(n), (np.arange(n) + 1) % n] = 1.0
    return S


def zigzag_coupling(n: int, j: int, t: float = T_CC) -> np.ndarray:
    """H_{j,j+1} of a zigzag (n,0) tube: two bonds per atom for even j, one for odd j."""
    if j % 2 == 0:
        return (t * (np.eye(n) + ring_shift(n).T)).astype(np.complex128)
    return (t * np.eye(n)).astype(np.complex128)


def zigzag_cnt(n: int, N: int, t: float = T_CC) -> Device:
    """Device of N rings of an (n,0) tube with leads that continue the ring parity."""
    if N < 1 or n < 1:
        raise ValueError("need n >= 1 atoms per ring and N >= 1 rings")
    h_diag = np.zeros((N, n, n), np.complex128)
    h_up = np.stack([zigzag_coupling(n, j, t) for j in range(N - 1)]) if N > 1 \
        else np.zeros((0, n, n), np.complex128)
    # right lead: device ring N + r is lead ring r
    right = Lead(period=2,
                 h_diag=np.zeros((2, n, n), np.complex128),
                 h_up=np.stack([zigzag_coupling(n, N, t), zigzag_coupling(n, N + 1, t)]),
                 tau=zigzag_coupling(n, N - 1, t))
    # left lead: device ring -1 - r is lead ring r; H_{-1-r,-2-r} = H_{-2-r,-1-r}^H
    left = Lead(period=2,
                h_diag=np.zeros((2, n, n), np.complex128),
                h_up=np.stack([zigzag_coupling(n, -2, t).conj().T,
                               zigzag_coupling(n, -3, t).conj().T]),
                tau=zigzag_coupling(n, -1, t).conj().T)
    return Device(h_diag=h_diag, h_up=h_up, left=left, right=right)


def random_device(N: int, b: int, seed: int, period: int = 1, scale: float = 1.0,
                  complex_couplings: bool = True) -> Device:
    """A generic Hermitian block-tridiagonal device with random periodic leads.

    Used for brute-force checks on tiny systems: nothing in it is nanotube-specific.
    """
    rng = np.random.default_rng(seed)

    def herm(m):
        a = rng.normal(size=(m, m)) + (1j * rng.normal(size=(m, m)) if complex_couplings else 0)
        return (scale * 0.5 * (a + a.conj().T)).astype(np.complex128)

    def gen(m):
        a = rng.normal(size=(m, m)) + (1j * rng.normal(size=(m, m)) if complex_couplings else 0)
        return (scale * a).astype(np.complex128)

    def lead():
        return Lead(period=period,
                    h_diag=np.stack([herm(b) for _ in range(period)]),
                    h_up=np.stack([gen(b) for _ in range(period)]),
                    tau=gen(b))

    h_diag = np.stack([herm(b) for _ in range(N)])
    h_up = np.stack([gen(b) for _ in range(N - 1)]) if N > 1 else np.zeros((0, b, b), np.complex128)
    return Device(h_diag=h_diag, h_up=h_up, left=lead(), right=lead())


def gershgorin_lower(dev: Device, U: np.ndarray) -> float:
    """Lower Gershgorin bound of the device plus leads (used to start the contour)."""
    N, b = dev.n_rings, dev.b
    diag = np.real(np.einsum("jii->ji", dev.h_diag)).reshape(-1) + U
    off = np.abs(dev.h_diag).sum(axis=2).reshape(-1) - np.abs(np.einsum("jii->ji", dev.h_diag)).reshape(-1)
    for j in range(N - 1):
        off[j * b:(j + 1) * b] += np.abs(dev.h_up[j]).sum(axis=1)
        off[(j + 1) * b:(j + 2) * b] += np.abs(dev.h_up[j]).sum(axis=0)
    off[:b] += np.abs(dev.left.tau).sum(axis=1)
    off[(N - 1) * b:] += np.abs(dev.right.tau).sum(axis=1)
    rows = diag - off
    lo = rows.min()
    for ld in (dev.left, dev.right):
        for r in range(ld.period):
            d = np.real(np.diag(ld.h_diag[r]))
            o = np.abs(ld.h_diag[r]).sum(axis=1) - np.abs(np.diag(ld.h_diag[r]))
            o = o + np.abs(ld.h_up[r]).sum(axis=1) + np.abs(ld.h_up[r - 1]).sum(axis=0)
            if r == 0:
                o = o + np.abs(ld.tau).sum(axis=0)
            lo = min(lo, (d - o).min())
    return float(lo)


# --------------------------------------------------------------------------
# Potential profiles (per atom, eV)
# --------------------------------------------------------------------------
def potential_smooth_ring(N: int, b: int, amplitude: float, seed: int) -> np.ndarray:
    """Ring-uniform smooth profile that vanishes at both contacts.

    s_j = sum_{m=1..4} (a_m/m) sin(pi m (j+1)/(N+1)), a_m ~ U(-1,1);
    U_j = amplitude * s_j / max|s|.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=4)
    j = np.arange(N)
    s = sum((a[m - 1] / m) * np.sin(np.pi * m * (j + 1) / (N + 1)) for m in range(1, 5))
    s = amplitude * s / np.max(np.abs(s))
    return np.repeat(s, b).astype(np.float64)


def potential_tanh_barrier(N: int, b: int, seed: int, height_range=(0.2, 0.5),
                           width: float = 10.0, noise: float = 0.01) -> tuple[np.ndarray, float]:
    """Gate-like barrier between N/4 and 3N/4 plus per-atom Gaussian noise.

    U_{j,i} = U_b/2 [tanh((j - N/4)/w) - tanh((j - 3N/4)/w)] + N(0, noise^2).
    Returns (U, U_b).
    """
    rng = np.random.default_rng(seed)
    Ub = float(rng.uniform(*height_range))
    j = np.arange(N, dtype=np.float64)
    prof = 0.5 * Ub * (np.tanh((j - N / 4) / width) - np.tanh((j - 3 * N / 4) / width))
    U = np.repeat(prof, b) + rng.normal(0.0, noise, size=N * b)
    return U.astype(np.float64), Ub


# --------------------------------------------------------------------------
# Quadrature grids
# --------------------------------------------------------------------------
def gauss_legendre(n: int) -> tuple[np.ndarray, np.ndarray]:
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def real_axis_gl(E_lo: float, E_hi: float, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes/weights on [E_lo, E_hi]."""
    if n == 0:
        return np.zeros(0), np.zeros(0)
    x, w = gauss_legendre(n)
    half, mid = 0.5 * (E_hi - E_lo), 0.5 * (E_hi + E_lo)
    return mid + half * x, half * w


def real_axis_midpoint(E_lo: float, E_hi: float, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Uniform midpoint rule on [E_lo, E_hi]."""
    h = (E_hi - E_lo) / n
    return E_lo + (np.arange(n) + 0.5) * h, np.full(n, h)


def semicircle_contour(E_b: float, E_top: float, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre rule on the upper semicircle from E_b to E_top.

    z(theta) = c + R exp(i theta), c = (E_b+E_top)/2, R = (E_top-E_b)/2, theta in (0, pi).
    Returned weights w_k integrate f along the path from E_b to E_top:
    sum_k w_k f(z_k) ~ int_{E_b}^{E_top} f dz, i.e. w_k = -i R e^{i theta_k} (pi/2) omega_k.
    """
    if n == 0:
        return np.zeros(0, np.complex128), np.zeros(0, np.complex128)
    x, w = gauss_legendre(n)
    c, R = 0.5 * (E_b + E_top), 0.5 * (E_top - E_b)
    th = 0.5 * np.pi * (x + 1.0)
    z = c + R * np.exp(1j * th)
    wz = -1j * R * np.exp(1j * th) * (0.5 * np.pi) * w
    return z.astype(np.complex128), wz.astype(np.complex128)


def window(bias: Bias, tail: float = FERMI_TAIL) -> tuple[float, float]:
    """(E_min, E_max) of Eq. 4: mu_min - f1 kT_min, mu_max + f2 kT_max."""
    E_min = min(bias.mu_L, bias.mu_R) - tail * min(bias.kT_L, bias.kT_R)
    E_max = max(bias.mu_L, bias.mu_R) + tail * max(bias.kT_L, bias.kT_R)
    return E_min, E_max


def nonequilibrium_grid(E_b: float, bias: Bias, n_c: int, n_r: int,
                        tail: float = FERMI_TAIL) -> EnergyGrid:
    """Contour part on [E_b, E_min] plus Gauss-Legendre real axis on [E_min, E_max]."""
    E_min, E_max = window(bias, tail)
    z_c, w_c = semicircle_contour(E_b, E_min, n_c)
    E_r, w_r = real_axis_gl(E_min, E_max, n_r)
    return EnergyGrid(z_c, w_c, E_r, w_r)


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------
def small_problem(seed: int = 1234) -> Problem:
    """(8,0) tube, 64 rings, smooth ring-uniform potential in [-0.3,0.3] eV,
    256 uniform real-axis energies in [-1,1] eV, V = 0.1 V, kT = 0.0259 eV."""
    n, N = 8, 64
    dev = zigzag_cnt(n, N)
    U = potential_smooth_ring(N, n, 0.3, seed)
    E, w = real_axis_midpoint(-1.0, 1.0, 256)
    grid = EnergyGrid(np.zeros(0, np.complex128), np.zeros(0, np.complex128), E, w)
    bias = Bias(mu_L=0.05, mu_R=-0.05)
    return Problem("cnt8_N64_real256", dev, U, 0.0, 0.0, bias, grid,
                   meta=dict(n=n, N=N, seed=seed))


def device_problem(N: int = 400, n: int = 17, seed: int = 2024, n_c: int = 512,
                   n_r: int = 1536, V: float = 0.3) -> Problem:
    """(17,0) tube with a tanh gate barrier, 512 contour + 1536 real-axis points,
    source/drain mu = +/- V/2 (default +/-0.15 eV)."""
    dev = zigzag_cnt(n, N)
    U, Ub = potential_tanh_barrier(N, n, seed)
    bias = Bias(mu_L=0.5 * V, mu_R=-0.5 * V)
    E_b = gershgorin_lower(dev, U) - 1.0
    grid = nonequilibrium_grid(E_b, bias, n_c, n_r)
    return Problem(f"cnt{n}_N{N}_c{n_c}_r{n_r}", dev, U, 0.0, 0.0, bias, grid,
                   meta=dict(n=n, N=N, seed=seed, U_b=Ub, E_b=E_b))


def subsample_grid(grid: EnergyGrid, n_c: int, n_r: int, seed: int) -> EnergyGrid:
    """A fixed random subset of a grid's nodes (weights kept as they are)."""
    rng = np.random.default_rng(seed)
    ic = np.sort(rng.choice(grid.n_c, size=min(n_c, grid.n_c), replace=False)) if grid.n_c else np.zeros(0, int)
    ir = np.sort(rng.choice(grid.n_r, size=min(n_r, grid.n_r), replace=False)) if grid.n_r else np.zeros(0, int)
    return EnergyGrid(grid.z_c[ic], grid.w_c[ic], grid.E_r[ir], grid.w_r[ir])


def with_grid(p: Problem, grid: EnergyGrid, name: Optional[str] = None) -> Problem:
    return Problem(name or p.name + "_sub", p.device, p.U, p.U_left, p.U_right, p.bias, grid,
                   p.eta, p.decim_tol, p.decim_max_iter, p.g_s, dict(p.meta))


def batch_problems(n_dev: int = 64, seed: int = 4040, chiralities=(10, 13, 17, 20, 23),
                   N_range=(200, 2000), ne_range=(512, 4096), contour_frac: float = 0.25,
                   V: float = 0.3) -> list:
    """Many zigzag tubes of uneven chirality, length and node count: n drawn
    from `chiralities`, N uniform in N_range, node count uniform in ne_range
    (a quarter on the contour, the rest on the real axis), each with its own
    tanh gate barrier."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_dev):
        n = int(rng.choice(chiralities))
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        ne = int(rng.integers(ne_range[0], ne_range[1] + 1))
        n_c = int(round(contour_frac * ne))
        out.append(device_problem(N=N, n=n, seed=int(seed * 1000 + k), n_c=n_c, n_r=ne - n_c, V=V))
    return out


# --------------------------------------------------------------------------
# Self-consistent bias points (serving requests)
# --------------------------------------------------------------------------
EPS0 = 8.8541878128e-12      # F/m
RING_SPACING = 0.1065e-9     # m, mean axial ring spacing of a zigzag tube (Table 1 mesh spacing)
LATTICE_A = 0.246e-9         # m, graphene lattice constant


@dataclass
class Electrostatics:
    """1-D finite-difference Poisson along the tube axis with a coaxial gate.

    Per ring j (potential phi_j in V, extra electrons rho_j - n_ref_j):
      -(eps_1d/dz^2)(phi_{j+1} - 2 phi_j + phi_{j-1}) + c_gate (phi_j - V_GS)
          = -e (rho_j - n_ref_j) / dz,
    phi_{-1} = 0 (source), phi_N = V_DS (drain); electron potential energy U_j = -phi_j (eV).
    """
    dz: float                 # m
    eps_1d: float             # F m
    c_gate: float             # F/m
    n_ref: np.ndarray         # (N,) electrons per ring of the neutral tube
    V_DS: float               # V
    V_GS: float               # V


@dataclass
class ScRequest:
    """One self-consistent bias point: device, grid, electrostatics, mixing settings."""
    name: str
    device: Device
    bias: Bias                # mu_L = source level, mu_R = mu_L - V_DS
    grid: EnergyGrid
    elec: Electrostatics
    eta: float = 1e-6
    decim_tol: float = 1e-12
    decim_max_iter: int = 64
    g_s: float = 2.0
    zeta: float = 0.1         # Broyden fraction
    tol: float = 1e-5         # stop when max_j |f_j / (rho_in_j + rho_out_j)| < tol
    history: int = 8
    max_iter: int = 100
    basis: int = 0            # 0: mode space when every block is ring-circulant; 1: real space
    norm: int = 0             # 0: relative charge change (Algorithm 3); 1: potential residual (eV)
    grid_density: Optional[tuple] = None   # (d1, d2, d3) nodes per kT: semi-adaptive real-axis grid
    grid_limits: tuple = (0.0, 0.0)        # guessed E_l1, E_l2 of every rebuild (eV)
    grid_a: float = 3.0
    grid_b: float = 1.0
    grid_refresh: int = 50    # NEGF passes between rebuilds (the first before pass 1)
    rho_init: Optional[np.ndarray] = None  # (N,) starting per-ring electron counts (warm start); None: n_ref
    deadline_ms: float = 0.0  # > 0: the server ends the request after this long (NEGF_ETIMEDOUT)
    meta: dict = field(default_factory=dict)

    @property
    def U_left(self) -> float:
        return 0.0

    @property
    def U_right(self) -> float:
        return -self.elec.V_DS


def cnt_electrostatics(n: int, N: int, V_DS: float, V_GS: float, kappa: float = 3.9,
                       t_ox: float = 10e-9) -> Electrostatics:
    """Coaxial gate around an (n,0) tube: r = d/2, d = a n / pi; c_gate = 2 pi eps0 kappa /
    ln((r + t_ox)/r); eps_1d = eps0 kappa pi ((r + t_ox)^2 - r^2) (axial flux through the
    oxide annulus); one electron per atom in the neutral tube."""
    r = 0.5 * LATTICE_A * n / np.pi
    c_gate = 2.0 * np.pi * EPS0 * kappa / np.log((r + t_ox) / r)
    eps_1d = EPS0 * kappa * np.pi * ((r + t_ox) ** 2 - r ** 2)
    return Electrostatics(RING_SPACING, float(eps_1d), float(c_gate), np.full(N, float(n)), float(V_DS),
                          float(V_GS))


def sc_request(n: int, N: int, V_DS: float, V_GS: float, n_c: int, n_r: int, mu_S: float = 0.0,
               name: Optional[str] = None, **kw) -> ScRequest:
    """A flat zigzag tube at a bias point; the contour starts well below any band
    the gate or drain can pull down."""
    dev = zigzag_cnt(n, N)
    bias = Bias(mu_L=mu_S, mu_R=mu_S - V_DS)
    E_b = -3.0 * abs(T_CC) - abs(V_DS) - abs(V_GS) - 1.0
    grid = nonequilibrium_grid(E_b, bias, n_c, n_r)
    return ScRequest(name or f"sc_cnt{n}_N{N}_Vds{V_DS:.3f}_Vgs{V_GS:.3f}", dev, bias, grid,
                     cnt_electrostatics(n, N, V_DS, V_GS), meta=dict(n=n, N=N), **kw)


def serving_requests(n_req: int, seed: int = 5555, chiralities=(10, 13, 17, 20, 23), N_range=(200, 2000),
                     ne_range=(512, 4096), contour_frac: float = 0.25, eta: float = 1e-6, adaptive: bool = True,
                     norm: int = 1, tol: float = 1e-6, grid_refresh: int = 50, **kw) -> list:
    """Requests drawn like the batching workload, with V_DS ~ U[0, 0.6] and V_GS ~ U[-0.5, 0.5].

    The drawn energy count ne sets the contour part (contour_frac of it) and the
    real-axis budget n_r = ne - n_c.  adaptive: the real axis is the semi-adaptive
    grid (Section 3.3) with densities (1, 2, 1) x n_r kT / (E_max - E_min) nodes
    per kT in its three parts, guessed limits (mu_R, mu_L), rebuilt before the
    first pass and every grid_refresh passes; otherwise n_r fixed Gauss-Legendre
    nodes.  norm = 1, tol = 1e-6: stop when the output charge would move the
    potential by less than 1e-6 eV."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_req):
        n = int(rng.choice(chiralities))
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        ne = int(rng.integers(ne_range[0], ne_range[1] + 1))
        n_c = int(round(contour_frac * ne))
        V_DS = float(rng.uniform(0.0, 0.6))
        V_GS = float(rng.uniform(-0.5, 0.5))
        n_r = ne - n_c
        if adaptive:
            r = sc_request(n, N, V_DS, V_GS, n_c, 0, eta=eta, norm=norm, tol=tol, **kw)
            E_min, E_max = window(r.bias)
            kT = min(r.bias.kT_L, r.bias.kT_R)
            rho = n_r * kT / (E_max - E_min)
            r.grid_density = (rho, 2.0 * rho, rho)
            r.grid_limits = (min(r.bias.mu_L, r.bias.mu_R), max(r.bias.mu_L, r.bias.mu_R))
            r.grid_refresh = grid_refresh
        else:
            r = sc_request(n, N, V_DS, V_GS, n_c, n_r, eta=eta, norm=norm, tol=tol, **kw)
        out.append(r)
    return out


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of `rate` requests per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# --------------------------------------------------------------------------
# Equilibrium grids
# --------------------------------------------------------------------------
def equilibrium_grid(E_b: float, mu: float, kT: float, n_arc: int, n_line: int, n_poles: int = 8,
                     start: float = 10.0, end: float = 40.0) -> tuple[EnergyGrid, int]:
    """Contour for the equilibrium density with Fermi-pole residues.

    The path leaves E_b on a circle centred on the real axis, reaches
    P = (mu - start kT) + i delta with delta = 2 n_poles pi kT (half-way between the
    n_poles-th and the next pole of F), and runs horizontally to (mu + end kT) + i delta.
    On that line F(z - mu) equals the real Fermi function of Re z, so both pieces
    are smooth; the n_poles poles below the line are returned for the residue sum.
    Nodes are Gauss-Legendre on each piece; weights include dz/dt."""
    delta = 2.0 * n_poles * np.pi * kT
    xp = mu - start * kT
    c = (xp * xp + delta * delta - E_b * E_b) / (2.0 * (xp - E_b))
    R = c - E_b
    th_p = np.arctan2(delta, xp - c)
    x, w = gauss_legendre(n_arc)
    t = 0.5 * (x + 1.0)
    th = np.pi + (th_p - np.pi) * t
    z_a = c + R * np.exp(1j * th)
    w_a = 1j * R * np.exp(1j * th) * (th_p - np.pi) * 0.5 * w
    x, w = gauss_legendre(n_line)
    t = 0.5 * (x + 1.0)
    x_end = mu + end * kT
    z_l = xp + 1j * delta + t * (x_end - xp)
    w_l = (x_end - xp) * 0.5 * w + 0j
    grid = EnergyGrid(np.concatenate([z_a, z_l]).astype(np.complex128),
                      np.concatenate([w_a, w_l]).astype(np.complex128), np.zeros(0), np.zeros(0))
    return grid, int(n_poles)


def neutral_grid(E_b: float, n_c: int) -> EnergyGrid:
    """Arc from E_b to 0 (the reference density rho_0 integrates up to E = 0)."""
    z_c, w_c = semicircle_contour(E_b, 0.0, n_c)
    return EnergyGrid(z_c, w_c, np.zeros(0), np.zeros(0))


def conductance_grid(mu: float, kT: float, n_r: int, tail: float = FERMI_TAIL) -> EnergyGrid:
    """Gauss-Legendre real-axis nodes on [mu - f kT, mu + f kT] for Eq. 6."""
    E_r, w_r = real_axis_gl(mu - tail * kT, mu + tail * kT, n_r)
    return EnergyGrid(np.zeros(0, np.complex128), np.zeros(0, np.complex128), E_r, w_r)
