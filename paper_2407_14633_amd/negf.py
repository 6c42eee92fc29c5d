"""ctypes binding of libnegf.so (include/negf.h): argument marshalling only.

Every step of a solve runs in the library's HIP kernels; this module converts
numpy arrays / torch tensors to pointers and status codes to exceptions.  It
raises if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .workload import Bias, Device, EnergyGrid, Lead, Problem

LIB_PATH = os.environ.get("NEGF_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnegf.so")

NEGF_OK, NEGF_EINVAL, NEGF_ENOMEM, NEGF_ENOCONV, NEGF_ESINGULAR, NEGF_EHIP = 0, -1, -2, -3, -4, -5
NEGF_ETIMEDOUT = -6
NEGF_PENDING = 1
FP64, FP32_BULK = 0, 1
STATUS_NAMES = {0: "NEGF_OK", -1: "NEGF_EINVAL", -2: "NEGF_ENOMEM", -3: "NEGF_ENOCONV",
                -4: "NEGF_ESINGULAR", -5: "NEGF_EHIP", -6: "NEGF_ETIMEDOUT", 1: "NEGF_PENDING"}

EXPORTED = [
    "negf_default_options", "negf_create_device", "negf_set_potential", "negf_set_potential_dev",
    "negf_solve", "negf_solve_ex", "negf_solve_dev", "negf_sync", "negf_lead_self_energy",
    "negf_set_profiling", "negf_kernel_times", "negf_device_bytes", "negf_destroy", "negf_last_error",
    "negf_workspace_create", "negf_workspace_destroy", "negf_workspace_bytes", "negf_workspace_set_profiling",
    "negf_workspace_kernel_times", "negf_workspace_set_grid_scale", "negf_batch_solve", "negf_batch_solve_dev",
    "negf_batch_sync", "negf_workspace_set_order", "negf_workspace_set_lead_basis", "negf_workspace_autotune", "negf_graph_create",
    "negf_graph_launch", "negf_graph_sync", "negf_graph_destroy", "negf_server_create", "negf_server_submit",
    "negf_server_poll", "negf_server_stats", "negf_server_destroy", "negf_modes_create",
    "negf_modes_set_potential", "negf_modes_solve", "negf_modes_destroy", "negf_semi_adaptive_grid",
    "negf_solve_dev_static", "negf_static_scratch_bytes", "negf_fp64_nodes", "negf_workspace_fp64_nodes",
    "negf_set_fp64_recompute", "negf_workspace_set_fp64_recompute", "negf_workspace_set_chains_per_wave",
    "negf_server_evict", "negf_server_set_time_slice",
]


class NegfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class negf_lead(C.Structure):
    _fields_ = [("period", C.c_int), ("h_diag", C.c_void_p), ("h_up", C.c_void_p), ("tau", C.c_void_p)]


class negf_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("eta", C.c_double), ("decim_tol", C.c_double),
                ("decim_max_iter", C.c_int), ("g_s", C.c_double), ("workspace_bytes", C.c_size_t)]


class negf_bias(C.Structure):
    _fields_ = [("mu_L", C.c_double), ("mu_R", C.c_double), ("kT_L", C.c_double), ("kT_R", C.c_double)]


class negf_outputs(C.Structure):
    _fields_ = [("charge", C.c_void_p), ("T", C.c_void_p), ("current", C.c_void_p), ("gr_diag", C.c_void_p),
                ("al_diag", C.c_void_p), ("ar_diag", C.c_void_p), ("decim_iters", C.c_void_p),
                ("T_rl", C.c_void_p)]


class negf_job(C.Structure):
    _fields_ = [("dev", C.c_void_p), ("bias", negf_bias), ("n_c", C.c_int), ("z_c", C.c_void_p),
                ("w_c", C.c_void_p), ("n_r", C.c_int), ("E_r", C.c_void_p), ("w_r", C.c_void_p),
                ("charge", C.c_void_p), ("T", C.c_void_p), ("current", C.c_void_p),
                ("sigma_cache", C.c_void_p), ("sigma_mode", C.c_int), ("n_poles", C.c_int),
                ("contour_no_fermi", C.c_int), ("conductance", C.c_void_p)]


class negf_schedule(C.Structure):
    _fields_ = [("grid_scale", C.c_int), ("order", C.c_int), ("ms_per_solve", C.c_double),
                ("chains_per_wave", C.c_int * 25)]


class negf_sc_request(C.Structure):
    _fields_ = [("n_rings", C.c_int), ("b", C.c_int), ("h_diag", C.c_void_p), ("h_up", C.c_void_p),
                ("left", C.c_void_p), ("right", C.c_void_p), ("opt", negf_options), ("mu_S", C.c_double),
                ("kT", C.c_double), ("V_DS", C.c_double), ("V_GS", C.c_double), ("n_c", C.c_int),
                ("z_c", C.c_void_p), ("w_c", C.c_void_p), ("n_r", C.c_int), ("E_r", C.c_void_p),
                ("w_r", C.c_void_p), ("dz", C.c_double), ("eps_1d", C.c_double), ("c_gate", C.c_double),
                ("n_ref", C.c_void_p), ("zeta", C.c_double), ("tol", C.c_double), ("history", C.c_int),
                ("max_iter", C.c_int), ("basis", C.c_int), ("norm", C.c_int), ("grid_density", C.c_double * 3),
                ("grid_l1", C.c_double), ("grid_l2", C.c_double), ("grid_a", C.c_double), ("grid_b", C.c_double),
                ("grid_refresh", C.c_int), ("rho_init", C.c_void_p), ("deadline_ms", C.c_double)]


class negf_sc_result(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("eps_max", C.c_double), ("current", C.c_double),
                ("t_queue_ms", C.c_double), ("t_run_ms", C.c_double), ("t_total_ms", C.c_double),
                ("n_r", C.c_int), ("mode_space", C.c_int), ("evictions", C.c_int)]


class negf_server_info(C.Structure):
    _fields_ = [("pending", C.c_int), ("running", C.c_int), ("passes", C.c_longlong), ("hbm_used", C.c_size_t),
                ("hbm_budget", C.c_size_t), ("workspace_bytes", C.c_size_t)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libnegf.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2407_14633_amd.build`")
    lib = C.CDLL(path)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    lib.negf_default_options.argtypes = [C.POINTER(negf_options)]
    lib.negf_default_options.restype = None
    lib.negf_create_device.argtypes = [C.POINTER(vp), i, i, vp, vp, C.POINTER(negf_lead), C.POINTER(negf_lead),
                                       C.POINTER(negf_options)]
    lib.negf_set_potential.argtypes = [vp, vp, d, d]
    lib.negf_set_potential_dev.argtypes = [vp, vp, d, d, vp]
    lib.negf_solve.argtypes = [vp, C.POINTER(negf_bias), i, vp, vp, i, vp, vp, vp, vp, vp]
    lib.negf_solve_ex.argtypes = [vp, C.POINTER(negf_bias), i, vp, vp, i, vp, vp, C.POINTER(negf_outputs)]
    lib.negf_solve_dev.argtypes = [vp, C.POINTER(negf_bias), i, vp, vp, i, vp, vp, vp, vp, vp, vp]
    lib.negf_sync.argtypes = [vp]
    lib.negf_server_evict.argtypes = [vp, C.c_longlong]
    lib.negf_server_evict.restype = C.c_int
    lib.negf_server_set_time_slice.argtypes = [vp, i]
    lib.negf_server_set_time_slice.restype = C.c_int
    lib.negf_workspace_set_chains_per_wave.argtypes = [vp, i, i]
    lib.negf_workspace_set_chains_per_wave.restype = C.c_int
    lib.negf_set_fp64_recompute.argtypes = [vp, i]
    lib.negf_set_fp64_recompute.restype = C.c_int
    lib.negf_workspace_set_fp64_recompute.argtypes = [vp, i]
    lib.negf_workspace_set_fp64_recompute.restype = C.c_int
    lib.negf_fp64_nodes.argtypes = [vp, C.POINTER(i)]
    lib.negf_fp64_nodes.restype = C.c_int
    lib.negf_workspace_fp64_nodes.argtypes = [vp, i, C.POINTER(i)]
    lib.negf_workspace_fp64_nodes.restype = C.c_int
    lib.negf_solve_dev_static.argtypes = [vp, C.POINTER(negf_bias), i, vp, vp, i, vp, vp, vp, vp, vp, vp]
    lib.negf_solve_dev_static.restype = C.c_int
    lib.negf_static_scratch_bytes.argtypes = []
    lib.negf_static_scratch_bytes.restype = sz
    lib.negf_lead_self_energy.argtypes = [vp, i, i, vp, vp, vp]
    lib.negf_set_profiling.argtypes = [vp, i]
    lib.negf_kernel_times.argtypes = [vp, C.POINTER(C.c_char_p), C.POINTER(d), C.POINTER(i), C.POINTER(i)]
    lib.negf_device_bytes.argtypes = [vp]
    lib.negf_device_bytes.restype = sz
    lib.negf_destroy.argtypes = [vp]
    lib.negf_destroy.restype = None
    lib.negf_last_error.argtypes = []
    lib.negf_last_error.restype = C.c_char_p
    lib.negf_workspace_create.argtypes = [C.POINTER(vp), sz]
    lib.negf_workspace_destroy.argtypes = [vp]
    lib.negf_workspace_destroy.restype = None
    lib.negf_workspace_bytes.argtypes = [vp]
    lib.negf_workspace_bytes.restype = sz
    lib.negf_workspace_set_profiling.argtypes = [vp, i]
    lib.negf_workspace_kernel_times.argtypes = [vp, C.POINTER(C.c_char_p), C.POINTER(d), C.POINTER(i),
                                                C.POINTER(i)]
    lib.negf_workspace_set_grid_scale.argtypes = [vp, i]
    lib.negf_batch_solve.argtypes = [vp, i, C.POINTER(negf_job)]
    lib.negf_batch_solve_dev.argtypes = [vp, i, C.POINTER(negf_job), vp]
    lib.negf_batch_sync.argtypes = [vp, C.POINTER(i)]
    lib.negf_workspace_set_order.argtypes = [vp, i]
    lib.negf_workspace_set_lead_basis.argtypes = [vp, i]
    lib.negf_workspace_autotune.argtypes = [vp, i, C.POINTER(negf_job), vp, i, C.POINTER(negf_schedule)]
    lib.negf_graph_create.argtypes = [C.POINTER(vp), i, C.POINTER(negf_job), sz, vp]
    lib.negf_graph_launch.argtypes = [vp, vp]
    lib.negf_graph_sync.argtypes = [vp, C.POINTER(i)]
    lib.negf_graph_destroy.argtypes = [vp]
    lib.negf_graph_destroy.restype = None
    lib.negf_modes_create.argtypes = [C.POINTER(vp), i, i, vp, vp, C.POINTER(negf_lead), C.POINTER(negf_lead),
                                      C.POINTER(negf_options), i, vp]
    lib.negf_modes_set_potential.argtypes = [vp, vp, d, d]
    lib.negf_modes_solve.argtypes = [vp, vp, C.POINTER(negf_bias), i, vp, vp, i, vp, vp, vp, vp, vp]
    lib.negf_semi_adaptive_grid.argtypes = [vp, C.POINTER(negf_bias), d, d, d, d, vp, vp, vp, i, C.POINTER(i), vp]
    lib.negf_semi_adaptive_grid.restype = C.c_int
    lib.negf_modes_destroy.argtypes = [vp]
    lib.negf_modes_destroy.restype = None
    for name in ("negf_modes_create", "negf_modes_set_potential", "negf_modes_solve"):
        getattr(lib, name).restype = C.c_int
    lib.negf_server_create.argtypes = [C.POINTER(vp), sz, i, sz]
    lib.negf_server_submit.argtypes = [vp, C.POINTER(negf_sc_request), C.POINTER(C.c_longlong)]
    lib.negf_server_poll.argtypes = [vp, C.c_longlong, i, C.POINTER(negf_sc_result), vp, vp, vp]
    lib.negf_server_stats.argtypes = [vp, C.POINTER(negf_server_info)]
    lib.negf_server_destroy.argtypes = [vp]
    lib.negf_server_destroy.restype = None
    for name in ("negf_server_create", "negf_server_submit", "negf_server_poll", "negf_server_stats"):
        getattr(lib, name).restype = C.c_int
    for name in ("negf_workspace_set_order", "negf_workspace_set_lead_basis", "negf_workspace_autotune",
                 "negf_graph_create", "negf_graph_launch", "negf_graph_sync"):
        getattr(lib, name).restype = C.c_int
    for name in ("negf_workspace_create", "negf_workspace_set_profiling", "negf_workspace_kernel_times",
                 "negf_workspace_set_grid_scale", "negf_batch_solve", "negf_batch_solve_dev", "negf_batch_sync"):
        getattr(lib, name).restype = C.c_int
    for name in ("negf_create_device", "negf_set_potential", "negf_set_potential_dev", "negf_solve",
                 "negf_solve_ex", "negf_solve_dev", "negf_sync", "negf_lead_self_energy", "negf_set_profiling",
                 "negf_kernel_times"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != NEGF_OK:
        raise NegfError(status, load().negf_last_error().decode())


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_options() -> negf_options:
    o = negf_options()
    load().negf_default_options(C.byref(o))
    return o


@dataclass
class SolveResult:
    charge: np.ndarray
    T: np.ndarray
    current: float
    gr_diag: Optional[np.ndarray] = None
    al_diag: Optional[np.ndarray] = None
    ar_diag: Optional[np.ndarray] = None
    decim_iters: Optional[np.ndarray] = None
    conductance: Optional[float] = None
    fp64_nodes: int = 0
    T_rl: Optional[np.ndarray] = None


class NegfDevice:
    """One device handle (negf_create_device ... negf_destroy)."""

    def __init__(self, dev: Device, precision: int = FP64, eta: float = 1e-6, decim_tol: float = 1e-12,
                 decim_max_iter: int = 64, g_s: float = 2.0, workspace_bytes: int = 0):
        lib = load()
        self.N, self.b = dev.n_rings, dev.b
        self._keep = []
        hd = _c(dev.h_diag, np.complex128)
        hu = _c(dev.h_up, np.complex128) if dev.n_rings > 1 else None
        leads = [self._lead(dev.left), self._lead(dev.right)]
        o = default_options()
        o.precision, o.eta, o.decim_tol, o.decim_max_iter, o.g_s = precision, eta, decim_tol, decim_max_iter, g_s
        o.workspace_bytes = workspace_bytes
        h = C.c_void_p()
        _check(lib.negf_create_device(C.byref(h), self.N, self.b, _ptr(hd), _ptr(hu), C.byref(leads[0]),
                                      C.byref(leads[1]), C.byref(o)))
        self.h = h
        self.precision = precision
        self._keep = []

    def _lead(self, ld: Lead) -> negf_lead:
        arrs = [_c(ld.h_diag, np.complex128), _c(ld.h_up, np.complex128), _c(ld.tau, np.complex128)]
        self._keep.extend(arrs)
        return negf_lead(ld.period, *(a.ctypes.data_as(C.c_void_p) for a in arrs))

    def close(self):
        if getattr(self, "h", None):
            load().negf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- host API
    def set_potential(self, U: np.ndarray, U_left: float = 0.0, U_right: float = 0.0):
        U = _c(U, np.float64)
        if U.shape != (self.N * self.b,):
            raise ValueError(f"U must have shape ({self.N * self.b},)")
        _check(load().negf_set_potential(self.h, _ptr(U), float(U_left), float(U_right)))

    def solve(self, bias: Bias, grid: EnergyGrid, details: bool = False) -> SolveResult:
        zc, wc = _c(grid.z_c, np.complex128), _c(grid.w_c, np.complex128)
        Er, wr = _c(grid.E_r, np.float64), _c(grid.w_r, np.float64)
        nc, nr, nb = zc.shape[0], Er.shape[0], self.N * self.b
        charge = np.zeros(nb)
        T = np.zeros(nr)
        cur = np.zeros(1)
        out = negf_outputs(_ptr(charge), _ptr(T), _ptr(cur), None, None, None, None, None)
        gr = al = ar = it = trl = None
        if details:
            trl = np.zeros(nr)
            out.T_rl = _ptr(trl)
            gr = np.zeros((nc, nb), np.complex128)
            al = np.zeros((nr, nb))
            ar = np.zeros((nr, nb))
            it = np.zeros((nc + nr, 2), np.int32)
            out.gr_diag, out.al_diag, out.ar_diag, out.decim_iters = _ptr(gr), _ptr(al), _ptr(ar), _ptr(it)
        b = negf_bias(bias.mu_L, bias.mu_R, bias.kT_L, bias.kT_R)
        _check(load().negf_solve_ex(self.h, C.byref(b), nc, _ptr(zc), _ptr(wc), nr, _ptr(Er), _ptr(wr),
                                    C.byref(out)))
        return SolveResult(charge, T, float(cur[0]), gr, al, ar, it, fp64_nodes=self.fp64_nodes(), T_rl=trl)

    def lead_self_energy(self, lead: int, z: np.ndarray):
        z = _c(np.atleast_1d(z), np.complex128)
        sig = np.zeros((z.shape[0], self.b, self.b), np.complex128)
        it = np.zeros(z.shape[0], np.int32)
        _check(load().negf_lead_self_energy(self.h, int(lead), z.shape[0], _ptr(z), _ptr(sig), _ptr(it)))
        return sig, it

    # -------------------------------------------------------------- device API
    def solve_dev(self, bias: Bias, zc, wc, Er, wr, charge, T=None, current=None, stream=None):
        """Enqueues a solve on `stream` (torch.cuda.Stream or raw handle); tensors are device tensors."""
        b = negf_bias(bias.mu_L, bias.mu_R, bias.kT_L, bias.kT_R)
        s = _stream_handle(stream)
        nc = 0 if zc is None else int(zc.shape[0])
        nr = 0 if Er is None else int(Er.shape[0])
        _check(load().negf_solve_dev(self.h, C.byref(b), nc, _tp(zc), _tp(wc), nr, _tp(Er), _tp(wr), _tp(charge),
                                     _tp(T), _tp(current), s))

    def solve_dev_static(self, bias: Bias, zc, wc, Er, wr, charge, T=None, current=None, stream=None):
        """solve_dev with every work buffer in the library's fixed device area (no allocation)."""
        b = negf_bias(bias.mu_L, bias.mu_R, bias.kT_L, bias.kT_R)
        s = _stream_handle(stream)
        nc = 0 if zc is None else int(zc.shape[0])
        nr = 0 if Er is None else int(Er.shape[0])
        _check(load().negf_solve_dev_static(self.h, C.byref(b), nc, _tp(zc), _tp(wc), nr, _tp(Er), _tp(wr),
                                            _tp(charge), _tp(T), _tp(current), s))

    def sync(self):
        _check(load().negf_sync(self.h))

    def set_fp64_recompute(self, policy: int):
        """FP32-bulk: 0 recompute the marked real nodes in FP64, 1 all of them, 2 none."""
        _check(load().negf_set_fp64_recompute(self.h, int(policy)))

    def fp64_nodes(self) -> int:
        """FP32-bulk: real-axis nodes of the last solve that were recomputed in FP64."""
        n = C.c_int(0)
        _check(load().negf_fp64_nodes(self.h, C.byref(n)))
        return int(n.value)

    def set_profiling(self, on: bool):
        _check(load().negf_set_profiling(self.h, 1 if on else 0))

    def kernel_times(self) -> dict:
        return _kernel_times(load().negf_kernel_times, self.h)

    def device_bytes(self) -> int:
        return int(load().negf_device_bytes(self.h))

    def semi_adaptive_grid(self, bias: Bias, E_l1: float, E_l2: float, density, a: float = 3.0, b: float = 1.0):
        """Refined three-part real-axis grid: (E_r, w_r, (E_l1, E_l2, E_s))."""
        dens = _c(density, np.float64)
        bb = negf_bias(bias.mu_L, bias.mu_R, bias.kT_L, bias.kT_R)
        n = C.c_int(0)
        lim = np.zeros(3)
        # capacity: every part at the largest density over the whole window, plus one node per part
        width = abs(bias.mu_L - bias.mu_R) + 28.0 * max(bias.kT_L, bias.kT_R)
        cap = int(np.ceil(float(np.max(dens)) * width / min(bias.kT_L, bias.kT_R))) + 3
        E, w = np.zeros(cap), np.zeros(cap)
        _check(load().negf_semi_adaptive_grid(self.h, C.byref(bb), E_l1, E_l2, a, b, _ptr(dens), _ptr(E), _ptr(w),
                                              cap, C.byref(n), _ptr(lim)))
        return E[:n.value].copy(), w[:n.value].copy(), tuple(lim)


def static_scratch_bytes() -> int:
    """Size of the fixed device area used by NegfDevice.solve_dev_static."""
    return int(load().negf_static_scratch_bytes())


def _kernel_times(fn, h) -> dict:
    n = C.c_int(16)
    names = (C.c_char_p * 16)()
    ms = (C.c_double * 16)()
    calls = (C.c_int * 16)()
    _check(fn(h, names, ms, calls, C.byref(n)))
    return {names[k].decode(): (ms[k], calls[k]) for k in range(min(16, n.value))}


@dataclass
class Job:
    """One entry of a batch: a device handle, its bias and its energy grid (optionally
    with Fermi-pole residue nodes, a zero-temperature contour, and Eq. 6)."""
    dev: NegfDevice
    bias: Bias
    grid: EnergyGrid
    n_poles: int = 0
    contour_no_fermi: bool = False
    conductance: bool = False


class Workspace:
    """negf_workspace: batched solves of many devices in the same launches."""

    def __init__(self, store_bytes: int = 0):
        h = C.c_void_p()
        _check(load().negf_workspace_create(C.byref(h), int(store_bytes)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().negf_workspace_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def bytes(self) -> int:
        return int(load().negf_workspace_bytes(self.h))

    def set_profiling(self, on: bool):
        _check(load().negf_workspace_set_profiling(self.h, 1 if on else 0))

    def kernel_times(self) -> dict:
        return _kernel_times(load().negf_workspace_kernel_times, self.h)

    def set_grid_scale(self, scale: int):
        _check(load().negf_workspace_set_grid_scale(self.h, int(scale)))

    def solve(self, jobs) -> list:
        """Host-array batch (synchronous); returns one SolveResult per job."""
        keep, arr, res = [], (negf_job * len(jobs))(), []
        for k, jb in enumerate(jobs):
            g = jb.grid
            zc, wc = _c(g.z_c, np.complex128), _c(g.w_c, np.complex128)
            Er, wr = _c(g.E_r, np.float64), _c(g.w_r, np.float64)
            charge, T, cur, cond = np.zeros(jb.dev.N * jb.dev.b), np.zeros(Er.shape[0]), np.zeros(1), np.zeros(1)
            keep += [zc, wc, Er, wr]
            arr[k] = negf_job(jb.dev.h, negf_bias(jb.bias.mu_L, jb.bias.mu_R, jb.bias.kT_L, jb.bias.kT_R),
                              zc.shape[0], _ptr(zc), _ptr(wc), Er.shape[0], _ptr(Er), _ptr(wr), _ptr(charge),
                              _ptr(T), _ptr(cur), None, 0, int(jb.n_poles), int(bool(jb.contour_no_fermi)),
                              _ptr(cond) if jb.conductance else None)
            res.append(SolveResult(charge, T, 0.0))
            res[-1]._cur = cur
            res[-1]._cond = cond if jb.conductance else None
        _check(load().negf_batch_solve(self.h, len(jobs), arr))
        for r in res:
            r.current = float(r._cur[0])
            r.conductance = None if r._cond is None else float(r._cond[0])
            del r._cur, r._cond
        return res

    def solve_dev(self, jobs, stream=None):
        """Device batch: jobs are dicts with dev, bias, zc, wc, Er, wr, charge, T, current (tensors)."""
        arr = _dev_jobs(jobs)
        _check(load().negf_batch_solve_dev(self.h, len(jobs), arr, _stream_handle(stream)))

    def fp64_nodes(self, n_jobs: int) -> list:
        """Per job of the last batch: real-axis nodes recomputed in FP64 (FP32-bulk jobs)."""
        a = (C.c_int * max(1, n_jobs))()
        _check(load().negf_workspace_fp64_nodes(self.h, int(n_jobs), a))
        return [int(a[k]) for k in range(n_jobs)]

    def set_chains_per_wave(self, b: int, chains: int):
        """Chains per wavefront for ring size b (0: as many as fit)."""
        _check(load().negf_workspace_set_chains_per_wave(self.h, int(b), int(chains)))

    def set_order(self, order: int):
        _check(load().negf_workspace_set_order(self.h, int(order)))

    def set_lead_basis(self, ring_modes: int):
        """1: ring-circulant leads decimated in the ring Fourier basis; 0: dense layers."""
        _check(load().negf_workspace_set_lead_basis(self.h, int(ring_modes)))

    def autotune(self, jobs, stream=None, reps: int = 2) -> negf_schedule:
        """Times every schedule on these device jobs and keeps the fastest."""
        best = negf_schedule()
        _check(load().negf_workspace_autotune(self.h, len(jobs), _dev_jobs(jobs), _stream_handle(stream),
                                              int(reps), C.byref(best)))
        return best

    def sync(self) -> int:
        """Waits for the last device batch; raises on a device-side error (attribute .job names it)."""
        fj = C.c_int(-1)
        st = load().negf_batch_sync(self.h, C.byref(fj))
        if st != NEGF_OK:
            e = NegfError(st, load().negf_last_error().decode())
            e.job = fj.value
            raise e
        return fj.value


def _dev_jobs(jobs):
    arr = (negf_job * len(jobs))()
    for k, jb in enumerate(jobs):
        b = jb["bias"]
        zc, Er = jb.get("zc"), jb.get("Er")
        arr[k] = negf_job(jb["dev"].h, negf_bias(b.mu_L, b.mu_R, b.kT_L, b.kT_R),
                          0 if zc is None else int(zc.shape[0]), _tp(zc), _tp(jb.get("wc")),
                          0 if Er is None else int(Er.shape[0]), _tp(Er), _tp(jb.get("wr")),
                          _tp(jb["charge"]), _tp(jb.get("T")), _tp(jb.get("current")),
                          _tp(jb.get("sigma_cache")), int(jb.get("sigma_mode", 0)))
    return arr


class Graph:
    """negf_graph: one batch solve recorded into a HIP graph, replayed with one launch."""

    def __init__(self, jobs, stream, store_bytes: int = 0):
        h = C.c_void_p()
        _check(load().negf_graph_create(C.byref(h), len(jobs), _dev_jobs(jobs), int(store_bytes),
                                        _stream_handle(stream)))
        self.h = h

    def launch(self, stream):
        _check(load().negf_graph_launch(self.h, _stream_handle(stream)))

    def sync(self) -> int:
        fj = C.c_int(-1)
        st = load().negf_graph_sync(self.h, C.byref(fj))
        if st != NEGF_OK:
            e = NegfError(st, load().negf_last_error().decode())
            e.job = fj.value
            raise e
        return fj.value

    def close(self):
        if getattr(self, "h", None):
            load().negf_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _tp(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def solve_problem(p: Problem, precision: int = FP64, details: bool = False, fp64_recompute: int = 0,
                  **kw) -> SolveResult:
    """Creates a handle for p.device, sets the potential and solves p's grid."""
    with NegfDevice(p.device, precision=precision, eta=p.eta, decim_tol=p.decim_tol,
                    decim_max_iter=p.decim_max_iter, g_s=p.g_s, **kw) as d:
        d.set_potential(p.U, p.U_left, p.U_right)
        if fp64_recompute:
            d.set_fp64_recompute(fp64_recompute)
        return d.solve(p.bias, p.grid, details=details)


class Server:
    """negf_server: self-consistent bias-point requests with continuous batching."""

    def __init__(self, hbm_budget: int, max_inflight: int = 64, store_bytes: int = 0):
        h = C.c_void_p()
        _check(load().negf_server_create(C.byref(h), int(hbm_budget), int(max_inflight), int(store_bytes)))
        self.h = h
        self._sizes = {}

    def submit(self, req, precision: int = FP64) -> int:
        """req: workload.ScRequest (its basis, norm and semi-adaptive grid settings
        included).  Returns the request id."""
        dev, g, e = req.device, req.grid, req.elec
        keep = []

        def arr(a, dt):
            a = _c(a, dt)
            keep.append(a)
            return _ptr(a)

        def lead(ld):
            return negf_lead(ld.period, arr(ld.h_diag, np.complex128), arr(ld.h_up, np.complex128),
                             arr(ld.tau, np.complex128))

        L, R = lead(dev.left), lead(dev.right)
        o = default_options()
        o.precision, o.eta, o.decim_tol, o.decim_max_iter, o.g_s = (precision, req.eta, req.decim_tol,
                                                                      req.decim_max_iter, req.g_s)
        r = negf_sc_request(dev.n_rings, dev.b, arr(dev.h_diag, np.complex128), arr(dev.h_up, np.complex128),
                            C.cast(C.pointer(L), C.c_void_p), C.cast(C.pointer(R), C.c_void_p), o,
                            req.bias.mu_L, req.bias.kT_L, e.V_DS, e.V_GS, g.n_c, arr(g.z_c, np.complex128),
                            arr(g.w_c, np.complex128), g.n_r, arr(g.E_r, np.float64), arr(g.w_r, np.float64),
                            e.dz, e.eps_1d, e.c_gate, arr(e.n_ref, np.float64), req.zeta, req.tol, req.history,
                            req.max_iter, req.basis, req.norm)
        if req.grid_density is not None:
            for p in range(3):
                r.grid_density[p] = float(req.grid_density[p])
            r.grid_l1, r.grid_l2 = (float(v) for v in req.grid_limits)
            r.grid_a, r.grid_b = float(req.grid_a), float(req.grid_b)
            r.grid_refresh = int(req.grid_refresh)
        if req.rho_init is not None:
            r.rho_init = arr(np.asarray(req.rho_init, np.float64), np.float64)
        r.deadline_ms = float(req.deadline_ms)
        rid = C.c_longlong()
        _check(load().negf_server_submit(self.h, C.byref(r), C.byref(rid)))
        self._sizes[rid.value] = (dev.n_rings * dev.b, req.max_iter)
        return rid.value

    def poll(self, rid: int, wait: bool = True):
        """dict(status, iterations, eps_max, current, t_queue_ms, t_run_ms, t_total_ms, charge, U),
        or None while the request runs (wait=False)."""
        nb, mi = self._sizes.get(rid, (0, 0))
        res = negf_sc_result()
        charge, U, tr = np.zeros(nb), np.zeros(nb), np.zeros(max(mi, 1))
        st = load().negf_server_poll(self.h, C.c_longlong(rid), 1 if wait else 0, C.byref(res), _ptr(charge),
                                     _ptr(U), _ptr(tr))
        if st == NEGF_PENDING:
            return None
        _check(st)
        self._sizes.pop(rid, None)
        return dict(status=res.status, iterations=res.iterations, eps_max=res.eps_max, current=res.current,
                    t_queue_ms=res.t_queue_ms, t_run_ms=res.t_run_ms, t_total_ms=res.t_total_ms, charge=charge,
                    U=U, trace=tr[:res.iterations].copy(), n_r=res.n_r, mode_space=bool(res.mode_space),
                    evictions=res.evictions)

    def evict(self, rid: int):
        """Evicts request rid to host state at the end of its next pass; it is queued again
        and resumes from that state (results bit-identical to an uninterrupted run)."""
        _check(load().negf_server_evict(self.h, C.c_longlong(rid)))

    def set_time_slice(self, passes: int):
        """Evict running requests after this many passes while others wait (0: never)."""
        _check(load().negf_server_set_time_slice(self.h, int(passes)))

    def stats(self) -> dict:
        info = negf_server_info()
        st = load().negf_server_stats(self.h, C.byref(info))
        return dict(status=st, pending=info.pending, running=info.running, passes=info.passes,
                    hbm_used=info.hbm_used, hbm_budget=info.hbm_budget, workspace_bytes=info.workspace_bytes)

    def close(self):
        if getattr(self, "h", None):
            load().negf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class ModeSpace:
    """negf_modes: a ring-circulant tube as independent scalar mode chains."""

    def __init__(self, dev: Device, modes=None, precision: int = FP64, eta: float = 1e-6,
                 decim_tol: float = 1e-12, decim_max_iter: int = 64, g_s: float = 2.0):
        self.N, self.b = dev.n_rings, dev.b
        keep = []

        def arr(a):
            a = _c(a, np.complex128)
            keep.append(a)
            return _ptr(a)

        leads = [negf_lead(ld.period, arr(ld.h_diag), arr(ld.h_up), arr(ld.tau)) for ld in (dev.left, dev.right)]
        o = default_options()
        o.precision, o.eta, o.decim_tol, o.decim_max_iter, o.g_s = precision, eta, decim_tol, decim_max_iter, g_s
        ml = None if modes is None else _c(modes, np.int32)
        h = C.c_void_p()
        _check(load().negf_modes_create(C.byref(h), self.N, self.b, arr(dev.h_diag),
                                        arr(dev.h_up) if self.N > 1 else None, C.byref(leads[0]), C.byref(leads[1]),
                                        C.byref(o), 0 if ml is None else int(ml.shape[0]), _ptr(ml)))
        self.h = h

    def set_potential(self, U_ring, U_left: float = 0.0, U_right: float = 0.0):
        U = _c(U_ring, np.float64)
        if U.shape != (self.N,):
            raise ValueError(f"U_ring must have shape ({self.N},)")
        _check(load().negf_modes_set_potential(self.h, _ptr(U), float(U_left), float(U_right)))

    def solve(self, ws: "Workspace", bias: Bias, grid: EnergyGrid) -> SolveResult:
        zc, wc = _c(grid.z_c, np.complex128), _c(grid.w_c, np.complex128)
        Er, wr = _c(grid.E_r, np.float64), _c(grid.w_r, np.float64)
        charge, T, cur = np.zeros(self.N * self.b), np.zeros(Er.shape[0]), np.zeros(1)
        b = negf_bias(bias.mu_L, bias.mu_R, bias.kT_L, bias.kT_R)
        _check(load().negf_modes_solve(self.h, ws.h, C.byref(b), zc.shape[0], _ptr(zc), _ptr(wc), Er.shape[0],
                                       _ptr(Er), _ptr(wr), _ptr(charge), _ptr(T), _ptr(cur)))
        return SolveResult(charge, T, float(cur[0]))

    def close(self):
        if getattr(self, "h", None):
            load().negf_modes_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
