"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments before touching the HIP runtime."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2407_14633_amd import negf as NG
from paper_2407_14633_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "negf.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(negf_[a-z0-9_]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(NG.LIB_PATH):
        pytest.fail("libnegf.so is not built (run `python -m paper_2407_14633_amd.build`)")
    return NG.load()


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    assert set(NG.EXPORTED) == set(syms)


def test_default_options(lib):
    o = NG.default_options()
    assert (o.precision, o.eta, o.decim_tol, o.decim_max_iter, o.g_s, o.workspace_bytes) == (0, 1e-6, 1e-12, 64, 2.0, 0)


def _create(lib, N=4, b=3, period=2, h_diag="ok", h_up="ok", left="ok", right="ok", opt=None, out="ok"):
    dev = W.random_device(max(N, 2), min(max(b, 1), 24), seed=1, period=period)
    hd = np.ascontiguousarray(dev.h_diag)
    hu = np.ascontiguousarray(dev.h_up)
    keep = []

    def mk(ld, mode):
        if mode is None:
            return None
        arrs = [np.ascontiguousarray(ld.h_diag), np.ascontiguousarray(ld.h_up), np.ascontiguousarray(ld.tau)]
        keep.extend(arrs)
        l = NG.negf_lead(ld.period, *(a.ctypes.data_as(C.c_void_p) for a in arrs))
        if mode == "badperiod":
            l.period = 3
        if mode == "zeroperiod":
            l.period = 0
        if mode == "nulltau":
            l.tau = None
        return C.byref(l)

    h = C.c_void_p()
    o = NG.default_options()
    for k, v in (opt or {}).items():
        setattr(o, k, v)
    st = lib.negf_create_device(C.byref(h) if out == "ok" else None, N, b,
                                hd.ctypes.data_as(C.c_void_p) if h_diag == "ok" else None,
                                hu.ctypes.data_as(C.c_void_p) if h_up == "ok" else None,
                                mk(dev.left, left), mk(dev.right, right), C.byref(o))
    return st, h


@pytest.mark.parametrize("kw,frag", [
    (dict(N=0), "n_rings"),
    (dict(b=0), "ring size"),
    (dict(b=25), "ring size"),
    (dict(h_diag=None), "h_diag"),
    (dict(h_up=None), "h_up"),
    (dict(left=None), "left lead"),
    (dict(right="badperiod"), "period"),      # a principal layer of more than two rings
    (dict(left="zeroperiod"), "period"),
    (dict(left="nulltau"), "NULL block"),
    (dict(opt=dict(precision=7)), "precision"),
    (dict(opt=dict(decim_tol=0.0)), "decim_tol"),
    (dict(opt=dict(decim_max_iter=0)), "decim_max_iter"),
    (dict(opt=dict(eta=-1.0)), "eta"),
    (dict(opt=dict(g_s=0.0)), "g_s"),
    (dict(out=None), "out"),
])
def test_create_rejects_bad_arguments(lib, kw, frag):
    st, h = _create(lib, **kw)
    assert st == NG.NEGF_EINVAL
    assert frag in lib.negf_last_error().decode()
    assert not h.value


def test_create_rejects_non_finite_hamiltonian(lib):
    dev = W.random_device(3, 2, seed=2)
    dev.h_diag[1, 0, 1] = np.nan
    with pytest.raises(NG.NegfError) as e:
        NG.NegfDevice(dev)
    assert e.value.status == NG.NEGF_EINVAL


def test_null_handle_calls_are_rejected(lib):
    b = NG.negf_bias(0.1, -0.1, 0.0259, 0.0259)
    z = np.zeros(4, np.complex128)
    assert lib.negf_set_potential(None, z.ctypes.data_as(C.c_void_p), 0.0, 0.0) == NG.NEGF_EINVAL
    assert lib.negf_solve(None, C.byref(b), 0, None, None, 4, z.ctypes.data_as(C.c_void_p),
                          z.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), None, None) == NG.NEGF_EINVAL
    assert lib.negf_sync(None) == NG.NEGF_EINVAL
    assert lib.negf_lead_self_energy(None, 0, 1, None, None, None) == NG.NEGF_EINVAL
    assert lib.negf_set_profiling(None, 1) == NG.NEGF_EINVAL
    assert lib.negf_device_bytes(None) == 0
    lib.negf_destroy(None)


def test_host_validation_errors_without_a_gpu(lib, monkeypatch):
    """Argument checks of negf_solve run before any HIP call (a fake handle is never dereferenced
    for these cases because validation fails first)."""
    b = NG.negf_bias(0.1, -0.1, 0.0, 0.0259)   # kT_L = 0 is invalid
    fake = C.c_void_p(1)
    E = np.zeros(4)
    charge = np.zeros(4)
    st = lib.negf_solve(fake, C.byref(b), 0, None, None, 4, E.ctypes.data_as(C.c_void_p),
                        E.ctypes.data_as(C.c_void_p), charge.ctypes.data_as(C.c_void_p), None, None)
    assert st == NG.NEGF_EINVAL and "kT" in lib.negf_last_error().decode()
    b = NG.negf_bias(0.1, -0.1, 0.0259, 0.0259)
    st = lib.negf_solve(fake, C.byref(b), 0, None, None, 0, None, None, charge.ctypes.data_as(C.c_void_p), None, None)
    assert st == NG.NEGF_EINVAL and "no energy nodes" in lib.negf_last_error().decode()
    st = lib.negf_solve(fake, C.byref(b), 2, None, None, 0, None, None, charge.ctypes.data_as(C.c_void_p), None, None)
    assert st == NG.NEGF_EINVAL and "contour" in lib.negf_last_error().decode()
    st = lib.negf_solve(fake, C.byref(b), 0, None, None, 4, E.ctypes.data_as(C.c_void_p),
                        E.ctypes.data_as(C.c_void_p), None, None, None)
    assert st == NG.NEGF_EINVAL and "charge" in lib.negf_last_error().decode()
    st = lib.negf_solve(fake, C.byref(b), -1, None, None, 4, E.ctypes.data_as(C.c_void_p),
                        E.ctypes.data_as(C.c_void_p), charge.ctypes.data_as(C.c_void_p), None, None)
    assert st == NG.NEGF_EINVAL and "negative" in lib.negf_last_error().decode()
    st = lib.negf_lead_self_energy(fake, 2, 1, E.ctypes.data_as(C.c_void_p), E.ctypes.data_as(C.c_void_p), None)
    assert st == NG.NEGF_EINVAL and "lead" in lib.negf_last_error().decode()


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_2407_14633_amd.negf")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            mod.load(str(tmp_path / "nope.so"))
    finally:
        mod._lib = saved


# ---- later entry points: argument checks that run before any HIP call ----
def test_batch_and_graph_reject_null(lib):
    assert lib.negf_batch_solve(None, 1, None) == NG.NEGF_EINVAL
    assert lib.negf_batch_solve_dev(None, 1, None, None) == NG.NEGF_EINVAL
    assert lib.negf_batch_sync(None, None) == NG.NEGF_EINVAL
    assert lib.negf_workspace_create(None, 0) == NG.NEGF_EINVAL
    assert lib.negf_workspace_set_grid_scale(None, 2) == NG.NEGF_EINVAL
    assert lib.negf_workspace_set_order(None, 0) == NG.NEGF_EINVAL
    assert lib.negf_workspace_set_lead_basis(None, 1) == NG.NEGF_EINVAL
    assert lib.negf_graph_create(None, 1, None, 0, None) == NG.NEGF_EINVAL
    assert lib.negf_graph_launch(None, None) == NG.NEGF_EINVAL
    assert lib.negf_graph_sync(None, None) == NG.NEGF_EINVAL
    assert lib.negf_workspace_bytes(None) == 0


def test_server_rejects_null(lib):
    assert lib.negf_server_create(None, 1 << 30, 4, 0) == NG.NEGF_EINVAL
    rid = C.c_longlong()
    assert lib.negf_server_submit(None, None, C.byref(rid)) == NG.NEGF_EINVAL
    assert lib.negf_server_poll(None, 1, 0, None, None, None, None) == NG.NEGF_EINVAL
    assert lib.negf_server_stats(None, None) == NG.NEGF_EINVAL
    assert lib.negf_server_evict(None, 1) == NG.NEGF_EINVAL
    assert lib.negf_server_set_time_slice(None, 2) == NG.NEGF_EINVAL


def test_modes_and_grid_reject_bad_arguments(lib):
    assert lib.negf_modes_create(None, 4, 3, None, None, None, None, None, 0, None) == NG.NEGF_EINVAL
    h = C.c_void_p()
    dev = W.random_device(4, 3, seed=2)        # not circulant: refused before any allocation
    keep = [np.ascontiguousarray(a) for a in (dev.h_diag, dev.h_up, dev.left.h_diag, dev.left.h_up,
                                               dev.left.tau, dev.right.h_diag, dev.right.h_up, dev.right.tau)]
    p = [k.ctypes.data_as(C.c_void_p) for k in keep]
    L = NG.negf_lead(dev.left.period, p[2], p[3], p[4])
    R = NG.negf_lead(dev.right.period, p[5], p[6], p[7])
    assert lib.negf_modes_create(C.byref(h), 4, 3, p[0], p[1], C.byref(L), C.byref(R), None, 0, None) == NG.NEGF_EINVAL
    assert "circulant" in lib.negf_last_error().decode()
    assert lib.negf_modes_set_potential(None, None, 0.0, 0.0) == NG.NEGF_EINVAL
    n = C.c_int()
    assert lib.negf_semi_adaptive_grid(None, None, 0.0, 0.0, 3.0, 1.0, None, None, None, 0, C.byref(n), None) \
        == NG.NEGF_EINVAL


def test_fp64_recompute_policy_rejected_without_gpu_work(lib):
    assert lib.negf_set_fp64_recompute(None, 0) == NG.NEGF_EINVAL
    assert lib.negf_workspace_set_fp64_recompute(None, 1) == NG.NEGF_EINVAL
    n = C.c_int(7)
    assert lib.negf_fp64_nodes(None, C.byref(n)) == NG.NEGF_EINVAL
