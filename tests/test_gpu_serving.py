"""Serving loop: self-consistent bias points with continuous batching on the GPU.

* Parity: a request's converged potential, charge and current match the CPU
  self-consistency oracle (same Algorithm 3 passes, FP64 NEGF oracle).
* Isolation: a request gives bit-identical results alone and among other
  requests that arrive while it runs.
* Admission: a budget that fits one request at a time serialises them; a
  request larger than the budget is refused at submission.
"""
import sys
from dataclasses import replace
import time

import numpy as np
import pytest

from oracle import sc_oracle as S
from paper_2407_14633_amd import workload as W

pytestmark = pytest.mark.gpu

GIB = 1 << 30


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_request(n=8, N=24, V_DS=0.2, V_GS=0.3, n_c=16, n_r=40, **kw):
    kw.setdefault("tol", 1e-8)
    return W.sc_request(n, N, V_DS, V_GS, n_c=n_c, n_r=n_r, **kw)


@pytest.mark.parametrize("case", [(8, 24, 0.2, 0.3, 0), (10, 30, 0.4, -0.3, 0), (8, 300, 0.2, 0.3, 0),
                                  (8, 300, 0.2, 0.3, 1)])
def test_server_matches_oracle(gpu_lib, case):
    # the 300-ring cases are longer than the self-consistency workgroup (256 threads),
    # so its Poisson scans run with several rings per thread
    negf = gpu_lib
    n, N, vds, vgs, norm = case
    req = (small_request(n, N, vds, vgs) if N < 100 else
           small_request(n, N, vds, vgs, n_c=8, n_r=16, norm=norm, tol=1e-8 if norm == 0 else 1e-7))
    say("sc request", req.name)
    ref = S.self_consistent(req)
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        got = srv.poll(srv.submit(req))
    say("passes gpu/oracle", got["iterations"], ref["iterations"], "eps", got["eps_max"], ref["eps_max"])
    assert got["status"] == negf.NEGF_OK and ref["converged"]
    assert got["iterations"] == ref["iterations"]
    dU = np.max(np.abs(got["U"] - ref["U"]))
    dq = np.max(np.abs(got["charge"] - ref["charge"])) / np.max(np.abs(ref["charge"]))
    dI = abs(got["current"] - ref["current"]) / max(abs(ref["current"]), 1e-30)
    say("dU", dU, "dq", dq, "dI", dI, "mode space", got["mode_space"])
    assert got["mode_space"]          # zigzag tubes are ring-circulant: the exact mode-space route
    assert dU < 1e-9 and dq < 1e-10 and dI < 1e-6


def test_server_mode_space_equals_real_space(gpu_lib):
    negf = gpu_lib
    req = small_request(13, 28, 0.35, 0.2)
    rs = replace(req, basis=1)
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        m = srv.poll(srv.submit(req))
        r = srv.poll(srv.submit(rs))
    dU = np.max(np.abs(m["U"] - r["U"]))
    dq = np.max(np.abs(m["charge"] - r["charge"])) / np.max(np.abs(r["charge"]))
    dI = abs(m["current"] - r["current"]) / abs(r["current"])
    say("modes/real passes", m["iterations"], r["iterations"], "dU", dU, "dq", dq, "dI", dI)
    assert m["mode_space"] and not r["mode_space"]
    assert m["status"] == r["status"] == negf.NEGF_OK
    assert m["iterations"] == r["iterations"]
    assert dU < 1e-10 and dq < 1e-10 and dI < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_server_potential_stop_and_grid_refresh_match_oracle(gpu_lib, precision):
    # eta = 1e-6, the 1e-6 eV potential-residual stop and a semi-adaptive grid
    # rebuilt before passes 1, 3, 5, ... (every 2 passes, so that several rebuilds
    # run inside the few passes of a small request)
    negf = gpu_lib
    tol = 1e-9 if precision == "fp64" else 1e-6
    req = small_request(10, 30, 0.4, -0.3, n_r=0, eta=1e-6, norm=1, tol=tol, grid_density=(2.0, 12.0, 4.0),
                        grid_limits=(-0.3, 0.1), grid_refresh=2)
    say("sc request", req.name, "eta", req.eta, "norm", req.norm, precision)
    ref = S.self_consistent(req)
    prec = negf.FP64 if precision == "fp64" else negf.FP32_BULK
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        got = srv.poll(srv.submit(req, precision=prec))
    dU = np.max(np.abs(got["U"] - ref["U"]))
    dq = np.max(np.abs(got["charge"] - ref["charge"])) / np.max(np.abs(ref["charge"]))
    dI = abs(got["current"] - ref["current"]) / max(abs(ref["current"]), 1e-30)
    say("passes gpu/oracle", got["iterations"], ref["iterations"], "n_r", got["n_r"], ref["n_r"], "eps",
        got["eps_max"], ref["eps_max"], "dU", dU, "dq", dq, "dI", dI)
    assert got["status"] == negf.NEGF_OK and ref["converged"] and got["mode_space"]
    assert got["n_r"] == ref["n_r"]
    assert ref["eps_max"] < tol and got["eps_max"] < tol
    if precision == "fp64":
        assert got["iterations"] == ref["iterations"]
        assert dU < 1e-9 and dq < 1e-10 and dI < 1e-6
    else:
        assert abs(got["iterations"] - ref["iterations"]) <= 2
        assert dU < 1e-5 and dq < 1e-5 and dI < 1e-4


def test_server_alone_and_in_mix_bitwise(gpu_lib):
    negf = gpu_lib
    target = small_request(10, 26, 0.3, 0.1, tol=1e-9)
    others = [small_request(8, 20, 0.1, -0.2), small_request(13, 18, 0.5, 0.4, n_c=12, n_r=30),
              small_request(10, 40, 0.25, 0.0, n_c=20, n_r=36)]
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        alone = srv.poll(srv.submit(target))
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        ids = [srv.submit(others[0])]
        time.sleep(0.05)
        tid = srv.submit(target)
        ids += [srv.submit(o) for o in others[1:]]
        mixed = srv.poll(tid)
        rest = [srv.poll(i) for i in ids]
    say("alone passes", alone["iterations"], "mixed", mixed["iterations"], [r["iterations"] for r in rest])
    assert alone["status"] == mixed["status"] == negf.NEGF_OK
    assert alone["iterations"] == mixed["iterations"]
    assert np.array_equal(alone["U"], mixed["U"])
    assert np.array_equal(alone["charge"], mixed["charge"])
    assert alone["current"] == mixed["current"]
    assert all(r["status"] == negf.NEGF_OK for r in rest)


def test_server_fp32_bulk_converges(gpu_lib):
    negf = gpu_lib
    req = small_request(10, 30, 0.4, -0.3, tol=1e-6)
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        a = srv.poll(srv.submit(req, precision=negf.FP64))
        b = srv.poll(srv.submit(req, precision=negf.FP32_BULK))
    say("fp32-bulk passes", b["iterations"], "max |dU| vs fp64", np.max(np.abs(a["U"] - b["U"])))
    assert b["status"] == negf.NEGF_OK
    assert np.max(np.abs(a["U"] - b["U"])) < 1e-2


def test_server_admission_by_footprint(gpu_lib):
    negf = gpu_lib
    reqs = [small_request(8, 24, 0.2, 0.3), small_request(8, 24, 0.1, 0.2)]
    store = 1 << 26
    # the footprint the server books for one such request
    with negf.Server(64 * GIB, store_bytes=store) as srv:
        rid = srv.submit(reqs[0])
        fp = 0
        for _ in range(2000):
            st = srv.stats()
            if st["running"] == 1:
                fp = st["hbm_used"] - 2 * store
                break
            time.sleep(0.001)
        srv.poll(rid)
    say("footprint", fp)
    assert fp > 0
    # a budget that holds one of these requests beside the two stores, not two
    with negf.Server(2 * store + int(1.5 * fp), store_bytes=store) as srv:
        ids = [srv.submit(r) for r in reqs]
        res = [srv.poll(i) for i in ids]
        st = srv.stats()
    say("queue ms", [r["t_queue_ms"] for r in res], "total ms", [r["t_total_ms"] for r in res], st)
    assert all(r["status"] == negf.NEGF_OK for r in res)
    # the second request waited for the first to finish
    assert res[1]["t_queue_ms"] >= res[0]["t_total_ms"] - 1.0
    with negf.Server(2 * store + int(1.5 * fp), store_bytes=store) as srv:
        with pytest.raises(negf.NegfError) as ei:
            srv.submit(small_request(17, 200, 0.2, 0.3, n_c=64, n_r=128))
        assert ei.value.status == negf.NEGF_ENOMEM


def test_server_rejects_bad_requests(gpu_lib):
    negf = gpu_lib
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        bad = small_request()
        bad.zeta = 0.0
        with pytest.raises(negf.NegfError) as ei:
            srv.submit(bad)
        assert ei.value.status == negf.NEGF_EINVAL
        with pytest.raises(negf.NegfError):
            srv.poll(12345)


def test_server_warm_start_matches_oracle(gpu_lib):
    # a bias point started from the converged charge of its neighbour (an I-V sweep)
    negf = gpu_lib
    first = small_request(10, 30, 0.30, 0.1)
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        a = srv.poll(srv.submit(first))
    rho = a["charge"].reshape(30, 10).sum(axis=1)
    nxt = replace(small_request(10, 30, 0.35, 0.1), rho_init=rho)
    cold = small_request(10, 30, 0.35, 0.1)
    ref = S.self_consistent(nxt)
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        got = srv.poll(srv.submit(nxt))
        c = srv.poll(srv.submit(cold))
    dU = np.max(np.abs(got["U"] - ref["U"]))
    say("warm passes gpu/oracle", got["iterations"], ref["iterations"], "cold", c["iterations"], "dU", dU,
        "first-pass norm warm/cold", got["trace"][0], c["trace"][0])
    assert got["status"] == negf.NEGF_OK and ref["converged"]
    assert got["iterations"] == ref["iterations"] and dU < 1e-9
    # the neighbour's charge is a better start: smaller first residual, no more passes
    assert got["trace"][0] < 0.5 * c["trace"][0] and got["iterations"] <= c["iterations"]


def _same(a, b):
    return (a["status"] == b["status"] and a["iterations"] == b["iterations"] and np.array_equal(a["U"], b["U"])
            and np.array_equal(a["charge"], b["charge"]) and a["current"] == b["current"]
            and np.array_equal(a["trace"], b["trace"]))


def test_server_eviction_resumes_bitwise(gpu_lib):
    # one slot and a time slice of two passes: the requests take turns, each evicted to
    # host state and re-admitted several times; every result equals its solo run
    negf = gpu_lib
    reqs = [small_request(10, 26, 0.3, 0.1, tol=1e-9),
            small_request(8, 30, 0.2, -0.2, n_r=0, eta=1e-6, norm=1, tol=1e-9, grid_density=(2.0, 10.0, 4.0),
                          grid_limits=(-0.2, 0.0), grid_refresh=3)]
    solo = []
    for r in reqs:
        with negf.Server(64 * GIB, store_bytes=GIB) as srv:
            solo.append(srv.poll(srv.submit(r)))
    with negf.Server(64 * GIB, max_inflight=1, store_bytes=GIB) as srv:
        srv.set_time_slice(2)
        ids = [srv.submit(r) for r in reqs]
        got = [srv.poll(i) for i in ids]
    say("evictions", [g["evictions"] for g in got], "passes", [g["iterations"] for g in got])
    assert all(g["evictions"] >= 1 for g in got)
    for s_, g in zip(solo, got):
        assert s_["status"] == negf.NEGF_OK and _same(s_, g)


def test_server_explicit_evict_and_deadline(gpu_lib):
    negf = gpu_lib
    req = small_request(10, 30, 0.4, -0.3, tol=1e-9)
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        base = srv.poll(srv.submit(req))
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        rid = srv.submit(req)
        srv.evict(rid)                       # takes effect at the end of its first pass
        got = srv.poll(rid)
        with pytest.raises(negf.NegfError):
            srv.evict(rid)                   # finished and released
    say("explicit eviction: evictions", got["evictions"], "passes", got["iterations"], base["iterations"])
    assert got["evictions"] == 1 and _same(base, got)
    # a deadline far shorter than one pass: the request ends with ETIMEDOUT
    with negf.Server(64 * GIB, store_bytes=GIB) as srv:
        late = srv.poll(srv.submit(replace(req, deadline_ms=1e-3)))
    assert late["status"] == negf.NEGF_ETIMEDOUT
