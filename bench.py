"""Energy-point solve throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload device|small|device1000|device2000|batch]
                    [--no-cpu-baseline] [--no-fp32]

One step = one full negf_solve_dev (decimation, both recursions, contour diagonals,
lead columns, energy sums) over the workload's energy grid, inputs already in HBM.
Prints one JSON line on stdout; per-kernel details go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2407_14633_amd import workload as W  # noqa: E402

METRIC = "RGF energy-point solves/sec (FP64 vs FP32-bulk) + p50/p99 I-V request latency"
FP64_PEAK_TFLOPS = 78.6     # MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3    # MI355X published FP32 vector peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(name: str) -> W.Problem:
    if name == "device":
        return W.device_problem(N=400)
    if name == "device1000":
        return W.device_problem(N=1000)
    if name == "device2000":
        return W.device_problem(N=2000)
    if name == "small":
        return W.small_problem()
    raise SystemExit(f"unknown workload {name}")


def ell_width(dev: W.Device) -> int:
    K = 1
    for H in dev.h_up:
        nz = np.abs(H) > 0
        K = max(K, int(nz.sum(axis=0).max()), int(nz.sum(axis=1).max()))
    return K


def is_circulant(M: np.ndarray) -> bool:
    b = M.shape[0]
    idx = (np.arange(b)[None, :] - np.arange(b)[:, None]) % b
    return bool(np.array_equal(M, M[0][idx]))


def lead_is_circulant(ld) -> bool:
    """Every block of the lead ring-circulant: the library decimates it in ring modes."""
    return (is_circulant(ld.tau) and all(is_circulant(m) for m in ld.h_diag)
            and all(is_circulant(m) for m in ld.h_up))


def algorithmic_flops(p: W.Problem, decim_iters: np.ndarray) -> dict:
    """Real flops per kernel launch, from the method's operation counts.

    Counting: a b x b complex Gauss-Jordan inverse = b^3 complex multiply-adds = 8 b^3
    flops; a dense b x b complex product = 8 b^3; an ELL product of width K = 8 b^2 K.
    """
    N, b = p.device.n_rings, p.device.b
    n_c, n_r = p.grid.n_c, p.grid.n_r
    inv, mul = 8.0 * b ** 3, 8.0 * b ** 3
    # recursions: one dense inverse per ring step (the sparse coupling products are
    # not counted), N-1 steps per chain plus the final inverse on real-axis chains;
    # two chains per node
    recur = 2 * (n_c + n_r) * (N - 1) * inv + 2 * n_r * inv
    cdiag = n_c * N * inv
    # lead columns: per ring one propagation product and one W Gamma product (+ b^2 dots)
    column = 2 * n_r * (N * (mul + 8.0 * b * b) + (N - 1) * mul)
    # decimation per doubling step: period 1 one b x b inverse + 6 products; period 2 one
    # 2b x 2b inverse (8 b x b inverse equivalents) + 8 products; the surface step
    # repeats the inverse and adds tau g tau^H
    per_it = {1: 1 * inv + 6 * mul, 2: 8 * inv + 8 * mul}
    fin = {1: inv + 2 * mul, 2: 8 * inv + 2 * mul}
    # ring-circulant leads are decimated as b scalar chains: per mode and doubling step
    # about 68 flops (one-ring layer) or 115 (two-ring layer, closed-form 2x2 inverse);
    # then per mode ~28 flops for g_s and Sigma_q and 8 b^2 for the back transform
    per_it_modes = {1: 68.0 * b, 2: 115.0 * b}
    fin_modes = 28.0 * b + 8.0 * b * b
    dec = 0.0
    for l, ld in enumerate((p.device.left, p.device.right)):
        if lead_is_circulant(ld):
            dec += per_it_modes[ld.period] * float(decim_iters[:, l].sum()) + fin_modes * len(decim_iters)
        else:
            dec += per_it[ld.period] * float(decim_iters[:, l].sum()) + fin[ld.period] * len(decim_iters)
    return {"recur": recur, "cdiag": cdiag, "column": column, "decimate": dec}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p: W.Problem, n_c: int = 16, n_r: int = 48, seed: int = 99) -> dict:
    """The oracle as it stands, timed on the host cores over a fixed sample of nodes,
    and in one thread on a smaller sample."""
    from concurrent.futures import ProcessPoolExecutor
    cores = min(os.cpu_count() or 1, 16, n_c + n_r)
    sub = W.subsample_grid(p.grid, n_c, n_r, seed)
    jobs = [("c", z) for z in sub.z_c] + [("r", E) for E in sub.E_r]
    one = W.subsample_grid(p.grid, 2, 6, seed + 1)
    t0 = time.perf_counter()
    for kind, x in [("c", z) for z in one.z_c] + [("r", E) for E in one.E_r]:
        _oracle_point((p, kind, x))
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_oracle_point, [(p, kind, x) for kind, x in jobs]))
    dt = time.perf_counter() - t0
    return {"value": len(jobs) / dt, "unit": "energy-point solves/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "one_thread": {"value": (one.n_c + one.n_r) / dt1, "unit": "energy-point solves/s",
                           "sample": f"{one.n_c} contour + {one.n_r} real-axis nodes (seed {seed + 1}), "
                                     f"{dt1:.2f} s"},
            "sample": f"{sub.n_c} contour + {sub.n_r} real-axis nodes of the same workload (seed {seed}), "
                      f"numpy/LAPACK oracle incl. decimation, one process per core (one BLAS thread each), "
                      f"{dt:.2f} s wall"}


def _oracle_point(args):
    from threadpoolctl import threadpool_limits
    from oracle import negf_oracle as O
    p, kind, x = args
    with threadpool_limits(1):   # one BLAS thread per worker: `cores` counts worker processes
        if kind == "c":
            return O.energy_point_contour(p, x)
        return O.energy_point_real(p, x)


def run(p: W.Problem, precision: int, steps: int, warmup: int):
    import torch
    from paper_2407_14633_amd import negf
    dev = torch.device("cuda:0")
    d = negf.NegfDevice(p.device, precision=precision, eta=p.eta, decim_tol=p.decim_tol,
                        decim_max_iter=p.decim_max_iter, g_s=p.g_s)
    d.set_potential(p.U, p.U_left, p.U_right)
    g = p.grid
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype=dt)
    zc = t(g.z_c.view(np.float64).reshape(-1, 2), torch.float64) if g.n_c else None
    wc = t(g.w_c.view(np.float64).reshape(-1, 2), torch.float64) if g.n_c else None
    Er = t(g.E_r, torch.float64) if g.n_r else None
    wr = t(g.w_r, torch.float64) if g.n_r else None
    nb = p.device.n_rings * p.device.b
    charge = torch.zeros(nb, dtype=torch.float64, device=dev)
    T = torch.zeros(max(g.n_r, 1), dtype=torch.float64, device=dev)
    cur = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        d.solve_dev(p.bias, zc, wc, Er, wr, charge, T, cur, stream)
    d.sync()
    d.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        d.solve_dev(p.bias, zc, wc, Er, wr, charge, T, cur, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d.sync()
    times = d.kernel_times()
    d.set_profiling(False)
    # one detailed host solve for the decimation step counts (not timed)
    res = d.solve(p.bias, p.grid, details=True)
    out = dict(ms_per_step=1e3 * dt / steps, times=times, iters=res.decim_iters,
               charge=charge.cpu().numpy(), current=float(cur.item()), T=T.cpu().numpy()[:g.n_r],
               fp64_nodes=res.fp64_nodes)
    d.close()
    return out


def batch_flops(ps) -> dict:
    """Recursion, contour-diagonal and lead-column flops of one batch solve (decimation
    omitted: its step counts are per node and not fetched for batches)."""
    tot = {"recur": 0.0, "cdiag": 0.0, "column": 0.0}
    for p in ps:
        f = algorithmic_flops(p, np.zeros((1, 2)))
        for k in tot:
            tot[k] += f[k]
    return tot


def run_batch(ps, precision: int, steps: int, warmup: int, grid_scale: int = 0, autotune: bool = False,
              graph: bool = False):
    """Times negf_batch_solve_dev over all problems of the batch, inputs resident in HBM;
    optionally after the schedule autotuner, and as replays of a captured HIP graph."""
    import torch
    from paper_2407_14633_amd import negf
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype=dt)
    devs, jobs = [], []
    for p in ps:
        d = negf.NegfDevice(p.device, precision=precision, eta=p.eta, decim_tol=p.decim_tol,
                            decim_max_iter=p.decim_max_iter, g_s=p.g_s)
        d.set_potential(p.U, p.U_left, p.U_right)
        devs.append(d)
        g = p.grid
        jobs.append(dict(dev=d, bias=p.bias,
                         zc=t(g.z_c.view(np.float64).reshape(-1, 2), torch.float64) if g.n_c else None,
                         wc=t(g.w_c.view(np.float64).reshape(-1, 2), torch.float64) if g.n_c else None,
                         Er=t(g.E_r, torch.float64) if g.n_r else None,
                         wr=t(g.w_r, torch.float64) if g.n_r else None,
                         charge=torch.zeros(p.device.n_rings * p.device.b, dtype=torch.float64, device=dev),
                         T=torch.zeros(max(g.n_r, 1), dtype=torch.float64, device=dev),
                         current=torch.zeros(1, dtype=torch.float64, device=dev)))
    ws = negf.Workspace()
    if grid_scale:
        ws.set_grid_scale(grid_scale)
    stream = torch.cuda.current_stream()
    schedule = None
    if autotune:
        best = ws.autotune(jobs, stream, reps=1)
        schedule = {"grid_scale": best.grid_scale, "order": best.order, "ms_per_solve": round(best.ms_per_solve, 2),
                    "chains_per_wave": {b: int(best.chains_per_wave[b]) for b in range(1, 25)
                                        if best.chains_per_wave[b]}}
        log(f"  autotuned schedule {schedule}")
    for _ in range(warmup):
        ws.solve_dev(jobs, stream)
    ws.sync()
    ws.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ws.solve_dev(jobs, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ws.sync()
    times = ws.kernel_times()
    out = dict(ms_per_step=1e3 * dt / steps, times=times, hbm_bytes=ws.bytes(),
               current=[float(j["current"].item()) for j in jobs],
               charge=[j["charge"].cpu().numpy() for j in jobs], schedule=schedule)
    ws.close()
    if graph:
        # the same batch recorded once into a HIP graph (private workspace), replayed
        gstream = torch.cuda.Stream()   # capture needs a created stream (default priority)
        torch.cuda.synchronize()
        with negf.Graph(jobs, gstream) as gph:
            gph.launch(gstream)
            gph.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                gph.launch(gstream)
            torch.cuda.synchronize()
            out["graph_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / steps
            gph.sync()
        log(f"  graph replay ms/step {out['graph_ms_per_step']:.2f}")
    for d in devs:
        d.close()
    return out


def bench_batch(a):
    """Batched form: 64 tubes of uneven chirality, length and node count in the same launches."""
    from paper_2407_14633_amd import negf
    ps = W.batch_problems()
    n_e = sum(p.grid.n_c + p.grid.n_r for p in ps)
    log(f"batch: {len(ps)} devices, {n_e} nodes, rings {min(p.device.n_rings for p in ps)}-"
        f"{max(p.device.n_rings for p in ps)}, chiralities {sorted(set(p.meta['n'] for p in ps))}")
    flops = batch_flops(ps)
    res = {}
    for name, prec, peak in (("f64", negf.FP64, FP64_PEAK_TFLOPS), ("f32_bulk", negf.FP32_BULK, FP32_PEAK_TFLOPS)):
        if name == "f32_bulk" and a.no_fp32:
            continue
        r = run_batch(ps, prec, a.steps, a.warmup, autotune=not a.no_autotune, graph=not a.no_graph)
        ms, calls = r["times"]["recur"]
        per_step = ms / a.steps          # a batch step runs one recursion launch per store chunk
        ach = flops["recur"] / (per_step * 1e-3) / 1e12
        log(f"batch {name} ms/step {r['ms_per_step']:.2f} kernels {r['times']} HBM workspace {r['hbm_bytes'] / 2**30:.1f} GiB")
        res[name] = dict(r=r, value=n_e / (r["ms_per_step"] * 1e-3), schedule=r["schedule"],
                         graph_ms_per_step=r.get("graph_ms_per_step"),
                         roofline={"kernel": "recur", "bound": "alu", "achieved": round(ach, 4), "peak": peak,
                                   "unit": "TFLOP/s", "frac": round(ach / peak, 5), "traffic": None,
                                   "ms_per_step": round(per_step, 4), "launches_per_step": calls // a.steps,
                                   "flops_per_step": flops["recur"]})
    r64 = res["f64"]
    line = {
        "metric": METRIC, "value": r64["value"], "unit": "energy-point solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": r64["r"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(ps)} zigzag (n,0) tubes, n in {{10,13,17,20,23}}, 200-2000 rings, "
                               f"512-4096 nodes each (25% contour), {n_e} nodes in one batched solve",
                   "n_devices": len(ps), "n_nodes": n_e},
        "roofline": r64["roofline"], "cpu_baseline": None,
        "fp32_bulk": None if "f32_bulk" not in res else {
            "value": res["f32_bulk"]["value"], "ms_per_step": res["f32_bulk"]["r"]["ms_per_step"],
            "roofline": res["f32_bulk"]["roofline"],
            # per job |I32 - I64| / |I64| over jobs carrying at least 1e-3 of the largest current,
            # and the largest |I32 - I64| relative to that largest current
            **_current_diffs(res["f32_bulk"]["r"]["current"], r64["r"]["current"])},
        "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in r64["r"]["times"].items()},
        "schedule": r64["schedule"], "graph_ms_per_step": r64["graph_ms_per_step"],
        "serving": None,
    }
    print(json.dumps(line), flush=True)


def run_serving(n_req: int, rate: float, seed: int = 5555, precision=None, max_inflight: int = 64,
                adaptive: bool = True, eta: float = 1e-6) -> dict:
    """Poisson arrivals of self-consistent bias-point requests (devices drawn like the batch
    workload, V_DS ~ U[0,0.6], V_GS ~ U[-0.5,0.5]; eta 1e-6, semi-adaptive real axis, stop at
    a 1e-6 eV potential residual) served with continuous batching."""
    from paper_2407_14633_amd import negf
    precision = negf.FP32_BULK if precision is None else precision
    reqs = W.serving_requests(n_req, seed, adaptive=adaptive, eta=eta)
    arrivals = W.poisson_arrivals(n_req, rate, seed + 1)
    import torch
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    with negf.Server(budget, max_inflight=max_inflight, store_bytes=8 << 30) as srv:
        t0 = time.perf_counter()
        ids = []
        for r, t_arr in zip(reqs, arrivals):
            delay = t_arr - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(r, precision=precision))
        res = []
        for k, i in enumerate(ids):
            res.append(srv.poll(i))
            log(f"  request {k} ({reqs[k].name}): status {res[-1]['status']}, {res[-1]['iterations']} passes, "
                f"eps {res[-1]['eps_max']:.2e}, {res[-1]['t_total_ms']:.0f} ms, n_r {res[-1]['n_r']}")
        wall = time.perf_counter() - t0
        st = srv.stats()
    lat = np.array([r["t_total_ms"] for r in res])
    it = np.array([r["iterations"] for r in res])
    ok = sum(r["status"] == negf.NEGF_OK for r in res)
    ne = np.array([q.grid.n_c + r["n_r"] for q, r in zip(reqs, res)])
    return {"rate_req_per_s": rate, "requests": n_req, "converged": int(ok),
            "precision": "fp32_bulk" if precision == negf.FP32_BULK else "f64",
            "mode_space": int(sum(r["mode_space"] for r in res)),
            "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
            "throughput_req_per_s": n_req / wall, "wall_s": wall,
            "passes_mean": float(it.mean()), "passes_max": int(it.max()),
            "eta": reqs[0].eta, "tol": reqs[0].tol, "norm": "potential residual (eV)" if reqs[0].norm == 1
            else "relative charge", "grid": "semi-adaptive" if adaptive else "fixed",
            "energy_nodes_mean": float(ne.mean()),
            "node_solves_per_s": float(np.sum(it * ne) / wall),
            "status_counts": {str(k): int(v) for k, v in zip(*np.unique([r["status"] for r in res],
                                                                          return_counts=True))},
            "server_passes": st["passes"], "hbm_budget_gib": budget / 2**30,
            "workload": f"{n_req} requests, Poisson arrivals at {rate} req/s (seed {seed})"}


def _knee(runs) -> dict:
    top = runs[-1]
    sat = top["throughput_req_per_s"] < 0.9 * top["rate_req_per_s"]
    return {"knee_req_per_s": top["throughput_req_per_s"] if sat else None,
            "knee": (f"saturates near {top['throughput_req_per_s']:.1f} req/s (offered {top['rate_req_per_s']})"
                     if sat else f"not reached: keeps up with {top['rate_req_per_s']} req/s")}


def serving_sweep(n_req: int, rates, precision=None, etas=(1e-6, 1e-3)) -> dict:
    """run_serving at each offered rate, for each broadening; the knee is the throughput the
    server sustains at the highest rate when it falls short of that rate."""
    out = {"requests_per_rate": n_req}
    for k, eta in enumerate(etas):
        runs = []
        for r in rates:
            runs.append(run_serving(n_req, r, precision=precision, eta=eta))
            log("serving", runs[-1])
        entry = {"eta": eta, "runs": runs, **_knee(runs)}
        if k == 0:
            out.update(entry)
            out["precision"] = runs[-1]["precision"]
        else:
            out[f"eta_{eta:g}"] = entry
    # the same stream with FP64 NEGF at the highest rate: in mode space the scalar chains
    # gain nothing from FP32, and the FP64 recomputation of the nodes the FP32 checks mark
    # (a third of the current-carrying subbands' nodes) makes FP32-bulk the slower form
    from paper_2407_14633_amd import negf
    if precision is None or precision == negf.FP32_BULK:
        r64 = run_serving(n_req, rates[-1], precision=negf.FP64, eta=etas[0])
        log("serving", r64)
        out["fp64_negf"] = r64
    return out


def _current_diffs(c32, c64) -> dict:
    c32, c64 = np.asarray(c32), np.asarray(c64)
    big = np.max(np.abs(c64))
    sel = np.abs(c64) >= 1e-3 * big
    return {"current_rel_diff_vs_fp64_max": float(np.max(np.abs(c32 - c64)[sel] / np.abs(c64[sel]))),
            "current_diff_vs_largest_current": float(np.max(np.abs(c32 - c64)) / big),
            "jobs_compared": int(sel.sum())}


def calibrate_copy(mib: int):
    """A plain device-to-device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 8}), flush=True)


def measured_traffic(kernel: str, b: int, precision: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH/WRITE summary,
    or None when the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    t = "double" if precision == "f64" else "float"
    src = os.path.join(ROOT, "paper_2407_14633_amd", "csrc", "negf_kernels.hpp")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    names = {"recur": f"negf::k_recur<{t}, {b}>", "cdiag": f"negf::k_cdiag<{t}, {b}>",
             "column": f"negf::k_column<{t}, {b}>", "decimate": f"negf::k_decimate_circ<{b}>"}
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md")):
        for line in open(path):
            if line.startswith("machine-readable: "):
                d = json.loads(line[len("machine-readable: "):])
                if d.get("source_hash") == h and names.get(kernel) in d.get("hbm_bytes", {}):
                    return d["hbm_bytes"][names[kernel]]
    return None


def golden_reference(p: W.Problem):
    """The oracle's stored full-grid result for this workload (written by
    tests/golden/make_device_reference.py), if there is one."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{p.name}.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path)
    return {"charge": d["charge"], "T": d["T"], "current": float(d["current"][0]), "file": os.path.relpath(path, ROOT)}


def errors_vs(ref, r) -> dict:
    """Charge (relative to max_i |charge_i|), current, and T(E) (relative to max_E T) against the oracle."""
    if ref is None:
        return None
    q, T = ref["charge"], ref["T"]
    return {"charge_rel": float(np.max(np.abs(r["charge"] - q)) / np.max(np.abs(q))),
            "current_rel": abs(r["current"] - ref["current"]) / abs(ref["current"]),
            "T_rel_to_max": float(np.max(np.abs(r["T"] - T)) / np.max(np.abs(T))),
            "oracle_file": ref["file"]}


def counted_flops(kernel: str, b: int, precision: str):
    """FLOPs per dispatch of `kernel` counted by rocprofv3's VALU instruction counters
    (committed summary), or None when the kernel source changed since."""
    import glob
    import hashlib
    t = "double" if precision == "f64" else "float"
    src = os.path.join(ROOT, "paper_2407_14633_amd", "csrc", "negf_kernels.hpp")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    name = {"recur": f"negf::k_recur<{t}, {b}>", "cdiag": f"negf::k_cdiag<{t}, {b}>",
            "column": f"negf::k_column<{t}, {b}>"}.get(kernel)
    for path in glob.glob(os.path.join(ROOT, "profiles", "valu_flops_*.md")):
        for line in open(path):
            if line.startswith("machine-readable: "):
                d = json.loads(line[len("machine-readable: "):])
                if d.get("source_hash") == h and name in d.get("counted_flops_per_dispatch", {}):
                    return d["counted_flops_per_dispatch"][name]
    return None


def roofline(p, r, peak_tflops, precision="f64"):
    flops = algorithmic_flops(p, r["iters"])
    best = None
    for k, (ms, calls) in r["times"].items():
        if k in flops and calls:
            avg = ms / calls
            if best is None or avg > best[1]:
                best = (k, avg)
    k, avg = best
    ach = flops[k] / (avg * 1e-3) / 1e12
    cnt = counted_flops(k, p.device.b, precision)
    return {"kernel": k, "bound": "alu", "achieved": round(ach, 4), "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": round(ach / peak_tflops, 5), "traffic": measured_traffic(k, p.device.b, precision),
            "avg_ms": round(avg, 4), "flops_per_launch": flops[k],
            "counted": None if cnt is None else {
                "flops_per_launch": cnt, "achieved": round(cnt / (avg * 1e-3) / 1e12, 4),
                "frac": round(cnt / (avg * 1e-3) / 1e12 / peak_tflops, 5),
                "source": "rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64/F32 + MFMA_MOPS, all lanes"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="device")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--requests", type=int, default=32, help="serving: requests per offered rate")
    ap.add_argument("--rates", default="10,200", help="serving: Poisson arrival rates (req/s), comma-separated")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="batch: skip the schedule autotuner")
    ap.add_argument("--no-graph", action="store_true", help="batch: skip the HIP-graph replay timing")
    ap.add_argument("--serving-fp64", action="store_true", help="serving: FP64 NEGF instead of FP32-bulk")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (HBM counter calibration)")
    a = ap.parse_args()
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs each energy-point solve on a single MI355X "
              "(energy nodes would shard across GPUs with one all-reduce of the charge; that path is not "
              "implemented).", file=sys.stderr)
        raise SystemExit(2)
    from paper_2407_14633_amd import negf
    if a.workload == "batch":
        bench_batch(a)
        return
    rates = [float(x) for x in a.rates.split(",") if x]
    serving_prec = negf.FP64 if a.serving_fp64 else negf.FP32_BULK
    if a.workload == "serving":
        sw = serving_sweep(a.requests, rates, serving_prec)
        top = sw["runs"][0]
        print(json.dumps({"metric": METRIC, "value": top["p99_latency_ms"], "unit": "ms (p99 request latency)",
                          "n_gpus": 1, "steps": a.requests, "warmup": 0, "ms_per_step": top["p50_latency_ms"],
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": top["precision"],
                          "data": "synthetic", "config": {"workload": top["workload"]}, "serving": sw}),
              flush=True)
        return
    p = make_problem(a.workload)
    n_e = p.grid.n_c + p.grid.n_r
    log(f"workload {p.name}: N={p.device.n_rings} b={p.device.b} n_c={p.grid.n_c} n_r={p.grid.n_r}")
    # the oracle's worker processes are forked before anything touches the GPU
    cpu = None if a.no_cpu_baseline else cpu_baseline(p)
    log("cpu baseline", cpu)
    r64 = run(p, negf.FP64, a.steps, a.warmup)
    log("fp64 ms/step", r64["ms_per_step"], "kernels", r64["times"])
    rf64 = roofline(p, r64, FP64_PEAK_TFLOPS)
    log("fp64 roofline", rf64)
    golden = golden_reference(p)
    fp32 = None
    if not a.no_fp32:
        r32 = run(p, negf.FP32_BULK, a.steps, a.warmup)
        log("fp32-bulk ms/step", r32["ms_per_step"], "kernels", r32["times"])
        rf32 = roofline(p, r32, FP32_PEAK_TFLOPS, "f32")
        err = float(np.max(np.abs(r32["charge"] - r64["charge"])) / np.max(np.abs(r64["charge"])))
        fp32 = {"value": n_e / (r32["ms_per_step"] * 1e-3), "ms_per_step": r32["ms_per_step"],
                "speedup_vs_fp64": r64["ms_per_step"] / r32["ms_per_step"],
                "roofline": rf32, "charge_rel_diff_vs_fp64": err,
                "current_rel_diff_vs_fp64": abs(r32["current"] - r64["current"]) / abs(r64["current"] or 1.0),
                "real_nodes_recomputed_fp64": r32["fp64_nodes"], "real_nodes": p.grid.n_r,
                "vs_oracle": errors_vs(golden, r32)}
    serving = None
    if not a.no_serving:
        serving = serving_sweep(a.requests, rates, serving_prec)
    line = {
        "metric": METRIC, "value": n_e / (r64["ms_per_step"] * 1e-3), "unit": "energy-point solves/s",
        "fp64_vs_oracle": errors_vs(golden, r64),
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{p.name}: zigzag (17,0) CNT tight binding, {p.device.n_rings} rings, "
                               f"{p.grid.n_c} contour + {p.grid.n_r} real-axis nodes, mu = +/-0.15 eV, eta 1e-6",
                   "n_rings": p.device.n_rings, "ring_size": p.device.b, "n_contour": p.grid.n_c,
                   "n_real": p.grid.n_r},
        "roofline": rf64, "cpu_baseline": cpu, "fp32_bulk": fp32,
        "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in r64["times"].items()},
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
