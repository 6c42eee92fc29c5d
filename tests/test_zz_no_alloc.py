"""Allocation-free solve (negf_solve_dev_static) against negf_solve_dev.

Both run the same kernels on the same inputs, so the results must agree bit for
bit (no arithmetic depends on the chunking of the recursion stores or on where
the work buffers live).  Two calls in a row, the second on a smaller input,
exercise the reuse of the fixed device area; a problem too large for the area
is rejected on the host before any kernel runs."""
import sys

import numpy as np
import pytest

from paper_2407_14633_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tensors(torch, p, dev):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = p.grid
    return dict(zc=t(g.z_c), wc=t(g.w_c), Er=t(g.E_r), wr=t(g.w_r))


def _solve(negf, torch, d, p, static, stream):
    dev = torch.device("cuda:0")
    x = _tensors(torch, p, dev)
    nb = p.device.n_rings * p.device.b
    charge = torch.full((nb,), -1.0, dtype=torch.float64, device=dev)
    T = torch.full((p.grid.n_r,), -1.0, dtype=torch.float64, device=dev)
    cur = torch.zeros(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        fn = d.solve_dev_static if static else d.solve_dev
        fn(p.bias, x["zc"], x["wc"], x["Er"], x["wr"], charge, T, cur, stream=stream)
    d.sync()
    torch.cuda.synchronize()
    return charge.cpu().numpy(), T.cpu().numpy(), float(cur.cpu()[0])


def _problem(n, N, n_c, n_r, seed):
    dev = W.zigzag_cnt(n, N)
    U, _ = W.potential_tanh_barrier(N, n, seed)
    bias = W.Bias(0.15, -0.15)
    grid = W.nonequilibrium_grid(W.gershgorin_lower(dev, U) - 1.0, bias, n_c, n_r)
    return W.Problem(f"cnt{n}_N{N}", dev, U, 0.0, 0.0, bias, grid)


def test_static_solve_equals_device_solve(gpu_lib):
    import torch
    negf = gpu_lib
    torch.cuda.set_device(0)
    s = torch.cuda.Stream()
    say("static area bytes", negf.static_scratch_bytes())
    # a (17,0) tube whose recursion stores do not fit the area at once (chunked),
    # then a smaller (8,0) tube on the same area
    cases = [(_problem(17, 200, 96, 288, 31), negf.FP64), (_problem(8, 40, 12, 40, 32), negf.FP64),
             (_problem(10, 64, 16, 48, 33), negf.FP32_BULK)]
    for p, prec in cases:
        say("case", p.name, p.grid.n_c, p.grid.n_r, "precision", prec)
        with negf.NegfDevice(p.device, precision=prec) as d:
            d.set_potential(p.U, p.U_left, p.U_right)
            ref = _solve(negf, torch, d, p, False, s)
            got = _solve(negf, torch, d, p, True, s)
            again = _solve(negf, torch, d, p, True, s)
        for what, r in (("first", got), ("repeat", again)):
            assert np.array_equal(r[0], ref[0]), f"{p.name} {what}: charge differs"
            assert np.array_equal(r[1], ref[1]), f"{p.name} {what}: T differs"
            assert r[2] == ref[2], f"{p.name} {what}: current differs"
        assert np.all(np.isfinite(ref[0])) and ref[0].min() > 0


def test_static_solve_rejects_oversized_problem(gpu_lib):
    import torch
    negf = gpu_lib
    torch.cuda.set_device(0)
    p = _problem(17, 400, 16, 16, 34)
    area = negf.static_scratch_bytes()
    # contour diagonals alone: n_c x N b x 16 bytes, beyond the area
    n_c = area // (400 * 17 * 16) + 8
    bias = W.Bias(0.15, -0.15)
    grid = W.nonequilibrium_grid(-9.0, bias, int(n_c), 4)
    p = W.Problem("big", p.device, p.U, 0.0, 0.0, bias, grid)
    with negf.NegfDevice(p.device) as d:
        d.set_potential(p.U)
        with pytest.raises(negf.NegfError) as e:
            _solve(negf, torch, d, p, True, torch.cuda.Stream())
        assert e.value.status == negf.NEGF_EINVAL and "static scratch" in str(e.value)
        # the handle stays usable
        small = _problem(17, 400, 4, 8, 35)
        ref = _solve(negf, torch, d, small, False, torch.cuda.Stream())
        got = _solve(negf, torch, d, small, True, torch.cuda.Stream())
        assert np.array_equal(got[0], ref[0]) and got[2] == ref[2]
