"""Writes the oracle's full-grid result for the (17,0), 400-ring device workload.

    python tests/golden/make_device_reference.py [N]

Calls only the CPU oracle (one process per core).  Output:
tests/golden/oracle_cnt17_N{N}_c512_r1536.npz with charge[N*17], T[1536], current,
decim_iters and the per-node diagonals needed for energy-resolved checks are not
stored (size).
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

os.environ.setdefault("OMP_NUM_THREADS", "1")      # one BLAS thread per worker process
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import negf_oracle as O  # noqa: E402
from paper_2407_14633_amd import workload as W  # noqa: E402


def _contour(args):
    N, z = args
    return O.energy_point_contour(W.device_problem(N=N), z)


def _real(args):
    N, E = args
    AL, AR, T, _ = O.energy_point_real(W.device_problem(N=N), E)
    return AL, AR, T


def main(N=400):
    p = W.device_problem(N=N)
    g = p.grid
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=os.cpu_count()) as ex:
        gr = np.array(list(ex.map(_contour, [(N, z) for z in g.z_c], chunksize=8)))
        real = list(ex.map(_real, [(N, E) for E in g.E_r], chunksize=8))
    AL = np.array([r[0] for r in real])
    AR = np.array([r[1] for r in real])
    T = np.array([r[2] for r in real])
    charge, current = O.reduce_energies(p, gr, AL, AR, T)
    out = os.path.join(HERE, f"oracle_cnt17_N{N}_c512_r1536.npz")
    np.savez_compressed(out, charge=charge, T=T, current=np.array([current]))
    print(f"wrote {out} in {time.time() - t0:.1f} s; current {current:.6e} A, charge range "
          f"[{charge.min():.6f}, {charge.max():.6f}]")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 400)
