"""Write the oracle's LHDM results on all 2000 instances of the uneven
nonnegative batch (seed 4000: m ~ U{32..512}, n = round(m U[2, 4]), A ~ U[0, 1],
10 %-dense U[0, 1] x, noise 1e-2).

Calls only ``oracle`` and ``workloads``.  Default parameters of the library
(tau1 = 0.6, tau2 = 0.15, delta = 0.9, kmax = 32, KKT tolerance 1e-9).  Stored in
``c4_seed4000_lhdm.npz``, per instance:

* ``P_len``, ``P_flat`` -- the final passive set in insertion order,
* ``counters``          -- status, outer, inner, jloop_drops, n_passive,
* ``obj``               -- ||b - A x||^2.

x itself is not stored: on the final passive set it is the least-squares
solution, which a test recomputes from A, b and P.

Usage: ``python tests/golden/make_batch_golden.py [processes]``.
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SEED = 4000
OUT = os.path.join(HERE, f"c4_seed{SEED}_lhdm.npz")


def _one(i):
    import oracle
    from workloads import make_c4_instance
    inst = make_c4_instance(i, SEED)
    x, info = oracle.oracle_lhdm(inst.A, inst.b, tau1=0.6, tau2=0.15, delta=0.9, kmax=32, kkt_tol=1e-9)
    return (info["passive"], [info["status"], info["outer_iters"], info["inner_iters"], info["jloop_drops"],
                              info["n_passive"]], info["objective"])


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    count = 2000
    t0 = time.perf_counter()
    with Pool(procs) as pool:
        res = pool.map(_one, range(count), chunksize=4)
    P_len = np.array([len(r[0]) for r in res], dtype=np.int32)
    P_flat = np.array([j for r in res for j in r[0]], dtype=np.int16)
    counters = np.array([r[1] for r in res], dtype=np.int32)
    obj = np.array([r[2] for r in res], dtype=np.float64)
    np.savez_compressed(OUT, P_len=P_len, P_flat=P_flat, counters=counters, obj=obj, seed=np.int64(SEED))
    print(f"{count} instances in {time.perf_counter() - t0:.0f} s with {procs} processes -> {OUT}; "
          f"status counts {np.bincount(counters[:, 0])}", flush=True)


if __name__ == "__main__":
    main()
