"""Write the oracle's LHDM path on the 4096 x 16384 Gaussian instance (seed 3000).

Calls only ``oracle`` and ``workloads``: every stored value comes from the CPU
oracle.  For each deviation threshold delta in {0.2, 0.5, 0.8} (tau1 = 0.6,
tau2 = 0.15, kmax = 32, KKT tolerance 1e-9) it stores, in
``c3_seed3000_delta<d>.npz``:

* ``passive``   -- the final ordered passive set,
* ``x``         -- the solution (all n entries),
* ``counters``  -- status, outer, inner, jloop_drops, n_passive,
* ``J_len``, ``J_flat``        -- the accepted block J of every outer step,
* ``drops``                    -- columns the feasibility loop on J dropped per step,
* ``rm_count``                 -- inner iterations of every outer step,
* ``rm_len``, ``rm_flat``      -- the columns removed by every inner iteration,
* ``nP``, ``obj``              -- |P| and ||b - A x||^2 after every outer step,
* ``seconds``, ``threads``     -- wall time of the solve and the BLAS thread count.

From ``J`` and the removal lists the ordered passive set after any outer step
can be rebuilt (append J, then delete each removal list in order).

Usage: ``python tests/golden/make_c3_golden.py 0.8`` (one delta per process;
a solve takes minutes to tens of minutes of CPU time).
"""
from __future__ import annotations

import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import make_c3  # noqa: E402

SEED = 3000
DELTAS = (0.2, 0.5, 0.8)


def golden_path(delta: float, seed: int = SEED) -> str:
    return os.path.join(HERE, f"c3_seed{seed}_delta{delta:.1f}.npz")


def run(delta: float, seed: int = SEED) -> str:
    inst = make_c3(seed)
    t0 = time.perf_counter()
    x, info = oracle.oracle_lhdm(inst.A, inst.b, tau1=0.6, tau2=0.15, delta=delta, kmax=32,
                                 kkt_tol=1e-9, record=True)
    secs = time.perf_counter() - t0
    tr = info["trace"]
    J_len = np.array([len(s["J"]) for s in tr], dtype=np.int32)
    J_flat = np.array([j for s in tr for j in s["J"]], dtype=np.int32)
    drops = np.array([s["drops"] for s in tr], dtype=np.int32)
    rm_count = np.array([len(s["removed"]) for s in tr], dtype=np.int32)
    rm_len = np.array([len(r) for s in tr for r in s["removed"]], dtype=np.int32)
    rm_flat = np.array([j for s in tr for r in s["removed"] for j in r], dtype=np.int32)
    nP = np.array([s["nP"] for s in tr], dtype=np.int32)
    obj = np.array([s["obj"] for s in tr], dtype=np.float64)
    counters = np.array([info["status"], info["outer_iters"], info["inner_iters"], info["jloop_drops"],
                         info["n_passive"]], dtype=np.int64)
    kkt = oracle.kkt_report(inst.A, inst.b, x)["kkt"]
    threads = os.environ.get("OPENBLAS_NUM_THREADS") or os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    out = golden_path(delta, seed)
    np.savez_compressed(out, passive=np.array(info["passive"], dtype=np.int32), x=x, counters=counters,
                        J_len=J_len, J_flat=J_flat, drops=drops, rm_count=rm_count, rm_len=rm_len,
                        rm_flat=rm_flat, nP=nP, obj=obj, seconds=np.float64(secs), threads=np.int32(int(threads)),
                        kkt=np.float64(kkt), delta=np.float64(delta), seed=np.int64(seed),
                        host=np.array(platform.processor() or platform.machine()))
    print(f"delta={delta} seed={seed}: status={info['status']} outer={info['outer_iters']} "
          f"inner={info['inner_iters']} jdrops={info['jloop_drops']} nP={info['n_passive']} kkt={kkt:.2e} "
          f"time={secs:.1f}s threads={threads} -> {out}", flush=True)
    return out


if __name__ == "__main__":
    ds = [float(a) for a in sys.argv[1:]] or list(DELTAS)
    for d in ds:
        run(d)
