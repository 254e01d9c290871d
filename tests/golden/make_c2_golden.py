"""Write the oracle's LHDM and LH results on the 20 sparse-recovery instances
(seeds 2000-2019: m = 1024, n = 4096, unit-norm Gaussian columns, 128-sparse
U[0.5, 1.5] planted x, noiseless).

Calls only ``oracle`` and ``workloads``; default parameters (tau1 = 0.6,
tau2 = 0.15, delta = 0.9, kmax = 32, KKT tolerance 1e-9).  Stored in
``c2_seeds2000-2019.npz``: for each method (``lhdm``, ``lh``) and seed, the
final passive set in insertion order (``<m>_P``, 128-plus entries per seed,
``<m>_P_len``), x on that set (``<m>_xP``) and the counters (``<m>_counters``:
status, outer, inner, jloop_drops, n_passive).

Usage: ``python tests/golden/make_c2_golden.py [processes]``.
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

SEEDS = list(range(2000, 2020))
OUT = os.path.join(HERE, "c2_seeds2000-2019.npz")


def _one(job):
    import oracle
    from workloads import make_c2
    method, seed = job
    inst = make_c2(seed)
    fn = oracle.oracle_lhdm if method == "lhdm" else oracle.oracle_lh
    x, info = fn(inst.A, inst.b)
    P = list(info["passive"])
    return method, seed, P, x[P], [info["status"], info["outer_iters"], info["inner_iters"], info["jloop_drops"],
                                   info["n_passive"]]


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    t0 = time.perf_counter()
    jobs = [(mth, s) for mth in ("lhdm", "lh") for s in SEEDS]
    with Pool(procs) as pool:
        res = pool.map(_one, jobs, chunksize=1)
    out = {"seeds": np.array(SEEDS, dtype=np.int32)}
    for mth in ("lhdm", "lh"):
        rr = sorted([r for r in res if r[0] == mth], key=lambda r: r[1])
        out[f"{mth}_P_len"] = np.array([len(r[2]) for r in rr], dtype=np.int32)
        out[f"{mth}_P"] = np.array([j for r in rr for j in r[2]], dtype=np.int32)
        out[f"{mth}_xP"] = np.concatenate([r[3] for r in rr]).astype(np.float64)
        out[f"{mth}_counters"] = np.array([r[4] for r in rr], dtype=np.int32)
    np.savez_compressed(OUT, **out)
    print(f"{len(jobs)} solves in {time.perf_counter() - t0:.0f} s with {procs} processes -> {OUT}", flush=True)


if __name__ == "__main__":
    main()
