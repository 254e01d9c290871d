#!/usr/bin/env python3
"""NNLS solves/sec at KKT tol 1e-9 on one MI355X: LHDM against plain LH on the same GPU.

Workload: the large Gaussian instance, m = 4096, n = 16384, A ~ N(0, 1/m), an
820-sparse planted x with |N(0,1)| + 0.1 values, noise std 1e-3, seed 3000
(generated on the host, uploaded to HBM before timing).  LHDM runs with
tau1 = 0.6, tau2 = 0.15, kmax = 32 and delta = 0.8 (the largest value of the
delta sweep); plain LH on the same instance gives the speedup.  One step = one
complete solve (every step of the method, initialisation to KKT).

Prints one JSON line.  Extra objects: ``roofline`` for the dominant kernel (the
dual pass, w = A^T r fused with the projected-norm update, timed live with HIP
events on the solve's stream),
``cpu_baseline`` (the CPU oracle on a bounded sample of the same solve) and
``lh`` (the plain Lawson-Hanson timing).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NNLS solves/sec at KKT tol 1e-9: LHDM vs plain LH, same GPU; batched + backward"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dual_gemv_c3_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2108_05345_amd", "csrc", "lhdm_large.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source():
    """Source text of the dual kernels: their argument struct, the lg_dual_ws
    and lg_colmat2 templates and the launcher (a change anywhere else leaves the
    counters valid)."""
    with open(KERNEL_SRC) as f:
        src = f.read()
    parts = []
    for start, end in (("struct ColmatArgs {", "\n};\n"),
                       ("template <int NT, int CT, int PF, bool DUAL, int DEPTH = 2>", "\n}\n"),
                       ("constexpr int DW_ROWS", "\n\n"),
                       ("template <int NT>\n__global__ __launch_bounds__(DW_WG) void lg_dual_ws", "\n}\n"),
                       ("static void colmat2_launch(", "\n}\n")):
        i = src.index(start)
        parts.append(src[i:src.index(end, i) + len(end)])
    return "".join(parts)


def kernel_hash():
    return hashlib.sha256(kernel_source().encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dual kernel from committed rocprofv3 counters,
    or None when they were taken on a different version of the kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def oracle_full_solve(delta):
    """Wall time of one complete oracle solve of the same instance, as stored by
    the script that wrote the oracle's path fixtures (measured on the host that
    ran it, with its BLAS thread count), or None when that fixture is absent."""
    path = os.path.join(GOLDEN_DIR, f"c3_seed3000_delta{delta:.1f}.npz")
    try:
        import numpy as np
        z = np.load(path, allow_pickle=False)
        return {"seconds": float(z["seconds"]), "solves_per_s": 1.0 / float(z["seconds"]),
                "blas_threads": int(z["threads"]), "host_cpu": str(z["host"]),
                "outer_iters": int(z["counters"][1]), "source": os.path.relpath(path, ROOT)}
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(inst, delta, outer_total, max_outer):
    """The CPU oracle on a bounded sample: the first `max_outer` outer steps of the
    same LHDM solve, scaled by the fraction of the GPU solve's outer steps (an
    estimate: the first steps are the costliest, so it understates the oracle's
    rate; the measured time of a whole oracle solve is reported beside it)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    _, info = oracle.oracle_lhdm(inst.A, inst.b, delta=delta, max_outer=max_outer)
    dt = time.perf_counter() - t0
    done = info["outer_iters"]
    frac = done / max(outer_total, 1)
    return {"value": frac / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "estimate": True,
            "sample": f"estimate: first {done} of {outer_total} outer steps of the same LHDM solve "
                      f"(delta={delta}) in {dt:.1f} s on the host, scaled by {done}/{outer_total}",
            "full_solve_measured": oracle_full_solve(delta)}


def _pmc_rows(path, counter):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def write_traffic(fetch_csv, write_csv):
    """HBM bytes per launch of the dual kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    1 GiB copy of --copy-calibration (1 GiB read, 1 GiB written)."""
    out = {"kernel": "dual pass (lg_dual_ws<NT>, lg_colmat2<3, 4, 2, true, 3>)",
           "workload": "gauss-4096x16384-k820-noise1e-3-seed3000"}
    total = 0.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc_rows(path, name)
        dual = [v for k, v in rows if "lg_dual_ws" in k or ("lg_colmat2" in k and "true" in k)]
        # the 1 GiB copy is by far the largest non-solver dispatch (blit or elementwise kernel)
        copy = [v for k, v in rows if "lg_" not in k and ("copy" in k.lower() or "elementwise" in k.lower())]
        if not dual or not copy:
            raise SystemExit(f"write-traffic: no dual or copy dispatches with {name} in {path}")
        copy_kib = max(copy)
        scale = (1 << 20) / copy_kib            # counter KiB -> true KiB for a known 1 GiB stream
        per = sum(dual) / len(dual) * scale * 1024.0
        out[name.lower()] = {"dispatches": len(dual), "raw_kib_per_dispatch": sum(dual) / len(dual),
                             "copy_kib": copy_kib, "scale": scale, "bytes_per_launch": per}
        total += per
    out["bytes_per_launch"] = total
    out["commands"] = [f"rocprofv3 --pmc {c} --output-format csv -d pmc_{c} -o run -- python3 bench.py --steps 1 "
                       "--warmup 0 --lh-steps 0 --cpu-outer 0 --max-outer 4 --copy-calibration"
                       for c in ("FETCH_SIZE", "WRITE_SIZE")]
    out["commands"].append("python3 bench.py --write-traffic pmc_FETCH_SIZE/run_counter_collection.csv "
                           "pmc_WRITE_SIZE/run_counter_collection.csv")
    out["kernel_src_sha256_16"] = kernel_hash()
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    log("wrote", TRAFFIC_FILE, out)


def check_converged(infos, what):
    """Every timed solve must have converged at KKT tol 1e-9 (the metric's condition)."""
    bad = [i for i in infos if i["status"] != 0 or not (i["kkt_residual"] <= 1e-9)]
    if bad:
        raise SystemExit(f"bench.py: {len(bad)} of {len(infos)} timed {what} solves did not converge: {bad[0]}")
    return max(i["kkt_residual"] for i in infos)


def _summary(infos):
    st = {}
    for i in infos:
        st[str(i["status"])] = st.get(str(i["status"]), 0) + 1
    return {"status_counts": st, "kkt_max": max(i["kkt_residual"] for i in infos),
            "outer_mean": sum(i["outer_iters"] for i in infos) / len(infos),
            "inner_mean": sum(i["inner_iters"] for i in infos) / len(infos),
            "passive_mean": sum(i["n_passive"] for i in infos) / len(infos)}


def _timed(fn, reps):
    """Median wall time (s) of `reps` synchronised calls after one untimed call."""
    import torch
    out = fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2], out


def run_config(name, reps, engine="auto"):
    """Throughput of the other workloads: C1 and C4 (batched, one persistent
    launch), C2 (single solves on the whole-device engine), C5 (batched forward
    and the backward).  Prints one JSON line; the default run (C3) is the
    headline measurement."""
    import numpy as np
    import torch

    import paper_2108_05345_amd as lhdm
    from workloads import make_c1, make_c2, make_c4_batch, make_c5_batch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    out = {"config": name, "data": "synthetic", "dtype": "f64", "timing": f"median of {reps} after 1 warm-up",
           "batch_engine": engine}
    if name in ("c1", "c4", "c5"):
        if name == "c1":
            insts = [make_c1(1000 + i) for i in range(1000)]
        elif name == "c4":
            insts = make_c4_batch(4000)
        else:
            insts = make_c5_batch(5000)
        As = [torch.from_numpy(np.ascontiguousarray(i.A)).to(dev) for i in insts]
        bs = [torch.from_numpy(i.b).to(dev) for i in insts]
        pool = lhdm.pack(As, bs)
        del As, bs
        B = len(insts)
        out["instances"] = B
        out["a_bytes"] = int(pool.A.numel() * 8)
        for meth, use_lh in (("lhdm", False), ("lh", True)):
            t, (x, passive, infos) = _timed(lambda: lhdm.solve_pooled(pool, use_lh=use_lh, engine=engine), reps)
            out[meth] = {"solves_per_s": B / t, "ms_per_batch": 1e3 * t, **_summary(infos)}
            log(name, meth, out[meth])
            if name == "c5" and meth == "lhdm":
                # backward of L = sum ||x_i - t_i||^2 through the final passive sets
                t_all = torch.from_numpy(np.concatenate([i.t for i in insts])).to(dev)
                gx = 2.0 * (x - t_all)
                tb, _ = _timed(lambda: lhdm.backward_pooled(pool, x, passive, gx), reps)
                out["backward"] = {"instances_per_s": B / tb, "ms_per_batch": 1e3 * tb,
                                   "grad_a_bytes_written": int(pool.A.numel() * 8)}
                log(name, "backward", out["backward"])
    elif name == "c2":
        count = 20
        res = {"lhdm": [], "lh": []}
        infos = {"lhdm": [], "lh": []}
        for i in range(count):
            inst = make_c2(2000 + i)
            A = torch.from_numpy(np.asfortranarray(inst.A)).to(dev)
            b = torch.from_numpy(inst.b).to(dev)
            for meth in ("lhdm", "lh"):
                fn = (lambda: lhdm.solve(A, b)) if meth == "lhdm" else (lambda: lhdm.lh_solve(A, b))
                t, r = _timed(fn, max(1, reps // 5))
                res[meth].append(t)
                infos[meth].append(r.info)
            log(name, i, {k: round(1e3 * v[-1], 2) for k, v in res.items()})
            del A, b
        out["instances"] = count
        for meth in ("lhdm", "lh"):
            ts = sorted(res[meth])
            out[meth] = {"solves_per_s": count / sum(ts), "ms_median": 1e3 * ts[len(ts) // 2],
                         **_summary(infos[meth])}
    elif name == "signflip":
        # signed sparse recovery by the positivity trick (Section 3.2): the
        # sign-flip inner loop (Section 4.2) against the ordinary inner loop,
        # for LH and LHDM, on the same GPU and instance ([A, -A] never formed)
        from workloads import make_signed
        m, n, k = 2048, 4096, 512
        inst = make_signed(m, n, k, 7000, noise_std=1e-3)
        A = torch.from_numpy(np.asfortranarray(inst.A)).to(dev)
        b = torch.from_numpy(inst.b).to(dev)
        out["workload"] = f"signed-gauss-{m}x{n}-k{k}-noise1e-3-seed7000"
        for meth, kmax in (("lh", 1), ("lhdm", 32)):
            for flip in (True, False):
                t, r = _timed(lambda: lhdm.solve_signed(A, b, sign_flip=flip, kmax=kmax), max(1, reps // 3))
                key = f"{meth}_{'signflip' if flip else 'innerloop'}"
                out[key] = {"solves_per_s": 1.0 / t, "ms_per_solve": 1e3 * t, **_summary([r.info])}
                log(name, key, out[key])
        out["lh_signflip_over_innerloop"] = out["lh_signflip"]["solves_per_s"] / out["lh_innerloop"]["solves_per_s"]
        out["lhdm_signflip_over_innerloop"] = (out["lhdm_signflip"]["solves_per_s"] /
                                               out["lhdm_innerloop"]["solves_per_s"])
        out["lhdm"], out["lh"] = out["lhdm_signflip"], out["lh_signflip"]
    elif name == "illcond":
        # moderately ill-conditioned instance (condition number ~1e6): LHDM against LH
        from workloads import make_illcond
        m, n, k = 2048, 8192, 160
        inst = make_illcond(m, n, k, 1e5, 8000)
        A = torch.from_numpy(np.asfortranarray(inst.A)).to(dev)
        b = torch.from_numpy(inst.b).to(dev)
        out["workload"] = f"illcond-uniform-rowscaled-{m}x{n}-k{k}-rowrange1e5-seed8000"
        for meth in ("lhdm", "lh"):
            fn = (lambda: lhdm.solve(A, b)) if meth == "lhdm" else (lambda: lhdm.lh_solve(A, b))
            t, r = _timed(fn, max(1, reps // 3))
            out[meth] = {"solves_per_s": 1.0 / t, "ms_per_solve": 1e3 * t, **_summary([r.info])}
            log(name, meth, out[meth])
    else:
        raise SystemExit(f"unknown config {name}")
    out["lhdm_over_lh"] = out["lhdm"]["solves_per_s"] / out["lh"]["solves_per_s"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lh-steps", type=int, default=1)
    ap.add_argument("--delta", type=float, default=0.8)
    ap.add_argument("--cpu-outer", type=int, default=3, help="outer steps of the oracle sample (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=2,
                    help="timed solves at each other delta of the sweep, 0.2 and 0.5 (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--max-outer", type=int, default=0,
                    help="cap on the outer steps of each solve (0: none; for short counter runs)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic file from two rocprofv3 --pmc counter_collection.csv "
                         "files (FETCH_SIZE, WRITE_SIZE) of a --copy-calibration run, then exit")
    ap.add_argument("--config", choices=("c1", "c2", "c4", "c5", "signflip", "illcond"),
                    help="measure another workload instead of the headline one (one JSON line)")
    ap.add_argument("--reps", type=int, default=10, help="timed repeats for --config")
    ap.add_argument("--panel", choices=("auto", "householder"), default="auto",
                    help="block factorisation of the whole-device engine (default: CholeskyQR2 where it applies)")
    ap.add_argument("--engine", choices=("auto", "fused", "fused2", "phased"), default="auto",
                    help="batched engine for --config c1|c4|c5 (default: the library's tuning table)")
    args = ap.parse_args()
    if args.config:
        if args.gpus != 1:
            print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
            sys.exit(2)
        run_config(args.config, args.reps, args.engine)
        return
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2108_05345_amd as lhdm
    from paper_2108_05345_amd import _lib
    from workloads import make_c3

    lib = _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    inst = make_c3(3000)
    m, n = inst.A.shape
    A = torch.from_numpy(np.asfortranarray(inst.A)).to(dev)
    b = torch.from_numpy(inst.b).to(dev)
    assert A.stride() == (1, m)

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")

    for _ in range(args.warmup):
        r = lhdm.solve(A, b, delta=args.delta, max_outer=args.max_outer, panel=args.panel)
        log("warmup lhdm", r.info)
    torch.cuda.synchronize()

    import ctypes
    lib.lhdm_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        r = lhdm.solve(A, b, delta=args.delta, max_outer=args.max_outer, panel=args.panel)
        infos.append(r.info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, kl, kb = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    lib.lhdm_profile_read(ctypes.byref(kms), ctypes.byref(kl), ctypes.byref(kb))
    lib.lhdm_profile_enable(0)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    value = args.steps / (t1 - t0)
    log("lhdm", infos[-1], f"{ms_per_step:.1f} ms/solve")
    kkt_worst = check_converged(infos, "LHDM") if args.max_outer == 0 else None

    lh_value = lh_ms = None
    lh_info = None
    if args.lh_steps > 0:
        torch.cuda.synchronize()
        lh_infos = []
        t2 = time.perf_counter()
        for _ in range(args.lh_steps):
            rl = lhdm.lh_solve(A, b)
            lh_infos.append(rl.info)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        lh_info = lh_infos[-1]
        lh_ms = 1e3 * (t3 - t2) / args.lh_steps
        lh_value = args.lh_steps / (t3 - t2)
        log("lh", lh_info, f"{lh_ms:.1f} ms/solve")
        lh_info = dict(lh_info, kkt_worst=check_converged(lh_infos, "LH"))

    # the other deviation thresholds of the sweep (same instance, same GPU)
    sweep = {}
    if args.sweep_steps > 0 and args.max_outer == 0:
        for d in (0.2, 0.5):
            if d == args.delta:
                continue
            r = lhdm.solve(A, b, delta=d, panel=args.panel)   # untimed first call
            torch.cuda.synchronize()
            sw_infos = []
            t4 = time.perf_counter()
            for _ in range(args.sweep_steps):
                sw_infos.append(lhdm.solve(A, b, delta=d, panel=args.panel).info)
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            sweep[f"delta_{d}"] = {"value": args.sweep_steps / (t5 - t4), "unit": "solves/s",
                                   "ms_per_solve": 1e3 * (t5 - t4) / args.sweep_steps,
                                   "kkt_worst": check_converged(sw_infos, f"LHDM delta={d}"),
                                   "info": sw_infos[-1]}
            log("lhdm delta", d, sweep[f"delta_{d}"])

    roof = None
    if kl.value > 0:
        avg_ms = kms.value / kl.value
        bytes_per = kb.value / kl.value
        achieved = bytes_per / (avg_ms * 1e-3) / 1e9
        traffic = measured_traffic()
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "dual pass: lg_dual_ws<NT> up to 32 directions, lg_colmat2<3, 4, 2, true, 3> up to 48 "
                          "(w = A^T r fused with the projected-norm update)",
                "launches": int(kl.value), "avg_us": round(avg_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": bytes_per}

    cpu = None
    if args.cpu_outer > 0:
        cpu = cpu_baseline(inst, args.delta, infos[-1]["outer_iters"], args.cpu_outer)
        log("cpu baseline", cpu)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gauss-4096x16384-k820-noise1e-3-seed3000", "m": m, "n": n,
                   "method": "lhdm", "tau1": 0.6, "tau2": 0.15, "delta": args.delta, "kmax": 32,
                   "kkt_tol": 1e-9},
        "lhdm_info": dict(infos[-1], kkt_worst=kkt_worst),
        "delta_sweep": sweep or None,
        "lh": None if lh_value is None else {"value": lh_value, "unit": "solves/s", "ms_per_solve": lh_ms,
                                             "info": lh_info},
        "speedup_vs_lh": None if lh_value is None else value / lh_value,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
