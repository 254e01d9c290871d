"""Autotuner of the batched engines (run on the target GPU).

For a grid of batch shapes (instances per compute unit x instance size) it
times the three batched engines of ``lhdm_solve_batched`` (fused with one or
two workgroups per compute unit, phased with one kernel per stage replayed as
a HIP graph) on synthetic instances, picks the fastest per shape and writes

* ``tuning_<arch>.json``: every timing, the device and the command, and
* ``csrc/lhdm_tuning.hpp``: the table the library is compiled with (rows in
  the order ``batch_engine`` tries them).

Instances: A ~ N(0, 1/m) with n = 3 m columns, a 10 %-dense planted x with
U[0.5, 1.5] values and noise std 1e-3 (the shape of the batched workloads
the library is used for).  Only the library under test is called.

    python -m paper_2108_05345_amd.autotune [--out-dir DIR] [--reps 3] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ENGINE_CODES = {"fused": 0, "fused2": 1, "phased": 2}

# (instances per compute unit, m); skipped when A would exceed the byte cap
PER_CU = [0.25, 0.5, 1.0, 2.0, 4.0, 8.0]
M_SIZES = [64, 128, 256, 512, 1024, 2048]
A_BYTES_CAP = 6e9


def _instances(torch, count, m, seed, dev):
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = 3 * m
    As, bs = [], []
    for _ in range(count):
        A = torch.randn(m, n, generator=g, dtype=torch.float64) / m ** 0.5
        x = torch.zeros(n, dtype=torch.float64)
        k = max(1, n // 10)
        idx = torch.randperm(n, generator=g)[:k]
        x[idx] = 0.5 + torch.rand(k, generator=g, dtype=torch.float64)
        b = A @ x + 1e-3 * torch.randn(m, generator=g, dtype=torch.float64)
        As.append(A.to(dev))
        bs.append(b.to(dev))
    return As, bs


def _time(lhdm, torch, pool, engine, reps):
    lhdm.solve_pooled(pool, engine=engine)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, infos = lhdm.solve_pooled(pool, engine=engine)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    bad = sum(1 for i in infos if i["status"] != 0)
    ts.sort()
    return ts[len(ts) // 2], bad


def header_text(rows, device):
    lines = [
        "// Batched-engine table: written by paper_2108_05345_amd/autotune.py from",
        f"// timings on {device}.  Rows are tried in order; the first whose",
        "// bounds hold gives the engine (0: fused, one workgroup per compute unit;",
        "// 1: fused, two per compute unit; 2: phased).",
        "#pragma once",
        "",
        "namespace lhdm {",
        "",
        "struct TuneRow {",
        "    double per_cu_hi;   // instances per compute unit <= this",
        "    int m_hi;           // largest m of the batch <= this",
        "    int engine;",
        "};",
        "",
        "static const TuneRow kTuneRows[] = {",
    ]
    for r in rows:
        lines.append(f"    {{{r['per_cu_hi']!r}, {r['m_hi']}, {r['engine']}}},")
    lines += ["    {1e300, 1 << 30, 0},", "};", "", "}  // namespace lhdm", ""]
    return "\n".join(lines)


def table_rows(results):
    """One row per measured (per_cu, m) cell, ordered so that the first match
    is the nearest measured cell at or above the batch's shape."""
    rows = []
    for pc in sorted({r["per_cu"] for r in results}):
        for m in sorted({r["m"] for r in results if r["per_cu"] == pc}):
            cell = [r for r in results if r["per_cu"] == pc and r["m"] == m][0]
            rows.append({"per_cu_hi": pc, "m_hi": m, "engine": ENGINE_CODES[cell["best"]]})
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out-dir", default=HERE, help="where tuning_<arch>.json and csrc/lhdm_tuning.hpp go")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="a reduced grid (smoke test of the tuner)")
    args = ap.parse_args(argv)

    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2108_05345_amd as lhdm

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    arch = getattr(props, "gcnArchName", "gfx").split(":")[0]
    per_cu = [0.5, 2.0] if args.quick else PER_CU
    m_sizes = [64, 256] if args.quick else M_SIZES
    results = []
    for m in m_sizes:
        for pc in per_cu:
            count = max(1, int(round(pc * cus)))
            if count * m * 3 * m * 8 > A_BYTES_CAP:
                continue
            As, bs = _instances(torch, count, m, 1000 * m + int(pc * 8), dev)
            pool = lhdm.pack(As, bs)
            del As, bs
            cell = {"per_cu": pc, "m": m, "n": 3 * m, "instances": count, "seconds": {}, "not_converged": {}}
            for eng in ENGINE_CODES:
                t, bad = _time(lhdm, torch, pool, eng, args.reps)
                cell["seconds"][eng] = t
                cell["not_converged"][eng] = bad
            cell["best"] = min(cell["seconds"], key=cell["seconds"].get)
            print(json.dumps(cell), flush=True)
            results.append(cell)
            del pool
            torch.cuda.empty_cache()
    rows = table_rows(results)
    device = f"{props.name} ({arch}, {cus} CUs)"
    os.makedirs(os.path.join(args.out_dir, "csrc"), exist_ok=True)
    with open(os.path.join(args.out_dir, f"tuning_{arch}.json"), "w") as f:
        json.dump({"device": device, "command": "python -m paper_2108_05345_amd.autotune " + " ".join(argv or sys.argv[1:]),
                   "instances": "A ~ N(0,1/m), n = 3m, 10%-dense planted x in U[0.5,1.5], noise 1e-3",
                   "cells": results, "rows": rows}, f, indent=1)
    with open(os.path.join(args.out_dir, "csrc", "lhdm_tuning.hpp"), "w") as f:
        f.write(header_text(rows, device))
    print(f"wrote {len(rows)} rows for {device}", flush=True)


if __name__ == "__main__":
    main()
