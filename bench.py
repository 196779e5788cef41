#!/usr/bin/env python3
"""Throughput of the sparse-projection randomized LU on one MI355X.

One step = one whole decomposition (Algorithm 1 with the exact least-squares
product): sketch, row-pivoted LU of the sketch, least-squares product,
column-pivoted LU, L = L_y L~, on a synthetic dense 16384 x 8192 FP64 matrix
with singular values i^-2 (k = 200, l = 210, s = 2048), resident in HBM.

Prints one JSON line.  `value` is decompositions per second; `roofline`
describes the stage whose kernel dominates the step among the
bandwidth/MFMA-bound ones, timed with HIP events on the library's stream
inside the timed region; `cpu_baseline` times the oracle on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "dense_16384x8192_invsq": dict(m=16384, n=8192, k=200, l=210, s=2048),
    "dense_1024x512_geometric": dict(m=1024, n=512, k=20, l=30, s=256),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense_16384x8192_invsq", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=30.0)
    return ap.parse_args()


def make_input(name, device):
    import numpy as np
    import synth
    w = WORKLOADS[name]
    if name == "dense_16384x8192_invsq":
        return synth.invsq_dense_torch(w["m"], w["n"], device=device)
    import torch
    return torch.from_numpy(synth.small_dense()).to(device)


def cpu_baseline(A_dev, w, seed, budget_s):
    """The oracle as it stands, on the host, on one full decomposition."""
    import numpy as np
    from oracle import rlu as R
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    A = A_dev.cpu().numpy()
    t0 = time.perf_counter()
    R.rlu(A, R.Params(w["k"], w["l"], w["s"], seed))
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "decomps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 full decomposition of the same {w['m']}x{w['n']} matrix ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1601_04280_amd as rlu

    dev = "cuda:0"
    w = WORKLOADS[args.workload]
    seed = 2
    A = make_input(args.workload, dev)
    torch.cuda.synchronize()
    ctx = rlu.Context(0)
    out = rlu.factor(A, k=w["k"], l=w["l"], s=w["s"], seed=seed, ctx=ctx)      # allocates outputs, checks
    for _ in range(args.warmup):
        rlu.factor(A, k=w["k"], l=w["l"], s=w["s"], seed=seed, ctx=ctx, out=out, check=False)
    torch.cuda.synchronize()
    ctx.stage_times()                                                          # clear
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rlu.factor(A, k=w["k"], l=w["l"], s=w["s"], seed=seed, ctx=ctx, out=out, check=False,
                   flags=rlu.RLU_FLAG_TIMING)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, calls = ctx.stage_times()
    info = out.info_dict()
    if info["status"] != 0:
        raise SystemExit(f"device-side failure during the timed steps: {info}")

    m, n, l = w["m"], w["n"], w["l"]
    ms_step = (t1 - t0) * 1e3 / args.steps
    per = {k: v / max(calls, 1) for k, v in stages.items()}
    sketch_bytes = m * n * A.element_size() + 8 * m * l
    sketch_gbs = sketch_bytes / (per["sketch"] * 1e-3) / 1e9
    contract_flops = 2.0 * m * n * l
    contract_tfs = contract_flops / (per["contract"] * 1e-3) / 1e12
    if per["contract"] >= per["sketch"]:
        roof = {"bound": "mfma", "kernel": "contract (W^T = A^T Lhat, FP64 MFMA)",
                "achieved": round(contract_tfs, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(contract_tfs / FP64_PEAK_TFLOPS, 4), "traffic": None}
    else:
        roof = {"bound": "hbm", "kernel": "sketch (fused SEM + SRFT)", "achieved": round(sketch_gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(sketch_gbs / HBM_PEAK_GBS, 4),
                "traffic": None}
    line = {
        "metric": "LU decomps/sec at fixed rel. error; sketch GB/s vs HBM peak; p99 latency",
        "value": round(1e3 / ms_step, 3),
        "unit": "decomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": w["k"], "l": l, "s": w["s"],
                   "storage": str(A.dtype).replace("torch.", ""), "precision": "f64"},
        "roofline": roof,
        "sketch": {"achieved": round(sketch_gbs, 1), "unit": "GB/s", "peak": HBM_PEAK_GBS,
                   "frac": round(sketch_gbs / HBM_PEAK_GBS, 4), "bytes": sketch_bytes},
        "contract": {"achieved": round(contract_tfs, 3), "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
                     "frac": round(contract_tfs / FP64_PEAK_TFLOPS, 4), "flops": contract_flops},
        "stages_ms": {k: round(v, 4) for k, v in per.items()},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A, w, seed, args.cpu_budget_s)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
