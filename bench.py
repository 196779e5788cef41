#!/usr/bin/env python3
"""Throughput of the sparse-projection randomized LU on one MI355X.

One step = one whole decomposition (Algorithm 1 with the exact least-squares
product): sketch, row-pivoted LU of the sketch, least-squares product,
column-pivoted LU, L = L_y L~.  The headline workload is a synthetic dense
16384 x 8192 FP64 matrix with singular values i^-2 (k = 200, l = 210,
s = 2048), resident in HBM.

Prints one JSON line.  `value` is decompositions per second of the headline
workload; `roofline` describes the stage whose kernels dominate the step
among the bandwidth/MFMA-bound ones, timed with HIP events on the library's
stream inside the timed region; `cpu_baseline` times the oracle on the host.
Unless --no-extras (or a shorter --extras list), the line also carries
  `forms`: the 32768 x 16384 FP32-stored matrix with sigma_i = exp(-i/100)
           (k = 500, l = 520, s = 4096) decomposed with the contraction in
           FP64, FP32 and BF16 + one refinement step, side by side, each with
           its relative residual ||LU - PAQ||_F / ||A||_F;
  `transforms`: the headline matrix sketched with the real Fourier and with
           the Walsh-Hadamard transform (time, sketch rate, residual);
  `second_projection`: the headline matrix with B from the paper's second
           projection Omega_2 (k2, l2 = 840, 4096; 840, 2048; 420, 2048)
           in place of the exact product: time, residual against the exact
           product's, and the rate of the Omega_2 pass over A;
  `csr`:   the 200000 x 100000 CSR matrix at 0.1% density with a rank-50
           plant (k = 100, l = 110, s = 4096);
  `serving`: the request mix through the continuous-batching loop: m
           log-uniform in [512, 8192], n in [256, 4096], k in {16 .. 256},
           l = k + 10, s = min(n, 8k), 30% BF16-refined, dense
           low-rank-plus-noise (sigma_i = 2^-(i-1), r = 20, noise 1e-10);
           Poisson arrivals at 0.05 (latency close to the service time
           alone), 0.5, 0.7 and 0.9 of the measured saturated rate, p50 /
           p99 latency (completion - arrival) and decomps/s;
  `accuracy`: the experiments of Section 4.1 (sigma_1..r = 1, then e^-10 down
           to e^-200) and 4.2 (sigma from 1 down to e^-100) on 5000 x 5000
           matrices: ||LU - PAQ||_F against Delta_r and the time, per rank r.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
EXTRAS = ("transforms", "second_projection", "forms", "csr", "serving", "accuracy")
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}

WORKLOADS = {
    "dense_16384x8192_invsq": dict(m=16384, n=8192, k=200, l=210, s=2048, precision="f64"),
    "dense_1024x512_geometric": dict(m=1024, n=512, k=20, l=30, s=256, precision="f64"),
    "dense_32768x16384_exp_fp32": dict(m=32768, n=16384, k=500, l=520, s=4096, precision="bf16"),
    "csr_200000x100000_planted": dict(m=200000, n=100000, k=100, l=110, s=4096, precision="f64"),
}
SEED = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense_16384x8192_invsq", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", choices=["f64", "f32", "bf16"], default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip every oracle run: the CPU baseline, the headline parity key and the forms' oracle errors")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated blocks to add to the line (default: all of %s)" % ", ".join(EXTRAS))
    ap.add_argument("--gaussian-data", action="store_true",
                    help="N(0,1) entries of the workload's shape instead of its spectrum (for counter runs: "
                         "the kernels' memory traffic does not depend on the values, and the profiler "
                         "cannot run the QR that builds the spectrum)")
    ap.add_argument("--probe-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers three times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    return ap.parse_args()


def make_input(name, device):
    """Device-resident input: a tensor (dense) or (row_ptr, col, val, m, n)."""
    import torch
    import synth
    if name == "dense_16384x8192_invsq":
        return synth.invsq_dense_torch(16384, 8192, device=device)
    if name == "dense_32768x16384_exp_fp32":
        return synth.exp_dense_fp32_torch(32768, 16384, device=device)
    if name == "csr_200000x100000_planted":
        rp, col, val = synth.planted_csr()
        return (torch.from_numpy(rp).to(device), torch.from_numpy(col).to(device),
                torch.from_numpy(val).to(device), 200000, 100000)
    return torch.from_numpy(synth.small_dense()).to(device)


def input_bytes(A):
    if isinstance(A, tuple):
        rp, col, val, m, n = A
        return rp.numel() * 4 + col.numel() * 4 + val.numel() * 8
    return A.numel() * A.element_size()


def run(rlu, A, w, precision, steps, warmup, ctx, flags=0, extra=None):
    """Warm-up, then `steps` timed decompositions; returns timings and the output.
    The bench owns the device, so the calls say so (RLU_FLAG_EXCLUSIVE: the LU
    panels are ordinary launches instead of cooperative ones)."""
    import torch
    kw = dict(k=w["k"], l=w["l"], s=w["s"], seed=SEED, ctx=ctx, precision=precision, **(extra or {}))
    if isinstance(A, tuple):
        kw["csr"] = A
        A = None
    base = flags | rlu.RLU_FLAG_EXCLUSIVE
    out = rlu.factor(A, flags=base, **kw)                       # allocates outputs, checks status
    for _ in range(warmup):
        rlu.factor(A, out=out, check=False, flags=base, **kw)
    torch.cuda.synchronize()
    ctx.stage_times()                                           # clear
    # timed: HIP events around the contraction only (the roofline's kernel);
    # events at every stage boundary would idle the device a few us each
    t0 = time.perf_counter()
    for _ in range(steps):
        rlu.factor(A, out=out, check=False, flags=rlu.RLU_FLAG_TIMING_CONTRACT | base, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, calls = ctx.stage_times()
    contract = stages["contract"] / max(calls, 1)
    # the stage breakdown, from the same number of calls after the timed region
    for _ in range(steps):
        rlu.factor(A, out=out, check=False, flags=rlu.RLU_FLAG_TIMING | base, **kw)
    torch.cuda.synchronize()
    stages, calls = ctx.stage_times()
    info = out.info_dict()
    if info["status"] != 0:
        raise SystemExit(f"device-side failure during the timed steps: {info}")
    per = {k: v / max(calls, 1) for k, v in stages.items()}
    per["contract_timed"] = contract
    return (t1 - t0) * 1e3 / steps, per, out


def rel_residual(A, out):
    """||LU - PAQ||_F / ||A||_F in FP64 on the device (a check, outside the timing)."""
    import torch
    A64 = A.double()
    pr, pc = out.perm_r.long(), out.perm_c.long()
    R = out.L @ out.U
    R -= A64[pr][:, pc]
    r = (torch.linalg.norm(R) / torch.linalg.norm(A64)).item()
    del R, A64
    torch.cuda.empty_cache()
    return r


def sketch_rate(A, w, per):
    byts = input_bytes(A) + 8 * w["m"] * w["l"]
    gbs = byts / (per["sketch"] * 1e-3) / 1e9
    return {"achieved": round(gbs, 1), "unit": "GB/s", "peak": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes": byts}


def contract_rate(w, per, precision):
    flops = 2.0 * w["m"] * w["n"] * w["l"] * (1 if precision != "bf16" else 5)  # BF16: W0, 3 split products, dW
    # the contraction's events inside the timed region; the BF16 form's product
    # also spans the solve stage, from the breakdown pass
    ms = per["contract"] + per["solve"] if precision == "bf16" else per.get("contract_timed", per["contract"])
    tfs = flops / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    return {"achieved": round(tfs, 3), "unit": "TFLOP/s", "peak": peak, "frac": round(tfs / peak, 4),
            "flops": flops}


def measured_traffic(kernel_key):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the kernel source as it is now (else None)."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)[kernel_key]
        src = os.path.join(HERE, rec["source"])
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if sha != rec["source_sha256"]:
            return None
        return rec["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    """The host's CPU as lscpu reports it (model, sockets x cores x threads)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = dict((a.strip(), b.strip()) for a, b in (ln.split(":", 1) for ln in out.splitlines() if ":" in ln))
        sockets = int(kv.get("Socket(s)", "1"))
        cores = int(kv.get("Core(s) per socket", "0"))
        tpc = int(kv.get("Thread(s) per core", "1"))
        info = {"model": kv.get("Model name", "?"), "sockets": sockets, "cores_per_socket": cores,
                "threads_per_core": tpc, "physical_cores": sockets * cores, "smt": tpc > 1,
                "logical_cpus": int(kv.get("CPU(s)", "0"))}
    except Exception as e:  # pragma: no cover
        info = {"model": f"lscpu failed: {e}"}
    try:
        info["cpus_available_to_process"] = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        pass
    return info


def cpu_baseline(A_dev, w, runs=3):
    """The oracle as it stands, on the host: `runs` full decompositions of the
    same matrix with the BLAS on every thread it was given (median), and one
    with the BLAS on a single thread.  Returns the record and the oracle's
    result of the last all-thread run (for the parity check)."""
    import numpy as np
    from oracle import rlu as R
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    A = A_dev.cpu().numpy()
    p = R.Params(w["k"], w["l"], w["s"], SEED)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        o = R.rlu(A, p)
        times.append(time.perf_counter() - t0)
        print(f"# cpu baseline: {times[-1]:.1f} s", file=sys.stderr, flush=True)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        R.rlu(A, p)
        t1 = time.perf_counter() - t0
    med = float(np.median(times))
    rec = {"value": round(1.0 / med, 5), "unit": "decomps/s", "cores": int(threads), "kind": "oracle",
           "sample": f"full decompositions of the same {w['m']}x{w['n']} matrix and seed: median of {runs} "
                     f"({', '.join(f'{t:.1f}' for t in times)} s) with the BLAS on {threads} threads; the "
                     "oracle's pivot loops are single-threaded NumPy, only its QR and products use the BLAS",
           "single_thread": {"value": round(1.0 / t1, 5), "unit": "decomps/s", "seconds": round(t1, 2)},
           "host": host_cpu()}
    return rec, o


def parity_block(rlu, A_dev, w, ctx, o):
    """The headline decomposition against the oracle's on the same matrix and
    seed: pivots, Y, and the product ||L_g U_g - L_o U_o||_F / ||A||_F (the
    A19 bar is 1e-10), formed on the device in FP64."""
    import numpy as np
    import torch
    g = rlu.factor(A_dev, k=w["k"], l=w["l"], s=w["s"], seed=SEED, ctx=ctx, keep_intermediates=True)
    torch.cuda.synchronize()
    dev = A_dev.device
    Lo, Uo = torch.from_numpy(o.L).to(dev), torch.from_numpy(o.U).to(dev)
    a_fro = torch.linalg.norm(A_dev.double()).item()
    diff = (torch.linalg.norm(g.L @ g.U - Lo @ Uo) / a_fro).item()
    Yo = torch.from_numpy(o.Y).to(dev)
    info = g.info_dict()
    res = {"oracle_seed": SEED,
           "perm_r_identical": bool(np.array_equal(g.perm_r.cpu().numpy(), o.perm_r)),
           "perm_c_identical": bool(np.array_equal(g.perm_c.cpu().numpy(), o.perm_c)),
           "lu_product_rel_diff": diff,
           "y_rel_diff": (torch.linalg.norm(g.Y - Yo) / torch.linalg.norm(Yo)).item(),
           "oracle_min_gap_y": float(o.min_gap_y), "oracle_min_gap_b": float(o.min_gap_b),
           "gpu_min_gap_y": info["min_gap_y"], "gpu_min_gap_b": info["min_gap_b"],
           "rel_residual_gpu": rel_residual(A_dev, g)}
    A64 = A_dev.double()
    Rm = Lo @ Uo
    Rm -= A64[torch.from_numpy(o.perm_r).to(dev)][:, torch.from_numpy(o.perm_c).to(dev)]
    res["rel_residual_oracle"] = (torch.linalg.norm(Rm) / a_fro).item()
    res["pass"] = bool(res["perm_r_identical"] and res["perm_c_identical"] and diff <= 1e-10
                       and res["y_rel_diff"] <= 1e-10)
    del g, Lo, Uo, Yo, A64, Rm
    torch.cuda.empty_cache()
    print(f"# parity with the oracle: pivots {res['perm_r_identical']}/{res['perm_c_identical']}, "
          f"product {diff:.2e}", file=sys.stderr, flush=True)
    return res


def unpermuted_product(L, U, perm_r, perm_c):
    """P^T (L U) Q^T: the approximation of A in A's own row and column order."""
    import torch
    D = torch.empty(L.shape[0], U.shape[1], dtype=torch.float64, device=L.device)
    D[perm_r.long().unsqueeze(1), perm_c.long().unsqueeze(0)] = L @ U
    return D


def forms_block(rlu, ctx, dev, with_oracle=True):
    import torch
    name = "dense_32768x16384_exp_fp32"
    w = WORKLOADS[name]
    A = make_input(name, dev)
    torch.cuda.synchronize()
    res = {"workload": name, "m": w["m"], "n": w["n"], "k": w["k"], "l": w["l"], "s": w["s"], "storage": "float32"}
    oracle = None
    if with_oracle:   # the FP64 oracle on the same matrix and seed, for the error of every form
        import numpy as np
        from oracle import rlu as R
        t0 = time.perf_counter()
        A64h = A.cpu().numpy().astype(np.float64)
        o = R.rlu(A64h, R.Params(w["k"], w["l"], w["s"], SEED))
        del A64h
        oracle = {"perm_r": o.perm_r, "perm_c": o.perm_c,
                  "LU": unpermuted_product(torch.from_numpy(o.L).to(dev), torch.from_numpy(o.U).to(dev),
                                           torch.from_numpy(o.perm_r).to(dev), torch.from_numpy(o.perm_c).to(dev))}
        oracle["rel_residual"] = (torch.linalg.norm(oracle["LU"] - A.double()) / torch.linalg.norm(A.double())).item()
        res["oracle"] = {"seconds": round(time.perf_counter() - t0, 1), "rel_residual": oracle["rel_residual"],
                         "min_gap_y": float(o.min_gap_y), "min_gap_b": float(o.min_gap_b)}
        del o
        print(f"# forms: oracle in {res['oracle']['seconds']} s", file=sys.stderr, flush=True)
    for prec in ("f64", "f32", "bf16"):
        ms, per, out = run(rlu, A, w, prec, steps=5, warmup=1, ctx=ctx)
        res[prec] = {"ms_per_step": round(ms, 3), "decomps_per_s": round(1e3 / ms, 3),
                     "rel_residual": rel_residual(A, out),
                     "contract": contract_rate(w, per, prec),
                     "stages_ms": {k: round(v, 4) for k, v in per.items()}}
        if oracle is not None:   # the error of this result against the FP64 oracle
            import numpy as np
            a_fro = torch.linalg.norm(A.double()).item()
            LUg = unpermuted_product(out.L, out.U, out.perm_r.long(), out.perm_c.long())
            res[prec]["vs_oracle"] = {
                "perm_r_identical": bool(np.array_equal(out.perm_r.cpu().numpy(), oracle["perm_r"])),
                "perm_c_identical": bool(np.array_equal(out.perm_c.cpu().numpy(), oracle["perm_c"])),
                "lu_rel_diff": (torch.linalg.norm(LUg - oracle["LU"]) / a_fro).item(),
                "residual_rel_diff": abs(res[prec]["rel_residual"] - oracle["rel_residual"]) / oracle["rel_residual"]}
            del LUg
        del out
        print(f"# forms {prec}: {ms:.2f} ms/step, residual {res[prec]['rel_residual']:.6e}", file=sys.stderr,
              flush=True)
    r64 = res["f64"]["rel_residual"]
    for prec in ("f32", "bf16"):
        res[prec]["residual_rel_diff_vs_f64"] = abs(res[prec]["rel_residual"] - r64) / r64
        res[prec]["speedup_vs_f64"] = round(res["f64"]["ms_per_step"] / res[prec]["ms_per_step"], 3)
    res["sketch"] = sketch_rate(A, w, per)
    del A
    torch.cuda.empty_cache()
    return res


def transforms_block(rlu, A, w, ctx, ms_fourier, per_fourier, out_fourier):
    """The headline matrix with the sketch's transform as the Walsh-Hadamard
    matrix (RLU_FLAG_HADAMARD) beside the real Fourier one: time, sketch rate,
    relative residual."""
    import torch
    res = {"fourier": {"ms_per_step": round(ms_fourier, 4), "decomps_per_s": round(1e3 / ms_fourier, 3),
                       "sketch": sketch_rate(A, w, per_fourier), "rel_residual": rel_residual(A, out_fourier)}}
    ms, per, out = run(rlu, A, w, "f64", steps=20, warmup=3, ctx=ctx, flags=rlu.RLU_FLAG_HADAMARD)
    res["hadamard"] = {"ms_per_step": round(ms, 4), "decomps_per_s": round(1e3 / ms, 3),
                       "sketch": sketch_rate(A, w, per), "rel_residual": rel_residual(A, out)}
    del out
    torch.cuda.empty_cache()
    print(f"# transforms: fourier {ms_fourier:.3f} ms, hadamard {ms:.3f} ms/step", file=sys.stderr, flush=True)
    return res


def second_block(rlu, A, w, ctx, ms_exact, out_exact, shapes=((840, 4096), (840, 2048), (420, 2048))):
    """The headline matrix with B from the paper's second projection Omega_2
    (k2 x m, SEM width l2; Algorithm 1 steps 4-5) instead of the exact
    product: time, relative residual, and the Omega_2 pass over A (the
    contraction stage: gather, transform, transpose) as a rate over A's bytes."""
    import torch
    r_exact = rel_residual(A, out_exact)
    res = {"exact": {"ms_per_step": round(ms_exact, 4), "decomps_per_s": round(1e3 / ms_exact, 3),
                     "rel_residual": r_exact}}
    for k2, l2 in shapes:
        ms, per, out = run(rlu, A, w, "f64", steps=20, warmup=3, ctx=ctx, extra={"k2": k2, "l2": l2})
        r = rel_residual(A, out)
        a_bytes = A.numel() * A.element_size()
        res[f"k2_{k2}_l2_{l2}"] = {
            "k2": k2, "l2": l2, "ms_per_step": round(ms, 4), "decomps_per_s": round(1e3 / ms, 3),
            "rel_residual": r, "residual_vs_exact": round(r / r_exact, 4),
            "omega2_pass_ms": round(per["contract_timed"], 4),
            "omega2_pass_GBs_over_A": round(a_bytes / (per["contract_timed"] * 1e-3) / 1e9, 1),
            "stages_ms": {k: round(v, 4) for k, v in per.items() if k != "contract_timed"}}
        del out
        torch.cuda.empty_cache()
        print(f"# second projection k2={k2} l2={l2}: {ms:.3f} ms/step, residual x{r / r_exact:.3f}",
              file=sys.stderr, flush=True)
    return res


def sweep_params(r, n):
    """k = r, l = r + 10, s = the power of two at or above 4 l (at most 8192)."""
    l = r + 10
    s = 1
    while s < 4 * l:
        s *= 2
    return dict(k=r, l=l, s=min(s, 8192))


def accuracy_block(rlu, ctx, dev, n=5000, ranks_41=(50, 100, 200, 300, 400, 500, 600, 700, 800, 900),
                   ranks_42=(10, 50, 100, 200, 300, 400, 500, 600, 700, 800, 900), steps=3):
    """The accuracy experiments of Section 4.1 and 4.2 on n x n matrices
    (singular vectors random): the error ||LU - PAQ||_F against
    Delta_r = sqrt(sum_{i > r} sigma_i^2) and the time per decomposition.
    4.1: sigma_1..r = 1, the rest from e^-10 down to e^-200, r varying (the
    matrix changes with r); 4.2: sigma from 1 down to e^-100, one matrix,
    rank r varying.  Ranks up to 900, the largest of Section 4.1 (l = r + 10)."""
    import numpy as np
    import torch
    import synth

    def one(A, sig, r):
        p = sweep_params(r, n)
        out = rlu.factor(A, seed=SEED, ctx=ctx, **p)
        for _ in range(1):
            rlu.factor(A, seed=SEED, ctx=ctx, out=out, check=False, **p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rlu.factor(A, seed=SEED, ctx=ctx, out=out, check=False, **p)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        pr, pc = out.perm_r.long(), out.perm_c.long()
        err = float(torch.linalg.norm(out.L @ out.U - A[pr][:, pc]))
        delta = float(np.sqrt(np.sum(np.asarray(sig)[r:] ** 2)))
        return {"r": r, **p, "ms": round(ms, 3), "err_fro": err, "delta_r": delta,
                "err_over_delta": round(err / delta, 4)}

    res = {"n": n, "sec_4_1": [], "sec_4_2": []}
    for r in ranks_41:
        sig = synth.spectrum_step_exp(n, r)
        A = synth.lowrank_dense_torch(n, n, sig, synth.DATA_SEED_BASE + 41 + r, device=dev)
        res["sec_4_1"].append(one(A, sig, r))
        del A
    sig = synth.spectrum_exp_range(n)
    A = synth.lowrank_dense_torch(n, n, sig, synth.DATA_SEED_BASE + 42, device=dev)
    for r in ranks_42:
        res["sec_4_2"].append(one(A, sig, r))
    del A
    torch.cuda.empty_cache()
    worst = max(x["err_over_delta"] for x in res["sec_4_1"] + res["sec_4_2"])
    print(f"# accuracy sweeps (n = {n}): worst ||LU - PAQ||_F / Delta_r = {worst}", file=sys.stderr, flush=True)
    return res


def csr_block(rlu, ctx, dev):
    import torch
    name = "csr_200000x100000_planted"
    w = WORKLOADS[name]
    A = make_input(name, dev)
    ms, per, out = run(rlu, A, w, "f64", steps=10, warmup=2, ctx=ctx)
    res = {"workload": name, "m": w["m"], "n": w["n"], "nnz": int(A[2].numel()), "k": w["k"], "l": w["l"],
           "s": w["s"], "ms_per_step": round(ms, 3), "decomps_per_s": round(1e3 / ms, 3),
           "sketch": sketch_rate(A, w, per), "stages_ms": {k: round(v, 4) for k, v in per.items()}}
    print(f"# csr: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    del out
    # the paper's second projection on the same input (time only)
    k2, l2 = 4 * w["l"], 2048
    ms2, per2, out2 = run(rlu, A, w, "f64", steps=10, warmup=2, ctx=ctx, extra={"k2": k2, "l2": l2})
    res["second_projection"] = {"k2": k2, "l2": l2, "ms_per_step": round(ms2, 3),
                                "decomps_per_s": round(1e3 / ms2, 3),
                                "stages_ms": {k: round(v, 4) for k, v in per2.items()}}
    print(f"# csr, second projection k2={k2} l2={l2}: {ms2:.2f} ms/step", file=sys.stderr, flush=True)
    del A, out2
    torch.cuda.empty_cache()
    return res


def serve_block(rlu, dev, counts=(300, 600, 2000, 600), fracs=(0.05, 0.5, 0.7, 0.9), n_sat=2000, max_inflight=8):
    import numpy as np
    import torch
    import synth
    shapes = synth.serving_shapes(max(counts + (n_sat,)), seed=7)
    # requests take top-left blocks of four 8192 x 4096 low-rank-plus-noise matrices
    base = [synth.lowrank_dense_torch(8192, 4096, synth.spectrum_geometric(20), 1000 + i, noise=1e-10, device=dev)
            for i in range(4)]
    torch.cuda.synchronize()
    infos = []
    srv = rlu.Server(hbm_budget_bytes=16 << 30, max_inflight=max_inflight)

    def submit(i):
        sh = shapes[i]
        out = rlu.alloc_factors(sh["m"], sh["n"], sh["l"], 0)
        infos.append(out.info)
        return srv.submit(base[i % 4][: sh["m"], : sh["n"]], k=sh["k"], l=sh["l"], s=sh["s"], seed=SEED + i,
                          precision=sh["precision"], out=out, sync_inputs=False)

    def run(arrivals):
        count = len(arrivals)
        outstanding, lat = {}, np.zeros(count)
        i = done = 0
        t0 = time.perf_counter()
        while done < count:
            now = time.perf_counter() - t0
            while i < count and arrivals[i] <= now:
                outstanding[submit(i)] = i
                i += 1
            for t in list(outstanding):
                if srv.poll(t) is not None:
                    j = outstanding.pop(t)
                    lat[j] = time.perf_counter() - t0 - arrivals[j]
                    done += 1
            if not outstanding and i < count:
                time.sleep(max(0.0, min(1e-3, arrivals[i] - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
        return wall, lat

    run(np.zeros(16))                                          # warm-up
    wall, _ = run(np.zeros(n_sat))                             # saturated: everything queued at t = 0
    sat = n_sat / wall
    res = {"workload": "serving_mix", "max_inflight": max_inflight, "pool_bytes": 16 << 30,
           "saturated_decomps_per_s": round(sat, 2), "bf16_fraction": round(
               sum(sh["precision"] == "bf16" for sh in shapes[: max(counts)]) / max(counts), 3), "runs": []}
    rng = np.random.default_rng(SEED + 1)
    for frac, count in zip(fracs, counts):
        rate = frac * sat
        arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
        wall, lat = run(arrivals)
        res["runs"].append({"rate_frac": frac, "rate_per_s": round(rate, 2), "requests": count,
                            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                            "mean_ms": round(float(lat.mean()) * 1e3, 3),
                            "decomps_per_s": round(count / wall, 2)})
        print(f"# serving {frac:.2f} x saturated ({rate:.0f}/s): p50 {res['runs'][-1]['p50_ms']} ms, "
              f"p99 {res['runs'][-1]['p99_ms']} ms", file=sys.stderr, flush=True)
    res["loop"] = srv.stats()
    srv.stop()
    bad = int((torch.stack(infos)[:, 0] != 0).sum().item())
    if bad:
        raise SystemExit(f"{bad} served requests reported a device-side failure")
    res["requests_checked"] = len(infos)
    del base
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.probe_copy:
        n = max(1, args.probe_copy // 8)
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "launches": 3, "bytes_read_per_launch": n * 8,
                          "bytes_written_per_launch": n * 8}), flush=True)
        return
    import paper_1601_04280_amd as rlu

    dev = "cuda:0"
    w = WORKLOADS[args.workload]
    precision = args.precision or w["precision"]
    ctx = rlu.Context(0)
    if args.gaussian_data and args.workload.startswith("dense"):
        g = torch.Generator(device=dev)
        g.manual_seed(SEED)
        dt = torch.float32 if "fp32" in args.workload else torch.float64
        A = torch.randn(w["m"], w["n"], generator=g, device=dev, dtype=torch.float64).to(dt)
    else:
        A = make_input(args.workload, dev)
    torch.cuda.synchronize()
    ms_step, per, out = run(rlu, A, w, precision, args.steps, args.warmup, ctx)
    print(f"# {args.workload} {precision}: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    sk = sketch_rate(A, w, per)
    is_csr = isinstance(A, tuple)
    if is_csr:
        ct = None
        roof_contract = False
    else:
        ct = contract_rate(w, per, precision)
        roof_contract = per["contract"] >= per["sketch"]
    if roof_contract:
        key = f"contract_{precision}_{args.workload}"
        traffic = measured_traffic(key)
        roof = {"bound": "mfma", "kernel": f"contract stage ({precision} MFMA GEMM W^T = A^T Lhat)",
                "achieved": ct["achieved"], "peak": ct["peak"], "unit": "TFLOP/s", "frac": ct["frac"],
                "traffic": traffic, "stage_ms": round(per.get("contract_timed", per["contract"]), 4)}
    else:
        key = f"sketch_{args.workload}"
        traffic = measured_traffic(key)
        roof = {"bound": "hbm", "kernel": "sketch (SEM + SRFT)", "achieved": sk["achieved"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": sk["frac"], "traffic": traffic}
    storage = "csr_f64" if is_csr else str(A.dtype).replace("torch.", "")
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
        "dtype": precision,
        "data": "synthetic" if not args.gaussian_data else "synthetic-gaussian",
        "config": {"workload": args.workload, "m": w["m"], "n": w["n"], "k": w["k"], "l": w["l"], "s": w["s"],
                   "storage": storage, "precision": precision, "launch": "exclusive device"},
        "roofline": roof,
        "sketch": sk,
        "stages_ms": {k: round(v, 4) for k, v in per.items() if k != "contract_timed"},
    }
    if ct is not None:
        line["contract"] = ct
    extras = set() if args.no_extras else {e.strip() for e in args.extras.split(",") if e.strip()}
    unknown = extras - set(EXTRAS)
    if unknown:
        raise SystemExit(f"unknown extras {sorted(unknown)}; choose from {EXTRAS}")
    if not is_csr and precision == "f64":
        if "transforms" in extras:
            line["transforms"] = transforms_block(rlu, A, w, ctx, ms_step, per, out)
        if "second_projection" in extras:
            line["second_projection"] = second_block(rlu, A, w, ctx, ms_step, out)
    del out
    if not args.no_cpu_baseline and not is_csr:
        line["cpu_baseline"], o = cpu_baseline(A, w)
        if not args.gaussian_data:
            line["parity"] = parity_block(rlu, A, w, ctx, o)
        del o
    del A
    torch.cuda.empty_cache()
    if "forms" in extras:
        line["forms"] = forms_block(rlu, ctx, dev, with_oracle=not args.no_cpu_baseline)
    if "csr" in extras:
        line["csr"] = csr_block(rlu, ctx, dev)
    if "serving" in extras:
        line["serving"] = serve_block(rlu, dev)
        # one slot: requests one at a time with the device to themselves,
        # launched as captured graphs (rlu_serve_stats)
        line["serving"]["one_slot"] = serve_block(rlu, dev, counts=(600,), fracs=(0.7,), n_sat=300, max_inflight=1)
    if "accuracy" in extras:
        line["accuracy"] = accuracy_block(rlu, ctx, dev)
    # release the library's streams and events while the runtime is whole
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
