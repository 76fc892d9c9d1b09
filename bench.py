#!/usr/bin/env python3
"""Benchmark of the POLFED hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

A step is one full POLFED solve (bounds Lanczos, filter order, block Lanczos
with the Chebyshev filter, full reorthogonalisation, T_m eigensolves,
Rayleigh-Ritz, residuals, eigenvectors copied back) of one synthetic chain.
The default workload is the L=18 J1-J2 chain (J2=1, Delta=1, W=2, 50
eigenpairs nearest the middle of the spectrum, block size 16, FP64).

Prints one JSON line: the metric is H.V applications per second (one
application = H~ applied to one vector; the solve's total over its wall
time), with the time to N_ev (ms_per_step), the roofline of the dominant
kernel (the fused Chebyshev step, HIP-event timed inside the library on the
stream it runs on), the oracle's CPU throughput on a bounded sample, and the
same solve with the FP32 filter for comparison.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "H·V applications/s (achieved HBM GB/s) + time to N_ev eigenpairs, FP32 vs FP64"


def _kernel_hash():
    with open(os.path.join(ROOT, "paper_2005_09534_amd", "csrc", "hv.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload, shape):
    """HBM bytes per step launch from committed rocprofv3 --pmc summaries
    (FETCH_SIZE / WRITE_SIZE, scaled by the copy-kernel calibration), or
    None when absent, taken on a different kernel source or launch shape."""
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_traffic.txt")
    if not os.path.exists(path) or shape is None:
        return None
    txt = open(path).read()
    kv = dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", txt, flags=re.M))
    if kv.get("kernel_source_sha256_16") != _kernel_hash():
        return None
    if kv.get("step_shape") != ",".join(str(int(v)) for v in shape):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _fp64_single_estimate(ctx, pf, wl, batch_s):
    """The plain FP64 path on the same realisations, one polfed_solve each:
    one realisation per (L, W) cell is solved and timed, and the time is
    scaled by the cell's size.  Compared with the batched FP32 solve."""
    import torch
    cells = {}
    for ch in wl.chains:
        cells.setdefault((ch.L, ch.W), []).append(ch)
    total, sample = 0.0, 0
    for (L, W), chs in sorted(cells.items()):
        ch = chs[0]
        m = pf.make_model(ch.L, ch.J1, ch.J2, ch.Delta, ch.h)
        o = pf.default_opts(block_size=0, precision=0, target_kind=0, target=wl.eps_target)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.solve(m, wl.nev, opts=o, vectors=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if r["status"] != pf.OK:
            print(f"warning: FP64 single solve of L={L} W={W} returned {r['status']}",
                  file=sys.stderr)
        total += dt * len(chs)
        sample += 1
    return {"time_s_estimate": total, "realisations": len(wl.chains), "sampled": sample,
            "sample": "one realisation per (L, W) cell, solved alone in FP64 (default block "
                      "size), time scaled by the cell's size",
            "batched_fp32_speedup": total / batch_s}


def _profiled_shape(workload):
    """Step shape recorded with the committed traffic counters, if they were
    taken on this kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", open(path).read(), flags=re.M))
    if kv.get("kernel_source_sha256_16") != _kernel_hash() or "step_shape" not in kv:
        return None
    return [int(v) for v in kv["step_shape"].split(",")]


def _cpu_baseline(wl, target_s=15.0, blocks=None):
    """The oracle's forward-recurrence filter (scipy CSR, FP64) on the
    workload's block shape (its first chain), timed on the host for
    ~target_s seconds."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import chain, chebyshev
    c = wl.chains[0]
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    s = wl.block if wl.block > 0 else (blocks[-1] if blocks else 16)
    X = np.random.default_rng(0).standard_normal((H.shape[0], s))
    E0, E1 = -2.0 * c.L, 2.0 * c.L  # any enclosing interval: cost is independent of it
    with threadpool_limits(1):
        t0 = time.perf_counter()
        chebyshev.filter_block(H, X, E0, E1, 0.0, 20)
        t20 = time.perf_counter() - t0
        K = max(20, int(20 * target_s / max(t20, 1e-6)))
        t0 = time.perf_counter()
        chebyshev.filter_block(H, X, E0, E1, 0.0, K)
        dt = time.perf_counter() - t0
    return {"value": K * s / dt, "unit": "H·V applications/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle forward-recurrence filter, K={K} steps on a {H.shape[0]}x{s} FP64 "
                      f"block of the same chain (scipy CSR SpMM, 1 thread), {dt:.1f} s"}


FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix


def _gram_roofline(ctx, pf, n, p, q, reps=20):
    """The Lanczos projection C = Q^T U (FP64 MFMA kernel k_gram + its
    reduction) at the solve's final shape: n x p basis against an n x q
    block.  HIP events on the stream the library runs on."""
    import torch
    Q = torch.randn((n, p), dtype=torch.float64, device="cuda")
    U = torch.randn((n, q), dtype=torch.float64, device="cuda")
    ctx.bind_stream()
    ctx.gram(Q, U)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.gram(Q, U)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    flops = 2.0 * n * p * q
    byts = 8.0 * n * (p + q)
    return {"kernel": "k_gram (FP64 MFMA 16x16x4, Q^T U) + reduction", "n": n, "p": p, "q": q,
            "us": 1e6 * s, "tflops": flops / s / 1e12,
            "mfma_frac": flops / s / 1e12 / FP64_MFMA_PEAK_TFLOPS,
            "gbs": byts / s / 1e9, "hbm_frac": byts / s / 1e9 / HBM_PEAK_GBS,
            "bound": "hbm" if flops / byts < FP64_MFMA_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS else "mfma"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3_fp64", "c3_fp32", "c4"])
    ap.add_argument("--shape", default="",
                    help="step shape threads,lpl,wg_per_cu,lds_tables,early_loads[,rank_incremental] (else the "
                         "profiled one, else tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the solve does not "
              "shard across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_09534_amd import polfed as pf
    from paper_2005_09534_amd import workloads

    wl = {"c1": workloads.c1, "c2": workloads.c2, "c3_fp64": lambda: workloads.c3("fp64"),
          "c3_fp32": lambda: workloads.c3("fp32"), "c4": workloads.c4}[args.workload]()
    c = wl.chains[0]
    prec = 1 if wl.precision == "fp32" else 0
    ctx = pf.Context(0)
    models = [pf.make_model(ch.L, ch.J1, ch.J2, ch.Delta, ch.h) for ch in wl.chains]
    model = models[0]
    opts = pf.default_opts(block_size=wl.block, K=wl.K, precision=prec, target_kind=0,
                           target=wl.eps_target)
    tune_s = 0.0
    from paper_2005_09534_amd import autotune
    t0 = time.perf_counter()
    if wl.block > 0:
        # the step-kernel shape of this (L, width, precision): the one the
        # committed rocprofv3 counters were taken on (when they match this
        # kernel source), else tuned; the FP32 comparison solve's shape is
        # tuned.  All outside the timed region.
        prof = _profiled_shape(args.workload)
        if args.shape:
            ctx.set_step_shape(c.L, wl.block, prec, *[int(v) for v in args.shape.split(",")])
        elif prof is not None:
            ctx.set_step_shape(c.L, wl.block, prec, *prof)
        else:
            autotune.tune_shape(ctx, c, wl.block, prec)
        if prec == 0 and not args.no_fp32:
            autotune.tune_shape(ctx, c, wl.block, 1)
    form_times = None
    if wl.block > 0 and len(models) == 1:
        # Clenshaw or the forward recurrence: one filter of the tuning order
        # timed both ways with the shape in force; the faster is kept
        form, secs = autotune.tune_form(ctx, c, wl.block, prec)
        form_times = {"chosen": "forward" if form == pf.FORM_FORWARD else "clenshaw",
                      "clenshaw_s": secs[pf.FORM_CLENSHAW], "forward_s": secs[pf.FORM_FORWARD]}
    tune_s = time.perf_counter() - t0
    if wl.block == 0:  # a workload without a fixed block size is autotuned
        t0 = time.perf_counter()
        by_L = {}
        for ch in wl.chains:
            by_L.setdefault(ch.L, []).append(ch)
        for L, chs in sorted(by_L.items()):
            # a sample of this length (batch throughput when batched); tunes
            # the step shape of every candidate width on the way
            autotune.tune_block(ctx, chs[:8] if len(models) > 1 else chs[0], wl.nev, prec)
        tune_s += time.perf_counter() - t0

    def step():
        if len(models) == 1:
            r = ctx.solve(model, wl.nev, opts=opts, vectors=True)
            return r, [r["info"]], [r["status"]]
        r = ctx.solve_batch(models, wl.nev, opts=opts, vectors=True)
        return r, r["info"], r["status"]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        r, inf, sts = step()
        infos.extend(inf)
        bad = [x for x in sts if x != pf.OK]
        if bad:
            print(f"warning: {len(bad)} solves with status != OK", file=sys.stderr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    apps = sum(i["hv_apps"] for i in infos)
    fbytes = sum(i["filter_bytes"] for i in infos)
    fgpu = sum(i["filter_gpu_s"] for i in infos)
    flaunch = sum(i["filter_launches"] for i in infos)
    achieved = fbytes / fgpu / 1e9 if fgpu > 0 else None
    last = infos[-1]
    line = {
        "metric": METRIC,
        "value": apps / wall,
        "unit": "H·V applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "realisations": len(models),
                   "L": sorted(set(ch.L for ch in wl.chains)),
                   "dim": [pf.dim(L) for L in sorted(set(ch.L for ch in wl.chains))],
                   "J2": c.J2, "Delta": c.Delta, "W": sorted(set(ch.W for ch in wl.chains)),
                   "nev": wl.nev, "block": sorted(set(i["block_size"] for i in infos)),
                   "K": last["K"] if len(models) == 1 else [min(i["K"] for i in infos), max(i["K"] for i in infos)],
                   "lanczos_blocks": last["m"] if len(models) == 1 else [min(i["m"] for i in infos), max(i["m"] for i in infos)],
                   "precision": wl.precision, "autotune_s": tune_s,
                   "filter_form": form_times,
                   "step_shape": (list(ctx.get_step_shape(c.L, wl.block, prec))
                                  if wl.block > 0 else None)},
        "time_to_nev_s": wall / args.steps,
        "solve": {k: last[k] for k in ("t_bounds", "t_filter", "t_orth", "t_eig", "t_rr",
                                       "t_refine", "t_total", "max_resid", "normH", "n_conv",
                                       "refine_passes")},
        "max_resid_rel": max(i["max_resid"] / i["normH"] for i in infos),
        # FP32 refinement passes per solve (-1: FP64 re-solve after a failed
        # refinement), as {passes: count}
        "refine_passes_hist": {str(k): v for k, v in sorted(
            __import__("collections").Counter(int(i["refine_passes"]) for i in infos).items())},
        "roofline": {
            "kernel": "k_step (fused Chebyshev step: matrix-free H~ gather + 3-term update)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": _traffic(args.workload, ctx.get_step_shape(c.L, wl.block, prec)
                                if wl.block > 0 else None),
            "avg_launch_us": 1e6 * fgpu / flaunch if flaunch else None,
            "algorithmic_bytes_per_launch": fbytes / flaunch if flaunch else None,
            "launches": flaunch,
        },
    }
    if not args.no_fp32 and prec == 0 and len(models) == 1:
        o32 = pf.default_opts(block_size=wl.block, K=wl.K, precision=1, target_kind=0,
                              target=wl.eps_target)
        ctx.solve(model, wl.nev, opts=o32, vectors=True)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r32 = ctx.solve(model, wl.nev, opts=o32, vectors=True)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t0
        i32 = r32["info"]
        import numpy as np
        # eigenvector error against the FP64 solve: sine of the angle between
        # corresponding vectors (the eigenvalues are simple here)
        ov = np.abs(np.sum(r32["V"] * r["V"], axis=0))
        sines = np.sqrt(np.clip(1.0 - ov * ov, 0.0, None))
        line["fp32_filter"] = {
            "time_to_nev_s": t32, "hv_apps_per_s": i32["hv_apps"] / t32,
            "max_resid_rel": i32["max_resid"] / i32["normH"], "refine_passes": i32["refine_passes"],
            "max_abs_eval_diff_vs_fp64": float(abs(r32["E"] - r["E"]).max()),
            "max_evec_sin_angle_vs_fp64": float(sines.max()),
            "speedup_vs_fp64": (wall / args.steps) / t32,
            "status": r32["status"]}
    line["gram"] = _gram_roofline(ctx, pf, pf.dim(c.L), int(last["m"]) * int(last["block_size"]),
                                  int(last["block_size"]))
    if len(models) > 1 and not args.no_fp32:
        line["fp64_single"] = _fp64_single_estimate(ctx, pf, wl, wall / args.steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = _cpu_baseline(wl, blocks=line["config"]["block"])
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
