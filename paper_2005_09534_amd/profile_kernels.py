"""Profiling driver for the Chebyshev step kernel (run under rocprofv3).

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- \
        python -m paper_2005_09534_amd.profile_kernels run --workload c5 --shape SHAPE
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT -o write -- \
        python -m paper_2005_09534_amd.profile_kernels run --workload c5 --shape SHAPE
    python -m paper_2005_09534_amd.profile_kernels summarize --workload c5 --shape SHAPE \
        --fetch OUT/.../fetch_counter_collection.csv --write OUT/.../write_counter_collection.csv \
        > profiles/k_step_c5_traffic.txt

SHAPE is the step shape bench.py ran with (its config.step_shape, comma
separated), so that the counters describe the launches the bench times.

``run`` applies the workload's filter (its chain, block width and precision)
for a fixed number of steps, then copies a buffer of known size with the
library's plain copy kernel (k_stream_copy, 16-byte loads and stores), whose
counter readings calibrate the byte counts.  Workload c5 is the L = 26 chain
with the FP64 filter (the bench's default line), c5_fp32 the same with FP32.  ``summarize`` turns the two counter CSVs into HBM bytes per step
launch and records the hash of the kernel source the counters were taken on.
"""

import argparse
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
# order of the untimed filter that loads the kernels' code before the timed one
WARMUP_K = 2


STEP_SOURCES = ("hv_kernels.h", "hv.hip", "hv_f32.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2005_09534_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _workload(name):
    """(workload, precision name) of a profile name."""
    from paper_2005_09534_amd import workloads
    wl = {"c1": workloads.c1, "c2": workloads.c2, "c3_fp64": lambda: workloads.c3("fp64"),
          "c3_fp32": lambda: workloads.c3("fp32"), "c5": workloads.c5,
          "c5_fp32": workloads.c5}[name]()
    prec = "fp64" if name == "c5" else wl.precision
    return wl, prec


def run(args):
    import torch
    from paper_2005_09534_amd import polfed as pf
    wl, precision = _workload(args.workload)
    c = wl.chains[0]
    ctx = pf.Context(0)
    m = pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h)
    n = pf.dim(c.L)
    s = wl.block if wl.block > 0 else 16
    dt = torch.float32 if precision == "fp32" else torch.float64
    # the operator of the solve: Lanczos bounds widened as the solver does,
    # target at the workload's rescaled energy
    E0, E1, r0, r1 = ctx.bounds(m, 200)
    w = E1 - E0
    E0w, E1w = E0 - r0 - 1e-3 * w, E1 + r1 + 1e-3 * w
    sigma_H = E0 + wl.eps_target * w
    sigma = (2.0 * sigma_H - (E0w + E1w)) / (E1w - E0w)
    X = torch.randn((n, s), device="cuda", dtype=torch.float64).to(dt)
    Y = torch.empty_like(X)
    if args.shape:
        ctx.set_step_shape(c.L, s, 1 if precision == "fp32" else 0,
                           *[int(v) for v in args.shape.split(",")])
    ctx.set_graphs(False)  # one dispatch per step, each counted
    # a short filter first, so that loading the kernels' code is not timed
    ctx.apply_filter(m, E0w, E1w, sigma, WARMUP_K, X, out=Y)
    torch.cuda.synchronize()
    ctx.filter_stats(reset=True)
    ctx.apply_filter(m, E0w, E1w, sigma, args.K, X, out=Y)
    torch.cuda.synchronize()
    st = ctx.filter_stats(reset=True)
    # calibration: the library's plain copy of COPY_BYTES bytes (a warm-up
    # copy and one timed copy, both counted)
    del X, Y
    torch.cuda.empty_cache()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ctx.stream_copy(a, b, reps=1)
    torch.cuda.synchronize()
    print(f"filter: {st['launches']:.0f} launches, {st['bytes'] / st['launches']:.0f} algorithmic "
          f"bytes/launch, {1e6 * st['gpu_s'] / st['launches']:.2f} us/launch (HIP events)")
    ctx.close()


def _read(path, counter, step_name):
    """(per-dispatch values of `counter` for the step kernel instantiation
    `step_name` in the timed filter, largest value for the library's copy
    kernel) from a rocprofv3 counter_collection CSV.  The WARMUP_K + 1
    dispatches of the warm-up filter come first and are left out."""
    step, copy = [], []
    with open(path) as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name") or ""
            if row.get("Counter_Name", counter) != counter:
                continue
            v = float(row.get("Counter_Value") or 0.0)
            if step_name in name:
                step.append((int(row.get("Dispatch_Id") or len(step)), v))
            elif "k_stream_copy" in name:
                copy.append(v)
    step = [v for _, v in sorted(step)[WARMUP_K + 1:]]
    return step, (max(copy) if copy else 0.0)


def summarize(args):
    wl, precision = _workload(args.workload)
    T = "float" if precision == "fp32" else "double"
    s = wl.block if wl.block > 0 else 16
    shape = [int(v) for v in args.shape.split(",")]
    slices = shape[6] if len(shape) > 6 and s % shape[6] == 0 else 1
    step_name = f"k_step<{T}, {s // slices},"  # the kernel's width is one slice
    fs, fc = _read(args.fetch, "FETCH_SIZE", step_name)
    ws, wc = _read(args.write, "WRITE_SIZE", step_name)
    if not fs or not ws or not fc or not wc:
        sys.exit("missing step or copy dispatches in the counter files")
    # the copy kernel reads and writes COPY_BYTES: scale KiB readings to bytes
    kf = COPY_BYTES / (fc * 1024.0)
    kw = COPY_BYTES / (wc * 1024.0)
    fetch = sum(fs) / len(fs) * 1024.0 * kf
    write = sum(ws) / len(ws) * 1024.0 * kw
    print(f"# HBM traffic of the Chebyshev step kernel ({step_name}...>), workload {args.workload}")
    print("# counters: rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (KiB per dispatch),")
    print("# each scaled by its reading for a device-to-device copy of COPY_BYTES bytes")
    print(f"# calibration: a {COPY_BYTES} B copy read {fc:.0f} KiB and wrote {wc:.0f} KiB")
    print(f"workload = {args.workload}")
    print(f"dispatches = {len(fs)}")
    print(f"fetch_kib_per_launch_raw = {sum(fs) / len(fs):.1f}")
    print(f"write_kib_per_launch_raw = {sum(ws) / len(ws):.1f}")
    print(f"fetch_scale = {kf:.4f}")
    print(f"write_scale = {kw:.4f}")
    print(f"hbm_fetch_bytes_per_launch = {fetch:.0f}")
    print(f"hbm_write_bytes_per_launch = {write:.0f}")
    print(f"hbm_bytes_per_launch = {fetch + write:.0f}")
    print(f"step_shape = {args.shape}")
    print(f"kernel_source_sha256_16 = {kernel_source_hash()}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="c2")
    r.add_argument("--K", type=int, default=64)
    r.add_argument("--shape", default="",
                   help="threads,lpl,wg_per_cu,lds_tables,early_loads,rank_incremental,xcd_slices")
    s = sub.add_parser("summarize")
    s.add_argument("--workload", default="c2")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--shape", required=True, help="the shape given to run")
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    run(a) if a.cmd == "run" else summarize(a)


if __name__ == "__main__":
    main()
