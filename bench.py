"""Benchmark of the MAPI hot path on one MI355X.

Workload (headline): dense symmetric covariance n = 16384, C = X X^T / 32768 with
X i.i.d. N(0, 1) rows centred (synthetic, seeded), stored in float32.  One step
is one MAPI solve of ITERS iterations (fixed count: products, float64 l1
normalisation and residual every iteration).  `value` is the product throughput
in Gelem/s (n^2 min-terms per iteration).  The same line carries RPI and the
BF16 / FP8 storage modes under "detail", the roofline of the dense product
kernel, and the FP64 CPU oracle timed on a bounded sample of the same work.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --mode kernels           # short run for rocprofv3 (copy reference + products)
    python bench.py --summarize STATS_DIR FETCH_DIR WRITE_DIR   # write profiles/ from rocprofv3 CSVs
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 16384
N_SAMPLES = 32768
ITERS = 20
HBM_PEAK_GBS = 8000.0
SEED = 2024
BYTES_PER_ELEM = {"f32": 4, "bf16": 2, "fp8": 1}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mavp_dense_n16384_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("dense_kernel.h", "k_dense_f32.hip", "k_dense_bf16.hip", "k_dense_fp8.hip"):
        with open(os.path.join(ROOT, "paper_2110_12065_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def product_bytes(dtype, n=N):
    """Algorithmic HBM bytes of one dense product launch: the matrix once, w and y once
    (plus the row scales for FP8)."""
    return BYTES_PER_ELEM[dtype] * float(n) * n + 8.0 * n + (4.0 * n if dtype == "fp8" else 0.0)


def load_traffic(dtype):
    """HBM bytes per launch of the dense product from committed rocprofv3 counter runs, or None
    (also None once the kernel sources changed after the counters were taken)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(dtype)


def time_solves(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def setup(autotune=True):
    import torch
    import synth
    import paper_2110_12065_amd as mp
    torch.cuda.set_device(0)
    log("generating the n=16384 covariance on the GPU")
    C = synth.dense_cov(N, N_SAMPLES, seed=SEED, device="cuda")
    w0 = torch.from_numpy(synth.start_vector(N, SEED + 1)).cuda()
    ctx = mp.default_context()
    mats = {"f32": (C, None)}
    for dt in ("bf16", "fp8"):
        mats[dt] = mp.mapi_quantize(C, dt, ctx=ctx)
    for dt, (A, rs) in mats.items():
        if autotune:
            shape, ms = mp.mapi_autotune_dense(A, "min1", reps=3, row_scale=rs, ctx=ctx)
            log(f"autotuned {dt}: {shape} {ms * 1e3:.1f} us")
        else:
            log(f"launch shape {dt}: {mp.mapi_tuning_get(mp._dtype_code(A), N, N, ctx=ctx)}")
    return torch, mp, ctx, C, w0, mats


def run_kernels_mode():
    """Short workload for rocprofv3: the copy reference (1 GiB -> 1 GiB) and every product
    kernel, five launches each, in the tuned launch shapes."""
    torch, mp, ctx, C, w0, mats = setup(autotune=not os.environ.get("MAPI_TUNE_CACHE"))
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    mp.mapi_copy_reference(src, dst, reps=5, ctx=ctx)
    for dt, (A, rs) in mats.items():
        for _ in range(5):
            mp.mapi_mavp(A, w0, "min1", row_scale=rs, ctx=ctx)
    torch.cuda.synchronize()
    log("kernels mode done")


# ------------------------------------------------------------------ profile summaries
def _read_csvs(d, pattern):
    rows = []
    for p in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _kernel_dtype(name):
    if "k_copy16" in name:
        return "copy"
    if "k_mavp_dense" not in name:
        return None
    # template argument order: storage type, product, ... (0 = f32, 1 = bf16, 2 = fp8)
    inside = name[name.index("<") + 1:]
    first = inside.split(",")[0].strip()
    return {"0": "f32", "1": "bf16", "2": "fp8"}.get(first)


def summarize(stats_dir, fetch_dir, write_dir, cmd_stats, cmd_fetch, cmd_write):
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    stats = _read_csvs(stats_dir, "*kernel_stats.csv")
    lines = ["# Kernel time summary: dense products at n = 16384 and the copy reference", "",
             f"Command: `{cmd_stats}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0) or 0)):
        nm = r.get("Name", r.get("KernelName", "?"))
        lines.append(f"| `{nm[:110]}` | {r.get('Calls')} | {float(r.get('AverageNs', 0)) / 1e3:.1f} | "
                     f"{float(r.get('MinNs', 0)) / 1e3:.1f} | {float(r.get('MaxNs', 0)) / 1e3:.1f} |")
    with open(os.path.join(ROOT, "profiles", "mavp_dense_n16384_kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_kernel(d, counter):
        acc = {}
        for r in _read_csvs(d, "*counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            dt = _kernel_dtype(r.get("Kernel_Name", ""))
            if dt is None:
                continue
            acc.setdefault(dt, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = float(1 << 30)
    # the copy of known size reads and writes exactly copy_bytes: scale the counters by it
    f_scale = copy_bytes / (fetch["copy"] * 1024.0) if fetch.get("copy") else None
    w_scale = copy_bytes / (write["copy"] * 1024.0) if write.get("copy") else None
    out = {"kernel_source_sha256_16": kernel_source_hash(), "commands": [cmd_fetch, cmd_write],
           "copy_reference_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_kib_per_launch": fetch, "write_kib_per_launch": write, "bytes_per_launch": {},
           "algorithmic_bytes_per_launch": {}}
    md = ["# HBM traffic of the dense product kernels (n = 16384)", "",
          f"FETCH_SIZE: `{cmd_fetch}`", "", f"WRITE_SIZE: `{cmd_write}`", "",
          "Counters are KiB per dispatch, scaled by the factor that maps the plain 1 GiB copy "
          f"reference onto its known size (fetch x{f_scale}, write x{w_scale}).", "",
          "| storage | FETCH KiB | WRITE KiB | scaled HBM bytes | algorithmic bytes | ratio |", "|---|---|---|---|---|---|"]
    for dt in ("f32", "bf16", "fp8"):
        if dt not in fetch or dt not in write or f_scale is None or w_scale is None:
            continue
        b = fetch[dt] * 1024.0 * f_scale + write[dt] * 1024.0 * w_scale
        out["bytes_per_launch"][dt] = b
        out["algorithmic_bytes_per_launch"][dt] = product_bytes(dt)
        md.append(f"| {dt} | {fetch[dt]:.0f} | {write[dt]:.0f} | {b:.4e} | {product_bytes(dt):.4e} | "
                  f"{b / product_bytes(dt):.3f} |")
    if "copy" in fetch:
        md.append(f"| copy reference | {fetch['copy']:.0f} | {write.get('copy', 0):.0f} | "
                  f"{2 * copy_bytes:.4e} | {2 * copy_bytes:.4e} | 1.000 |")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    with open(os.path.join(ROOT, "profiles", "mavp_dense_n16384_traffic.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps(out, indent=1))


# ------------------------------------------------------------------ benchmark
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="bench", choices=["bench", "kernels"])
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--commands", nargs=3, default=["", "", ""], help="commands that produced the three dirs")
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize, *args.commands)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    if args.mode == "kernels":
        run_kernels_mode()
        return

    import numpy as np
    torch, mp, ctx, C, w0, mats = setup()
    sync = torch.cuda.synchronize
    elems = float(N) * N * ITERS

    def step(meth, dt):
        A, rs = mats[dt]
        fn = mp.mapi_solve if meth == "mapi" else mp.rpi_solve
        return lambda: fn(A, w0, max_iters=ITERS, row_scale=rs, check_every=ITERS, ctx=ctx)

    def kernel_avg_ms(fn):
        ctx.timing(True)
        ctx.timing_reset()
        for _ in range(max(2, args.steps // 2)):
            fn()
        ms, n = ctx.timing_get("mavp")
        ctx.timing(False)
        return ms / max(n, 1), n

    detail = {}
    head = None
    for meth in ("mapi", "rpi"):
        for dt in ("f32", "bf16", "fp8"):
            fn = step(meth, dt)
            for _ in range(args.warmup if (meth, dt) == ("mapi", "f32") else 1):
                fn()
            log(f"timing {meth} {dt}")
            sec = time_solves(fn, args.steps, sync)
            k_ms, launches = kernel_avg_ms(fn)
            gbs = product_bytes(dt) / (k_ms * 1e-3) / 1e9
            detail[f"{meth}_{dt}"] = {"gelem_s": elems / sec / 1e9, "ms_per_solve": sec * 1e3,
                                      "product_kernel_us": k_ms * 1e3, "product_kernel_gbs": gbs,
                                      "hbm_frac": gbs / HBM_PEAK_GBS}
            if (meth, dt) == ("mapi", "f32"):
                head = (sec, k_ms, launches, gbs)

    sec, k_ms, launches, achieved = head
    value = elems / sec / 1e9
    traffic = load_traffic("f32")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the FP64 CPU oracle on a bounded sample")
        Ch = C.cpu().numpy().astype(np.float64)
        w = w0.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        its = 0
        while time.perf_counter() - t0 < 12.0 and its < 40:
            y = oracle.mavp(Ch, w)
            w = y / np.abs(y).sum()
            its += 1
        dt_s = time.perf_counter() - t0
        cpu = {"value": its * float(N) * N / dt_s / 1e9, "unit": "Gelem/s", "cores": 1, "kind": "oracle",
               "sample": f"{its} full MAPI iterations (min1 product + l1 normalisation) of the n=16384 FP64 "
                         f"oracle, numpy, one thread, {dt_s:.1f} s"}
        del Ch

    out = {
        "metric": "MAVP Gelem/s (MAPI, dense n=16384 float32, fixed 20-iteration solves)",
        "value": value,
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense symmetric covariance n=16384 (X 16384x32768 N(0,1), rows centred), "
                               "float32 storage, MAPI min1, 20 iterations per step",
                   "n": N, "iterations_per_step": ITERS},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_mavp_dense<f32,min1>", "launches_timed": launches,
                     "algorithmic_bytes_per_launch": product_bytes("f32"), "avg_launch_us": k_ms * 1e3},
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
