"""Benchmark of the MAPI hot path on one MI355X.

Workload (headline): dense symmetric covariance n = 16384, C = X X^T / 32768 with
X i.i.d. N(0, 1) rows centred (synthetic, seeded), stored in float32.  One step
is one MAPI solve of ITERS iterations (fixed count: products, float64 l1
normalisation and residual every iteration).  `value` is the product throughput
in Gelem/s (n^2 min-terms per iteration).  The same line carries RPI and the
BF16 / FP8 storage modes under "detail", the roofline of the dense product
kernel, and the FP64 CPU oracle timed on a bounded sample of the same work.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2110_12065_amd", "csrc", "k_dense.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(dtype):
    """HBM bytes per launch of the dense product from committed rocprofv3 counter runs, or None."""
    p = os.path.join(ROOT, "profiles", "mavp_dense_n16384_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None                     # kernel changed since the counters were taken
    return t.get("bytes_per_launch", {}).get(dtype)


def time_solves(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="comma list of detail modes to run (default all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2110_12065_amd as mp

    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    log("generating the n=16384 covariance on the GPU")
    C = synth.dense_cov(N, N_SAMPLES, seed=SEED, device="cuda")
    w0 = torch.from_numpy(synth.start_vector(N, SEED + 1)).cuda()
    ctx = mp.default_context()
    elems = float(N) * N * ITERS

    def mapi_step(A, rs=None):
        return lambda: mp.mapi_solve(A, w0, max_iters=ITERS, row_scale=rs, check_every=ITERS, ctx=ctx)

    def rpi_step(A, rs=None):
        return lambda: mp.rpi_solve(A, w0, max_iters=ITERS, row_scale=rs, check_every=ITERS, ctx=ctx)

    def kernel_avg_ms(step):
        ctx.timing(True)
        ctx.timing_reset()
        for _ in range(max(2, args.steps // 2)):
            step()
        ms, n = ctx.timing_get("mavp")
        ctx.timing(False)
        return ms / max(n, 1), n

    # ---------------------------------------------------------------- headline: FP32 MAPI
    head = mapi_step(C)
    for _ in range(args.warmup):
        head()
    log("timing fp32 MAPI")
    sec = time_solves(head, args.steps, sync)
    value = elems / sec / 1e9
    avg_ms, launches = kernel_avg_ms(head)
    bytes_launch = 4.0 * N * N + 8.0 * N          # A once, w once (per block from L2), y once
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic("f32")

    detail = {"mapi_f32": {"gelem_s": value, "ms_per_solve": sec * 1e3, "product_kernel_ms": avg_ms,
                           "product_kernel_gbs": achieved}}
    only = set(filter(None, args.only.split(",")))

    def want(k):
        return not only or k in only

    if want("rpi_f32"):
        f = rpi_step(C)
        f()
        s = time_solves(f, args.steps, sync)
        k_ms, _ = kernel_avg_ms(f)
        detail["rpi_f32"] = {"gelem_s": elems / s / 1e9, "ms_per_solve": s * 1e3, "product_kernel_ms": k_ms,
                             "product_kernel_gbs": bytes_launch / (k_ms * 1e-3) / 1e9}
    for dt, bpe in (("bf16", 2), ("fp8", 1)):
        if not (want(f"mapi_{dt}") or want(f"rpi_{dt}")):
            continue
        q, s8 = mp.mapi_quantize(C, dt, ctx=ctx)
        for meth, mk in (("mapi", mapi_step), ("rpi", rpi_step)):
            key = f"{meth}_{dt}"
            if not want(key):
                continue
            f = mk(q, s8)
            f()
            s = time_solves(f, args.steps, sync)
            k_ms, _ = kernel_avg_ms(f)
            b = bpe * float(N) * N + 8.0 * N + (4.0 * N if dt == "fp8" else 0.0)
            detail[key] = {"gelem_s": elems / s / 1e9, "ms_per_solve": s * 1e3, "product_kernel_ms": k_ms,
                           "product_kernel_gbs": b / (k_ms * 1e-3) / 1e9, "hbm_frac": b / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del q, s8

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the FP64 CPU oracle on a bounded sample")
        Ch = C.cpu().numpy().astype(np.float64)
        w = w0.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        its = 0
        while True:
            y = oracle.mavp(Ch, w)
            w = y / np.abs(y).sum()
            its += 1
            if time.perf_counter() - t0 > 10.0 or its >= 8:
                break
        dt = time.perf_counter() - t0
        cpu = {"value": its * float(N) * N / dt / 1e9, "unit": "Gelem/s", "cores": 1, "kind": "oracle",
               "sample": f"{its} full MAPI iterations (min1 product + l1 normalisation) of the n=16384 FP64 "
                         f"oracle, numpy single-threaded, {dt:.1f} s"}
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
                     "kernel": "k_mavp_dense<f32,min1>", "launches_timed": launches},
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
