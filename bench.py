"""Benchmark of the MAPI hot path on one MI355X.

Workload (headline): dense symmetric covariance n = 16384, C = X X^T / 32768 with
X i.i.d. N(0, 1) rows centred (synthetic, seeded), stored in float32.  One step
is one MAPI solve of ITERS iterations (tolerance 0, so all ITERS run): every
iteration forms the min1 product, its float64 l1 normaliser, the float32 iterate
and the float64 residual ||w_t - w_{t-1}||_1, and advances the stop rule.  The
iterate and residual of iteration t are formed inside product t + 1 and the
stop rule for t is advanced by product t + 2 (or by the last normalisation
kernel), one launch per iteration.  `value` is the product throughput in Gelem/s
(n^2 min-terms per iteration).  The same line carries RPI and the
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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 16384
N_SAMPLES = 32768
ITERS = 20
HBM_PEAK_GBS = 8000.0
SEED = 2024
# Solves stop at tol 1e-6 or, once the float32 iterate stops improving, after this
# many iterations without a new smallest residual (the float32 floor of an
# l2-normalised iterate is about sqrt(n) * 6e-8, above 1e-6 for large n).
STALL = 10
BYTES_PER_ELEM = {"f32": 4, "bf16": 2, "fp8": 1}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mavp_dense_n16384_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ops.h", "common.h", "dense_kernel.h", "k_dense_f32.hip", "k_dense_bf16.hip", "k_dense_fp8.hip"):
        with open(os.path.join(ROOT, "paper_2110_12065_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def csr_source_hash():
    h = hashlib.sha256()
    for f in ("ops.h", "k_csr.hip", "k_csr_split.hip"):
        with open(os.path.join(ROOT, "paper_2110_12065_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PR_N, PR_SEED = 1 << 22, 2022


def csr_bytes(n, nnz):
    """Algorithmic bytes of one PageRank product: links (col, val) and row pointers once, w and y once."""
    return 8.0 * nnz + 4.0 * (n + 1) + 8.0 * n


def load_csr_traffic():
    """HBM bytes per launch of the MAPI PageRank product on the 2^22-node graph from committed
    counter runs, or None (also None once the product's sources changed)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f).get("csr") or {}
    if t.get("source_sha256_16") != csr_source_hash():
        return None
    return t.get("bytes_per_launch")


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
            shape, ms = mp.mapi_autotune_dense(A, "min1", reps=10, row_scale=rs, ctx=ctx)
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
    mp.mapi_read_reference(C, reps=5, ctx=ctx)
    for dt, (A, rs) in mats.items():
        for _ in range(5):
            mp.mapi_mavp(A, w0, "min1", row_scale=rs, ctx=ctx)
    del src, dst
    # three MAPI PageRank products on the 2^22-node graph: the column-split product (the layout
    # of this size, here built before the first product), then the plain CSR product
    g = _graph(PR_N, PR_SEED)
    rp, col, val = (torch.from_numpy(g[x]).cuda() for x in ("row_ptr", "col", "val"))
    mp.mapi_pagerank_split_after(0, ctx=ctx)
    mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=3, check_every=3, ctx=ctx)
    plain = mp.Context()
    mp.mapi_pagerank_split_config(0, ctx=plain)
    mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=3, check_every=3, ctx=plain)
    del rp, col, val
    # one min-covariance build (min1) of the PCA workload, 4096 x 65536
    import synth
    X, clean = synth.pca_data_device(4096, 65536, 77, "cuda")
    del clean
    mp.mapi_mingram(X, 1.0 / 65536, "min1", ctx=ctx)
    torch.cuda.synchronize()
    log("kernels mode done")


# ------------------------------------------------------------------ profile summaries
def _bench_line(path):
    """The last JSON line of a benchmark log (a profiler may print after it)."""
    with open(path) as f:
        lines = [x for x in f.read().splitlines() if x.startswith("{")]
    return json.loads(lines[-1]) if lines else {}


READ_REPS = 10          # timed launches per launch shape of the read reference


def _read_csvs(d, pattern):
    rows = []
    for p in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _kernel_dtype(name):
    if "k_copy16" in name:
        return "copy"
    if "k_read16" in name:
        return "read"
    if "k_csr_product<0," in name:
        return "csr_plain"
    if "k_csr_split_product<0," in name:
        return "csr_split"
    if "k_csr_split_combine<0," in name:
        return "csr_combine"
    if "k_split_hub_values<float>" in name:
        return "csr_hubval"
    if "k_mavp_dense" not in name:
        return None
    # template argument order: storage type, product, ... (0 = f32, 1 = bf16, 2 = fp8)
    inside = name[name.index("<") + 1:]
    first = inside.split(",")[0].strip()
    return {"0": "f32", "1": "bf16", "2": "fp8"}.get(first)


SECTION_KERNELS = ("k_gram_min", "k_gram_reduce", "k_gram_mfma", "k_solve_small", "k_mb_batches", "k_mb_iterate",
                   "k_deflate", "k_mgs_append", "k_mavp_dense", "k_finalize")
SECTIONS_PROFILE = "pca4096x65536_n256_minibatch_kernel_stats.md"


def summarize_sections(stats_dir, cmd, bench_json=None):
    """profiles/ summary of the kernels of the PCA (4096 x 65536), n = 256 and mini-batch sections
    from a rocprofv3 --kernel-trace --stats run, beside the benchmark's own host timings."""
    stats = _read_csvs(stats_dir, "*kernel_stats.csv")
    det = {}
    if bench_json and os.path.exists(bench_json):
        det = _bench_line(bench_json).get("detail", {})
    lines = ["# Kernel time summary: PCA 4096 x 65536 (min-covariance and covariance builds, top-8 "
             "solves), the n = 256 solve, mini-batch MAPI (Alg. 3)", "", f"Command: `{cmd}`", "",
             "Kernels of these sections by total time (the product and normalisation rows include the "
             "headline benchmark's launches, which every run makes first):", "",
             "| kernel | calls | average (us) | min (us) | max (us) |", "|---|---|---|---|---|"]
    keep = [r for r in stats if any(k in r.get("Name", r.get("KernelName", "")) for k in SECTION_KERNELS)]
    by = {}
    for r in sorted(keep, key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))[:24]:
        nm = r.get("Name", r.get("KernelName", "?"))
        lines.append(f"| `{nm[:110]}` | {r.get('Calls')} | {float(r.get('AverageNs', 0)) / 1e3:.1f} | "
                     f"{float(r.get('MinNs', 0)) / 1e3:.1f} | {float(r.get('MaxNs', 0)) / 1e3:.1f} |")
    for r in keep:
        nm = r.get("Name", r.get("KernelName", ""))
        for k in SECTION_KERNELS:
            if k in nm:
                tot, calls = by.get(k, (0.0, 0))
                by[k] = (tot + float(r.get("TotalDurationNs", 0) or 0), calls + int(r.get("Calls", 0) or 0))
    pca, small = det.get("pca", {}), det.get("small", {})
    lines += ["", "Against the benchmark's host timings (same run):", "",
              "| quantity | rocprofv3 | benchmark |", "|---|---|---|"]
    if "k_gram_min" in by:
        t, c = by["k_gram_min"]
        tr, cr = by.get("k_gram_reduce", (0.0, 0))
        lines.append(f"| min1 build at 4096 x 65536: `k_gram_min` (+ `k_gram_reduce`) per build | "
                     f"{t / max(c, 1) / 1e6:.2f} ms (+ {tr / max(cr, 1) / 1e6:.2f} ms, shared with the other builds) | "
                     f"{pca.get('gram_min1_ms', float('nan')):.2f} ms per `mapi_mingram` call |")
    if "k_gram_mfma" in by:
        t, c = by["k_gram_mfma"]
        lines.append(f"| covariance build on the matrix cores, per launch | {t / max(c, 1) / 1e6:.2f} ms | "
                     f"{pca.get('gram_dot_ms', float('nan')):.2f} ms per call |")
    # the one-block solve per product: template argument 0 = min1 (MAPI), 3 = ordinary product (RPI)
    for meth, tag in (("mapi", "k_solve_small<0>"), ("rpi", "k_solve_small<3>")):
        rows = [r for r in keep if tag in r.get("Name", r.get("KernelName", ""))]
        if not rows:
            continue
        t = sum(float(r.get("TotalDurationNs", 0) or 0) for r in rows)
        c = sum(int(r.get("Calls", 0) or 0) for r in rows)
        it = small.get(f"{meth}_iters") or 200
        lines.append(f"| n = 256 one-block solve ({meth.upper()}, {it} iterations), per launch | "
                     f"{t / max(c, 1) / 1e3:.1f} us ({t / max(c, 1) / 1e3 / it:.2f} us per iteration) | "
                     f"{small.get(f'{meth}_plain_us_per_iter', float('nan')):.2f} us per iteration (host clock, "
                     f"launch and state read-back included) |")
    for k in ("k_mb_batches", "k_mb_iterate"):
        if k in by:
            t, c = by[k]
            lines.append(f"| `{k}` per launch | {t / max(c, 1) / 1e3:.1f} us | |")
    out = os.path.join(ROOT, "profiles", SECTIONS_PROFILE)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    log(f"wrote {out}")


def summarize(stats_dir, fetch_dir, write_dir, cmd_stats, cmd_fetch, cmd_write, bench_json=None):
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    stats = _read_csvs(stats_dir, "*kernel_stats.csv")
    lines = ["# Kernel time summary: the benchmark at n = 16384 (dense products, normalisation)", "",
             f"Command: `{cmd_stats}`", "",
             "Top kernels by total time (the first row is the covariance build by rocBLAS in the set-up; "
             "the product rows include the autotuner's trial launches of the same shape).", "",
             "| kernel | calls | average (us) | min (us) | max (us) |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))[:24]:
        nm = r.get("Name", r.get("KernelName", "?"))
        lines.append(f"| `{nm[:110]}` | {r.get('Calls')} | {float(r.get('AverageNs', 0)) / 1e3:.1f} | "
                     f"{float(r.get('MinNs', 0)) / 1e3:.1f} | {float(r.get('MaxNs', 0)) / 1e3:.1f} |")
    # the timed launches: the last 100 dispatches of each storage type's min1 product (the
    # benchmark's live event timing covers exactly those)
    trace = _read_csvs(stats_dir, "*kernel_trace.csv")
    live = {}
    if bench_json and os.path.exists(bench_json):
        det = _bench_line(bench_json).get("detail", {})
        live = {dt: det.get(f"mapi_{dt}", {}).get("product_kernel_us") for dt in ("f32", "bf16", "fp8")}
        live.update({f"read_{dt}": v.get("us") for dt, v in det.get("read_reference", {}).items()})
    if trace:
        lines += ["", "Timed launches (the last 100 dispatches of the MAPI min1 product per storage type before "
                  "the read reference, which follows the solves; later sections launch the same kernels on "
                  "other shapes) against the benchmark's own HIP-event timing of the same launches:", "",
                  "| storage | kernel | rocprofv3 average (us) | benchmark events (us) |", "|---|---|---|---|"]
        reads = [int(r["Start_Timestamp"]) for r in trace if "k_read16" in r["Kernel_Name"]]
        t_read = min(reads) if reads else float("inf")
        for dt, code in (("f32", "0"), ("bf16", "1"), ("fp8", "2")):
            ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), r["Kernel_Name"])
                        for r in trace if r["Kernel_Name"].startswith(f"void mapi::k_mavp_dense<{code}, 0,")
                        and int(r["Start_Timestamp"]) < t_read)
            if not ds:
                continue
            last = ds[-100:]
            avg = sum(x[1] for x in last) / len(last) / 1e3
            ev = live.get(dt)
            lines.append(f"| {dt} | `{last[-1][2][:48]}` | {avg:.1f} | {ev:.1f} |" if ev else
                         f"| {dt} | `{last[-1][2][:48]}` | {avg:.1f} | - |")
        # the read reference per matrix (f32, bf16, fp8): 12 launch shapes, each one untimed
        # and READ_REPS timed launches; the reference is the fastest shape's average
        rd = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                    for r in trace if "k_read16" in r["Kernel_Name"])
        per = 12 * (1 + READ_REPS)
        if len(rd) >= 3 * per:
            lines += ["", "Read reference (plain streaming read of the same matrix, `k_read16`; the fastest of 12 "
                      "launch shapes), timed launches:", "",
                      "| matrix | rocprofv3 average (us) | benchmark events (us) |", "|---|---|---|"]
            for k, dt in enumerate(("f32", "bf16", "fp8")):
                grps = [rd[k * per + g * (1 + READ_REPS) + 1:k * per + (g + 1) * (1 + READ_REPS)] for g in range(12)]
                avg = min(sum(x[1] for x in grp) / len(grp) for grp in grps) / 1e3
                ev = live.get(f"read_{dt}")
                lines.append(f"| {dt} | {avg:.1f} | {ev:.1f} |" if ev else f"| {dt} | {avg:.1f} | - |")
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
    parts = ("csr_split", "csr_combine")
    if all(k in fetch and k in write for k in parts) and f_scale is not None and w_scale is not None:
        nnz = int(_graph(PR_N, PR_SEED)["col"].size)
        alg = csr_bytes(PR_N, nnz)
        per = {k: fetch[k] * 1024.0 * f_scale + write[k] * 1024.0 * w_scale
               for k in ("csr_hubval",) + parts + ("csr_plain",) if k in fetch and k in write}
        b = per["csr_split"] + per["csr_combine"] + per.get("csr_hubval", 0.0)
        out["csr"] = {"source_sha256_16": csr_source_hash(), "n": PR_N, "nnz": nnz,
                      "fetch_kib": {k: fetch[k] for k in per}, "write_kib": {k: write[k] for k in per},
                      "bytes_per_launch": b, "bytes_per_kernel": per, "algorithmic_bytes_per_launch": alg}
        md += ["", f"PageRank MAPI product at n = 2^22 ({nnz} links; algorithmic bytes = 8 per link + 4 per row "
                   "pointer + 8 per node for w and y). One product is the gather of the hub values, the "
                   "column-split kernel and its combine kernel (the default at this size); the plain CSR product "
                   "is measured beside it:", "",
               "| kernel | FETCH KiB | WRITE KiB | scaled HBM-side bytes | algorithmic bytes | ratio |",
               "|---|---|---|---|---|---|"]
        names = {"csr_hubval": "`k_split_hub_values`", "csr_split": "`k_csr_split_product`",
                 "csr_combine": "`k_csr_split_combine`", "csr_plain": "`k_csr_product` (plain)"}
        for k, v in per.items():
            md.append(f"| {names[k]} | {fetch[k]:.0f} | {write[k]:.0f} | {v:.4e} | "
                      f"{alg if k in ('csr_split', 'csr_plain') else 0:.4e} | {v / alg:.3f} |")
        md.append(f"| split product (hub values, product, combine) | | | {b:.4e} | {alg:.4e} | {b / alg:.3f} |")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    with open(os.path.join(ROOT, "profiles", "mavp_dense_n16384_traffic.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps(out, indent=1))


LIMITER_KERNELS = (("k_mavp_dense<0, 0,", "f32 product (min1)"), ("k_mavp_dense<1, 0,", "bf16 product (min1)"),
                   ("k_mavp_dense<2, 0,", "fp8 product (min1)"), ("k_read16", "read reference"),
                   ("k_copy16", "copy reference"), ("k_csr_split_product<0,", "PageRank split product (MAPI)"),
                   ("k_csr_split_combine<0,", "PageRank split combine (MAPI)"),
                   ("k_csr_product<0,", "PageRank plain product (MAPI)"), ("k_gram_min<0,", "min-Gram build (min1)"))


def summarize_counters(dirs, cmds, out_name="kernel_limiters_counters.md"):
    """profiles/ summary of limiter counters (one rocprofv3 --pmc pass per directory) for the
    dense products, the bandwidth references, the PageRank products and the min-Gram build:
    the mean value per dispatch of each counter."""
    table = {}
    counters = []
    for d in dirs:
        for r in _read_csvs(d, "*counter_collection.csv"):
            nm = r.get("Kernel_Name", "")
            for key, label in LIMITER_KERNELS:
                if key in nm:
                    c = r["Counter_Name"]
                    if c not in counters:
                        counters.append(c)
                    table.setdefault(label, {}).setdefault(c, []).append(float(r["Counter_Value"]))
    lines = ["# Limiter counters: dense products, bandwidth references, PageRank products, min-Gram build", "",
             "One `rocprofv3 --pmc` pass per row group of counters, each over `bench.py --mode kernels` "
             "(n = 16384 products in the tuned shapes, the 1 GiB read and copy references, three MAPI PageRank "
             "products at 2^22 nodes with the split and the plain layout, one min1 build at 4096 x 65536). "
             "Values are means per dispatch.", ""]
    lines += [f"Pass {i + 1}: `{c}`" for i, c in enumerate(cmds)] + [""]
    lines += ["| kernel | " + " | ".join(counters) + " |", "|---" * (len(counters) + 1) + "|"]
    for _, label in LIMITER_KERNELS:
        if label not in table:
            continue
        vals = [table[label].get(c) for c in counters]
        lines.append(f"| {label} | " + " | ".join(f"{sum(v) / len(v):.4g}" if v else "-" for v in vals) + " |")
    out = os.path.join(ROOT, "profiles", out_name)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    log(f"wrote {out}")


def bench_launch_cost(mp, ctx, mats, w0, detail):
    """Fixed and per-byte cost of one launch: bare products (no normaliser, the tuned shape of
    the n = 16384 bucket) and the read reference on the first m rows of each stored matrix
    (m = 2048 ... 16384, full rows), fitted as t = fixed + bytes / rate; beside them the solve's
    own product launch (the iterate formed inside it) at m = n."""
    out = {}
    ms_rows = (2048, 4096, 8192, 16384)
    for dt, (A, rs) in mats.items():
        shape = mp.mapi_tuning_get(mp._dtype_code(A), N, N, ctx=ctx)
        xs, tp, tr = [], [], []
        for m in ms_rows:
            Am = A[:m]
            rm = rs[:m] if rs is not None else None
            xs.append(float(Am.numel() * Am.element_size()))
            tp.append(mp.mapi_mavp_timed(Am, w0, shape, "min1", reps=20, row_scale=rm, ctx=ctx) * 1e3)
            tr.append(mp.mapi_read_reference(Am, reps=READ_REPS, ctx=ctx) * 1e3)
        fp, fr = np.polyfit(xs, tp, 1), np.polyfit(xs, tr, 1)
        solve_us = detail.get(f"mapi_{dt}", {}).get("product_kernel_us")
        out[dt] = {"rows": list(ms_rows), "bytes": xs, "product_us": tp, "read_us": tr,
                   "product_fixed_us": float(fp[1]), "product_rate_gbs": float(1e-3 / fp[0]),
                   "read_fixed_us": float(fr[1]), "read_rate_gbs": float(1e-3 / fr[0]),
                   "solve_product_us": solve_us,
                   "solve_minus_bare_us": (solve_us - tp[-1]) if solve_us else None}
        log(f"launch cost {dt}: product {fp[1]:.1f} us + bytes at {1e-3 / fp[0]:.0f} GB/s; read {fr[1]:.1f} us "
            f"+ bytes at {1e-3 / fr[0]:.0f} GB/s; bare product at n {tp[-1]:.1f} us, in the solve {solve_us or 0:.1f} us")
    return out


# ------------------------------------------------------------------ other workloads
def _loguniform_sizes(rng, k, lo, hi):
    return [int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi)))))) for _ in range(k)]


def bench_batched(mp, ctx, torch, k=128, seed=5):
    """Ragged generated problems (n log-uniform in [64, 8192], tol 1e-6): batched BF16 MAPI in one
    persistent launch versus one-at-a-time float32 MAPI and RPI (generation included in both)."""
    rng = np.random.default_rng(seed)
    sizes = _loguniform_sizes(rng, k, 64, 8192)
    seeds = [70000 + i for i in range(k)]
    out = {"instances": k, "sizes": "log-uniform 64..8192", "tol": 1e-6}

    def batched(dt, meth):
        probs = [mp.problem_generated(n, s, dt, meth, max_iters=1000, tol=1e-6, stall_iters=STALL)
                 for n, s in zip(sizes, seeds)]
        mp.mapi_solve_batched(probs[:4], ctx=ctx)                  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = mp.mapi_solve_batched(probs, ctx=ctx)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        return k / dt_s, infos, probs

    def plain(meth):
        fn = mp.mapi_solve if meth == "mapi" else mp.rpi_solve
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n, s in zip(sizes, seeds):
            A, w0 = mp.mapi_generate_dense(n, s, ctx=ctx)
            w, info = fn(A, w0, max_iters=1000, tol=1e-6, check_every=4, stall_iters=STALL, ctx=ctx)
            res.append((w, info))
        torch.cuda.synchronize()
        return k / (time.perf_counter() - t0), res

    for dt, meth in (("bf16", "mapi"), ("f32", "mapi"), ("f32", "rpi")):
        log(f"batched {dt} {meth}: {k} instances")
        sps, infos, probs = batched(dt, meth)
        log(f"batched {dt} {meth}: {sps:.1f} solves/s, mean iters {np.mean([i['iters'] for i in infos]):.1f}")
        out[f"batched_{dt}_{meth}_solves_s"] = sps
        out[f"batched_{dt}_{meth}_mean_iters"] = float(np.mean([i["iters"] for i in infos]))
        out[f"batched_{dt}_{meth}_converged"] = int(sum(i["converged"] for i in infos))
        if (dt, meth) == ("bf16", "mapi"):
            bf16_probs = probs
    for meth in ("mapi", "rpi"):
        log(f"one-at-a-time f32 {meth}")
        sps, res = plain(meth)
        log(f"one-at-a-time f32 {meth}: {sps:.1f} solves/s")
        out[f"plain_f32_{meth}_solves_s"] = sps
        out[f"plain_f32_{meth}_mean_iters"] = float(np.mean([r[1]["iters"] for r in res]))
        if meth == "mapi":
            errs = [float((p.out - w).abs().sum() / w.abs().sum()) for p, (w, _) in zip(bf16_probs, res)]
            out["bf16_batched_vs_f32_plain_mapi_max_rel_l1"] = max(errs)
    return out


def bench_small(mp, ctx, torch, n=256, iters=200, tol=1e-7, seed=SEED, copies=256):
    """The n=256 covariance (X 256x1024 N(0,1), rows centred, b0 ~ U(-1,1)): 200 iterations or
    tol 1e-7, MAPI and RPI.  Latency-bound (the matrix is 256 KiB): microseconds per iteration of
    the plain path, and solves/s of the batched kernel on `copies` instances of the same problem
    (one block iterates each)."""
    import synth
    C = torch.from_numpy(synth.dense_cov(n, 4 * n, seed)).cuda()
    w0 = torch.from_numpy(synth.start_vector(n, seed + 1)).cuda()
    out = {"n": n, "max_iters": iters, "tol": tol}
    for meth in ("mapi", "rpi"):
        fn = mp.mapi_solve if meth == "mapi" else mp.rpi_solve
        _, info = fn(C, w0, max_iters=iters, tol=tol, check_every=16, ctx=ctx)
        reps = 20
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn(C, w0, max_iters=iters, tol=tol, check_every=16, ctx=ctx)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        out[f"{meth}_iters"] = info["iters"]
        out[f"{meth}_plain_us_per_iter"] = sec / max(info["iters"], 1) * 1e6
        if meth == "mapi":
            # the one-block solve writes the min1 term as fma(med3(a, -|w|, |w|), s_w, acc) with
            # s_w = +-1 (an exact sign flip); the multiply-free form (sign flip, med3, add; the
            # same bits) timed beside it
            out["mapi_term"] = "fma(med3(a, -|w|, |w|), s_w, acc), s_w = +-1 from the sign bit of w"
            os.environ["MAPI_MIN1_FORM"] = "xor"
            try:
                wx, ix = fn(C, w0, max_iters=iters, tol=tol, check_every=16, ctx=ctx)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn(C, w0, max_iters=iters, tol=tol, check_every=16, ctx=ctx)
                torch.cuda.synchronize()
                out["mapi_xor_form_us_per_iter"] = (time.perf_counter() - t0) / reps / max(ix["iters"], 1) * 1e6
            finally:
                del os.environ["MAPI_MIN1_FORM"]
            wf, _ = fn(C, w0, max_iters=iters, tol=tol, check_every=16, ctx=ctx)
            out["mapi_xor_form_same_bits"] = bool(torch.equal(wx, wf))
        # the FP64 oracle at the same iteration count (rounding only: same matrix, same start)
        import oracle
        wg, _ = fn(C, w0, max_iters=info["iters"], check_every=16, ctx=ctx)
        orc = oracle.mapi if meth == "mapi" else oracle.rpi
        ref = orc(C.cpu().numpy().astype(np.float64), w0.cpu().numpy().astype(np.float64), info["iters"]).w
        g = wg.double().cpu().numpy()
        out[f"{meth}_rel_l1_vs_oracle"] = float(np.abs(g - ref).sum() / np.abs(ref).sum())
        out[f"{meth}_plain_solves_s"] = 1.0 / sec
        probs = [mp.problem_dense(C, meth, w0=w0, max_iters=iters, tol=tol) for _ in range(copies)]
        mp.mapi_solve_batched(probs[:2], ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mp.mapi_solve_batched(probs, ctx=ctx)
        torch.cuda.synchronize()
        out[f"{meth}_batched_solves_s"] = copies / (time.perf_counter() - t0)
        log(f"small n={n} {meth}: {info['iters']} iterations, {out[f'{meth}_plain_us_per_iter']:.1f} us/iteration, "
            f"batched {out[f'{meth}_batched_solves_s']:.0f} solves/s")
    return out


def bench_hybrid(mp, ctx, torch, D=16384, seed=31):
    """The Sec. 3.2 spectrum at D=16384: C = V diag(1, 0.9, ..., 0.9) V^T = 0.9 I + 0.1 v v^T
    (float32, 1 GiB; top eigenvector v, eigen-gap 0.1) from a random start.  1 - cos^2(w_t, v) after
    fixed iteration counts for RPI, MAPI and MAPI (5 iterations) -> RPI, as in the paper's
    comparison figure; every iteration costs one product launch of the same kernel."""
    import synth
    v = torch.from_numpy(synth.start_vector(D, seed)).cuda()
    C = torch.outer(v, v) * 0.1
    C.diagonal().add_(0.9)
    w0 = torch.from_numpy(synth.start_vector(D, seed + 1)).cuda()
    vd = v.double() / torch.linalg.norm(v.double())
    out = {"D": D, "spectrum": "1, 0.9 (D-1 times)"}

    def gap(w):
        wd = w.double()
        c = float(torch.dot(wd, vd) / torch.linalg.norm(wd))
        return max(0.0, 1.0 - c * c)

    out["rpi"] = {t: gap(mp.rpi_solve(C, w0, max_iters=t, check_every=t, ctx=ctx)[0])
                  for t in (5, 10, 20, 40, 80, 160, 320)}
    out["mapi"] = {t: gap(mp.mapi_solve(C, w0, max_iters=t, check_every=t, ctx=ctx)[0]) for t in (1, 2, 3, 5, 10, 20)}
    out["mapi5_then_rpi"] = {k: gap(mp.mapi_hybrid_solve(C, w0, mapi_iters=5, rpi_iters=k, check_every=8, ctx=ctx)[0])
                             for k in (0, 5, 10, 20, 40)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mp.rpi_solve(C, w0, max_iters=100, check_every=100, ctx=ctx)
    torch.cuda.synchronize()
    out["ms_per_iteration"] = (time.perf_counter() - t0) * 1e3 / 100
    target = 1e-8

    def first(curve, extra=0):
        hit = [t for t, g in sorted(curve.items()) if g <= target]
        return hit[0] + extra if hit else None

    out["iterations_to_1e-8"] = {"rpi": first(out["rpi"]), "mapi": first(out["mapi"]),
                                 "mapi5_then_rpi": first(out["mapi5_then_rpi"], 5)}
    log(f"hybrid D={D}: 1-cos2 RPI {out['rpi']}, MAPI {out['mapi']}, MAPI5->RPI {out['mapi5_then_rpi']}")
    del C
    return out


def bench_minibatch(mp, ctx, torch, N=10 ** 6, D=10, s=1000, T=100, runs=256, seed=41):
    """Algorithm 3 on the Sec. 3.2 construction (N = 10^6 samples, D = 10, eigen-gap 0.1):
    `runs` independent runs (own batches and start vectors), one block each, with and without
    momentum, min1 (Algorithm 3) and dot (the stochastic power method it modifies).  Reports
    samples/s, batch-matrix terms/s and the mean 1 - cos^2 of w_T to the top eigenvector."""
    import synth
    X, v1 = synth.sec32_data(N, D, seed)
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(synth.minibatch_indices(runs, T, s, N, seed + 1)).cuda()
    W0 = torch.from_numpy(np.stack([synth.start_vector(D, seed + 2 + r) for r in range(runs)])).cuda()
    vd = torch.from_numpy(v1).cuda()
    out = {"N": N, "D": D, "s": s, "T": T, "runs": runs}
    for op in ("min1", "dot"):
        for beta in (0.0, 0.2):
            mp.mapi_minibatch(Xd, B, beta, W0, op=op, ctx=ctx)          # warm, workspace sized
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            W, _ = mp.mapi_minibatch(Xd, B, beta, W0, op=op, final_l2=True, ctx=ctx)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            cos = (W.double() @ vd).abs()
            key = f"{op}_beta{beta}"
            out[key] = {"ms": sec * 1e3, "samples_s": runs * T * s / sec, "terms_s": runs * T * s * D * D / sec,
                        "mean_one_minus_cos2": float((1 - cos * cos).mean()),
                        "median_one_minus_cos2": float((1 - cos * cos).median())}
            log(f"minibatch {key}: {sec * 1e3:.2f} ms, {runs * T * s / sec / 1e9:.2f} G samples/s, "
                f"median 1-cos2 {out[key]['median_one_minus_cos2']:.2e}")
    return out


def bench_image(mp, ctx, torch, D=128, N=10, seed=1):
    """Algorithm 2 at the Sec. 3.1 sizes: a synthetic 128 x 128 image, N = 10 copies with 3 of 16
    tiles replaced by U[0,1] noise; MAPI with the min1 product (eq. 3), MAPI with the min2 product
    (eq. 4; Table 1's min2-PI column) and RPI, each vector to an l1 change < 1e-6 (stall rule).  Reports the wall time of the whole pipeline (min-covariance of 16384 pixels, two solves,
    the deflation, the reconstruction) and the mean PSNR of the N reconstructions and of the inputs."""
    import synth
    clean, V = synth.occluded_images(D, N, seed)
    Vd = torch.from_numpy(V).cuda()
    w0 = torch.from_numpy(synth.start_vector(D * D, seed + 1)).cuda()
    cl = torch.from_numpy(clean).cuda().double()

    def psnr(x):
        mse = float(((x.double() - cl) ** 2).mean())
        return 10.0 * np.log10(1.0 / mse)

    out = {"D": D, "N": N, "pixels": D * D, "inputs_psnr_db": float(np.mean([psnr(Vd[:, i]) for i in range(N)]))}
    for tag, meth, op in (("mapi", "mapi", "min1"), ("mapi_min2", "mapi", "min2"), ("rpi", "rpi", "min1")):
        run = lambda: mp.mapi_image_reconstruct(Vd, w0, meth, max_iters=500, tol=1e-6, check_every=8,
                                               stall_iters=STALL, op=op, ctx=ctx)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R, W, infos = run()
        torch.cuda.synchronize()
        out[f"{tag}_ms"] = (time.perf_counter() - t0) * 1e3
        out[f"{tag}_iters"] = [i["iters"] for i in infos]
        out[f"{tag}_psnr_db"] = float(np.mean([psnr(R[:, i]) for i in range(N)]))
        log(f"image {tag}: {out[f'{tag}_ms']:.1f} ms, iterations {out[f'{tag}_iters']}, "
            f"PSNR {out[f'{tag}_psnr_db']:.2f} dB (inputs {out['inputs_psnr_db']:.2f} dB)")
    return out


def bench_pca(mp, ctx, torch, D=4096, N=65536, k=8, seed=77):
    import synth
    log("PCA: generating X 4096 x 65536 on the GPU")
    X, clean = synth.pca_data_device(D, N, seed, "cuda")
    if not bool(torch.isfinite(X).all()):
        raise RuntimeError("PCA input has non-finite entries")
    W0 = torch.from_numpy(synth.start_vectors(D, k, seed + 1)).cuda()
    terms = D * (D + 1) / 2 * N
    out = {"D": D, "N": N, "k": k}
    for op in ("min1", "dot"):
        mp.mapi_mingram(X, 1.0 / N, op, ctx=ctx)
        torch.cuda.synchronize()
        s = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            A = mp.mapi_mingram(X, 1.0 / N, op, ctx=ctx)
            torch.cuda.synchronize()
            s = min(s, time.perf_counter() - t0)
        out[f"gram_{op}_ms"] = s * 1e3
        out[f"gram_{op}_gterms_s"] = terms / s / 1e9
        # sampled entries against the FP64 oracle, relative to the sum of |terms| (the bound's scale)
        import oracle
        rng = np.random.default_rng(3)
        pairs = [(0, 0), (D - 1, D - 1), (0, D - 1)] + [tuple(int(v) for v in p) for p in rng.integers(0, D, (5, 2))]
        Ah = A[[i for i, _ in pairs], [j for _, j in pairs]].double().cpu().numpy()
        worst = 0.0
        for (i, j), a in zip(pairs, Ah):
            xi, xj = X[i].double().cpu().numpy(), X[j].double().cpu().numpy()
            ref = oracle.mingram_entry(np.stack([xi, xj]), 0, 1, 1.0 / N, op)
            scale = (np.minimum(np.abs(xi), np.abs(xj)) if op == "min1" else np.abs(xi * xj)).sum() / N
            worst = max(worst, abs(a - ref) / scale)
        out[f"gram_{op}_sampled_err_vs_oracle"] = worst
        if op == "min1":
            # per 16 terms of a lane's 4 x 4 tile: 16 med3, 16 FMAs (sign of b as +-1) and 4 sign
            # words, over every term of the 128 x 128 tiles the build computes (diagonal tiles
            # whole), against the vector ALU rate (256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz)
            T = (D + 127) // 128
            executed = T * (T + 1) / 2 * 128 * 128 * N
            out["gram_min1_executed_terms"] = executed
            out["gram_min1_valu_frac"] = executed * 2.25 / s / 78.6e12
            out["gram_min1_term"] = ("fma(med3(a, -|b|, |b|), s_b, acc), s_b = +-1 from the sign bit of b: an "
                                     "exact sign flip in one instruction with the add, not a product of data")
            # the same build with the term as sign-bit flip, med3 and add (three instructions;
            # the same bits): the multiply-free form's time beside it
            os.environ["MAPI_MIN1_FORM"] = "xor"
            try:
                Ax = mp.mapi_mingram(X, 1.0 / N, op, ctx=ctx)
                torch.cuda.synchronize()
                sx = float("inf")
                for _ in range(3):
                    t0 = time.perf_counter()
                    Ax = mp.mapi_mingram(X, 1.0 / N, op, ctx=ctx)
                    torch.cuda.synchronize()
                    sx = min(sx, time.perf_counter() - t0)
            finally:
                del os.environ["MAPI_MIN1_FORM"]
            out["gram_min1_xor_form_ms"] = sx * 1e3
            out["gram_min1_xor_form_same_bits"] = bool(torch.equal(Ax, A))
            del Ax
        else:
            # the covariance runs on the matrix cores: 2 flops per term against the FP32 MFMA peak
            out["gram_dot_tflops"] = 2.0 * terms / s / 1e12
            out["gram_dot_mfma_frac"] = 2.0 * terms / s / 157.3e12
        del A
    cn = torch.linalg.norm(clean)
    for meth in ("mapi", "rpi"):
        log(f"PCA top-{k} {meth}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, infos = mp.mapi_pca_topk(X, k, W0, method=meth, max_iters=1000, tol=1e-6, check_every=8, ctx=ctx)
        torch.cuda.synchronize()
        out[f"pca_{meth}_ms"] = (time.perf_counter() - t0) * 1e3
        out[f"pca_{meth}_iters"] = [i["iters"] for i in infos]
        out[f"pca_{meth}_converged"] = int(sum(i["converged"] for i in infos))
        recon = P @ (P.t() @ clean)
        out[f"pca_{meth}_reconstruction_error"] = float(torch.linalg.norm(clean - recon) / cn)
        # where the time goes: a second run with the kernel timers (events around each launch)
        ctx.timing(True)
        ctx.timing_reset()
        mp.mapi_pca_topk(X, k, W0, method=meth, max_iters=1000, tol=1e-6, check_every=8, ctx=ctx)
        torch.cuda.synchronize()
        out[f"pca_{meth}_kernel_ms"] = {kind: ctx.timing_get(kind)[0] for kind in ("gram", "mavp", "finalize", "deflate")}
        ctx.timing(False)
        if meth == "mapi":
            p_mapi = P[:, 0].clone()
    # the factored operator X (+) (X^T (+) w) / N (not a method of the paper): the first vector to
    # the same stop rule, streaming X twice per iteration instead of building A once
    log("PCA: factored operator, first vector")
    mp.mapi_factored_solve(X, W0[:, 0].contiguous(), max_iters=2, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wf, inf = mp.mapi_factored_solve(X, W0[:, 0].contiguous(), max_iters=1000, tol=1e-6, check_every=8,
                                     stall_iters=STALL, ctx=ctx)
    torch.cuda.synchronize()
    s = time.perf_counter() - t0
    wf2 = wf.double() / torch.linalg.norm(wf.double())
    out["factored_iters"] = inf["iters"]
    out["factored_converged"] = inf["converged"]
    out["factored_ms"] = s * 1e3
    out["factored_ms_per_iteration"] = s * 1e3 / max(inf["iters"], 1)
    out["factored_gbs"] = 2.0 * 4.0 * D * N * inf["iters"] / s / 1e9     # X read twice per iteration
    out["factored_abs_cos_vs_mapi_vector"] = float(abs(torch.dot(wf2, p_mapi.double())))
    log(f"PCA factored: {inf['iters']} iterations in {s * 1e3:.1f} ms, {out['factored_gbs']:.0f} GB/s, "
        f"|cos| to the MAPI vector {out['factored_abs_cos_vs_mapi_vector']:.4f}")
    del X, clean
    return out


_GRAPHS = {}


def _graph(n, seed):
    """The power-law graph of the PageRank workload (host CSR), generated once per run."""
    import synth
    if (n, seed) not in _GRAPHS:
        _GRAPHS[(n, seed)] = synth.powerlaw_graph(n, seed)
    return _GRAPHS[(n, seed)]


def bench_pagerank(mp, ctx, torch, n=1 << 22, seed=2022):
    log("PageRank: generating the 2^22-node graph on the host")
    g = _graph(n, seed)
    traffic = load_csr_traffic() if (n, seed) == (PR_N, PR_SEED) else None
    rp, col, val = (torch.from_numpy(g[x]).cuda() for x in ("row_ptr", "col", "val"))
    nnz = int(g["col"].size)
    bytes_iter = 8.0 * nnz + 4.0 * (n + 1) + 8.0 * n        # links, row pointers, w once, y once
    out = {"n": n, "nnz": nnz}
    # `ctx` has the default policy (plain products for the first 4 iterations, the split layout
    # built only if the solve is still running); `eager` builds the split layout before the first
    # product, so its per-product times are the split kernel's alone
    eager = mp.Context()
    mp.mapi_pagerank_split_after(0, ctx=eager)
    for meth in ("mapi", "rpi"):
        log(f"PageRank {meth}")
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=2, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, info = mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=300, tol=1e-8, stall_iters=10,
                                   check_every=4, ctx=ctx)
        torch.cuda.synchronize()
        s = time.perf_counter() - t0
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=2, ctx=eager)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=300, tol=1e-8, stall_iters=10, check_every=4,
                         ctx=eager)
        torch.cuda.synchronize()
        s_eager = time.perf_counter() - t0
        # per product: a fixed 10-product run (tol 0), so that every timed launch does its
        # work (after the stop rule has fired, the launches of a converged run return at once)
        eager.timing(True)
        eager.timing_reset()
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=10, ctx=eager)
        ms, launches = eager.timing_get("csr")
        eager.timing(False)
        kms = ms / max(launches, 1)
        out[f"{meth}_iters"] = info["iters"]
        out[f"{meth}_converged"] = info["converged"]
        out[f"{meth}_final_residual"] = info["residual"]
        out[f"{meth}_ms_total"] = s * 1e3
        out[f"{meth}_ms_total_split_from_first"] = s_eager * 1e3
        out[f"{meth}_csr_kernel_us"] = kms * 1e3
        out[f"{meth}_gedges_s"] = nnz / (kms * 1e-3) / 1e9
        out[f"{meth}_csr_kernel_gbs"] = bytes_iter / (kms * 1e-3) / 1e9
    # the MAPI iterate against the FP64 oracle (CSR form) at the GPU's iteration count: the rank
    # signal is the deviation from 1/n, so its relative l1 error and the top-100 overlap
    import oracle
    wm, im = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=300, tol=1e-8, stall_iters=10, check_every=4,
                              ctx=ctx)
    ref = oracle.pagerank(n, g["row_ptr"], g["col"], g["val"], 0.85, "mapi", np.full(n, 1.0 / n), im["iters"]).w
    wg = wm.double().cpu().numpy()
    dev_g, dev_r = wg - 1.0 / n, ref - 1.0 / n
    out["mapi_oracle_iters"] = im["iters"]
    out["mapi_rel_l1_vs_oracle"] = float(np.abs(wg - ref).sum() / np.abs(ref).sum())
    out["mapi_deviation_rel_l1_vs_oracle"] = float(np.abs(dev_g - dev_r).sum() / np.abs(dev_r).sum())
    top_g, top_r = np.argsort(-wg, kind="stable")[:100], np.argsort(-ref, kind="stable")[:100]
    out["mapi_top100_overlap_vs_oracle"] = len(set(top_g.tolist()) & set(top_r.tolist()))
    # the float64 iterate (mapi_pagerank_f64): time per product and the same comparison
    mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=2, f64=True, ctx=ctx)
    ctx.timing(True)
    ctx.timing_reset()
    w64, i64 = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=im["iters"], f64=True, ctx=ctx)
    torch.cuda.synchronize()
    ms, launches = ctx.timing_get("csr")
    ctx.timing(False)
    g64 = w64.cpu().numpy()
    out["mapi_f64_csr_kernel_us"] = ms / max(launches, 1) * 1e3
    out["mapi_f64_deviation_rel_l1_vs_oracle"] = float(np.abs((g64 - 1.0 / n) - dev_r).sum() / np.abs(dev_r).sum())
    out["mapi_f64_top100_overlap_vs_oracle"] = len(set(np.argsort(-g64, kind="stable")[:100].tolist())
                                                   & set(top_r.tolist()))
    log(f"PageRank float64 iterate: {out['mapi_f64_csr_kernel_us']:.0f} us per product, top-100 overlap "
        f"{out['mapi_f64_top100_overlap_vs_oracle']} (float32: {out['mapi_top100_overlap_vs_oracle']})")
    # the plain CSR product on the same graph (no column split), per product
    plain = mp.Context()
    mp.mapi_pagerank_split_config(0, ctx=plain)
    for meth in ("mapi", "rpi"):
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=2, ctx=plain)
        plain.timing(True)
        plain.timing_reset()
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=10, ctx=plain)
        ms, launches = plain.timing_get("csr")
        plain.timing(False)
        out[f"{meth}_plain_csr_kernel_us"] = ms / max(launches, 1) * 1e3
    log(f"PageRank products: split {out['mapi_csr_kernel_us']:.0f} us (MAPI) / {out['rpi_csr_kernel_us']:.0f} us "
        f"(RPI), plain {out['mapi_plain_csr_kernel_us']:.0f} / {out['rpi_plain_csr_kernel_us']:.0f} us; solves "
        f"{out['mapi_ms_total']:.1f} / {out['rpi_ms_total']:.1f} ms (split from the first product: "
        f"{out['mapi_ms_total_split_from_first']:.1f} / {out['rpi_ms_total_split_from_first']:.1f} ms)")
    plain.close()
    eager.close()
    # Sec. 3.3's comparison at the 1e-8 stop, with the float64 iterate (the float32 iterate's
    # floor, about 5e-8 in l1 at this n, stops RPI short of it): iterations and time to an l1
    # change below 1e-8, MAPI against RPI
    for meth in ("mapi", "rpi"):
        mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=2, f64=True, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=500, tol=1e-8, check_every=4, f64=True,
                                  ctx=ctx)
        torch.cuda.synchronize()
        s = time.perf_counter() - t0
        out[f"{meth}_f64_to_1e-8_iters"] = inf["iters"]
        out[f"{meth}_f64_to_1e-8_converged"] = inf["converged"]
        out[f"{meth}_f64_to_1e-8_residual"] = inf["residual"]
        out[f"{meth}_f64_to_1e-8_ms"] = s * 1e3
        log(f"PageRank float64 {meth} to 1e-8: {inf['iters']} iterations, converged {inf['converged']}, "
            f"{s * 1e3:.1f} ms")
    # counter bytes of the MAPI product (FETCH_SIZE + WRITE_SIZE, scaled; the gathers of w are
    # counted as the L2 fills they cause)
    out["mapi_csr_traffic_bytes"] = traffic
    if traffic:
        out["mapi_csr_traffic_ratio"] = traffic / bytes_iter
        out["mapi_csr_traffic_gbs"] = traffic / (out["mapi_csr_kernel_us"] * 1e-6) / 1e9
    return out


def _cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def oracle_workers():
    """Worker processes for the row-parallel oracle runs: the usable host CPUs, at most 16."""
    return max(1, min(16, _cpu_info()["usable_cpus"] or 1))


_ORACLE_A = None


def _oracle_worker_init(shm_name, shape):
    # a spawned worker (it never touches the GPU) maps the shared FP64 matrix
    global _ORACLE_A, _ORACLE_SHM
    from multiprocessing import shared_memory
    _ORACLE_SHM = shared_memory.SharedMemory(name=shm_name)
    _ORACLE_A = np.ndarray(shape, dtype=np.float64, buffer=_ORACLE_SHM.buf)


def _oracle_worker_rows(task):
    import oracle
    r0, r1, w = task
    return oracle.mavp(_ORACLE_A[r0:r1], w)


def oracle_parallel_iterations(A, w0, seconds, max_iters, workers, rows=256):
    """MAPI iterations of the unchanged oracle product with its rows split over `workers` spawned
    processes (the matrix in shared memory, one block of rows per task); returns (iterations,
    seconds).  The processes are children started with a fresh interpreter."""
    import multiprocessing as mproc
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(create=True, size=A.nbytes)
    try:
        As = np.ndarray(A.shape, dtype=np.float64, buffer=shm.buf)
        As[:] = A
        blocks = [(r, min(A.shape[0], r + rows)) for r in range(0, A.shape[0], rows)]
        with mproc.get_context("spawn").Pool(workers, _oracle_worker_init, (shm.name, A.shape)) as pool:
            pool.map(_oracle_worker_rows, [(0, 1, w0)] * workers)          # start-up, untimed
            w = np.asarray(w0, dtype=np.float64)
            its = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < seconds and its < max_iters:
                y = np.concatenate(pool.map(_oracle_worker_rows, [(a, b, w) for a, b in blocks]))
                w = y / np.abs(y).sum()
                its += 1
            dt = time.perf_counter() - t0
        del As
        return its, dt
    finally:
        shm.close()
        shm.unlink()


def bench_oracle():
    """The FP64 CPU oracle, untuned, on bounded samples of each workload, one host thread:
    per-iteration and per-solve times (extrapolated where the whole workload would take minutes)."""
    import oracle
    import synth
    out = dict(_cpu_info())
    # n = 256 covariance, 200 MAPI iterations (a whole solve)
    C = synth.dense_cov(256, 1024, SEED)
    w0 = synth.start_vector(256, SEED + 1)
    t0 = time.perf_counter()
    oracle.mapi(C, w0, 200)
    s = time.perf_counter() - t0
    out["small_n256_ms_per_solve"] = s * 1e3
    out["small_n256_us_per_iter"] = s / 200 * 1e6
    log(f"oracle n=256: {s * 1e3:.0f} ms per 200-iteration solve")
    # min-covariance of the PCA workload (4096 x 65536): the build on 64 coordinates, extrapolated
    D, Nn = 4096, 65536
    Xs = synth.pca_data(64, Nn, 77)
    t0 = time.perf_counter()
    oracle.mingram(Xs, 1.0 / Nn, "min1")
    s = time.perf_counter() - t0
    rate = 64 * 64 * Nn / s
    out["pca_min_gram_terms_s"] = rate
    out["pca_min_gram_s_extrapolated"] = D * (D + 1) / 2 * Nn / rate
    out["pca_min_gram_sample"] = "64 x 64 entries over 65536 samples (all ordered pairs)"
    log(f"oracle min-Gram: {rate / 1e6:.0f} M terms/s, full build ~{out['pca_min_gram_s_extrapolated']:.0f} s")
    # PageRank at 2^22: one iteration of each product (CSR form)
    n = 1 << 22
    g = _graph(n, 2022)
    dang = oracle.dangling_mask(n, g["col"])
    w = np.full(n, 1.0 / n)
    for meth, fn in (("mapi", oracle.pagerank_mavp_csr), ("rpi", oracle.pagerank_rpi_csr)):
        t0 = time.perf_counter()
        fn(n, g["row_ptr"], g["col"], g["val"], 0.85, w, dang)
        out[f"pagerank_{meth}_ms_per_iter"] = (time.perf_counter() - t0) * 1e3
    log(f"oracle PageRank: MAPI {out['pagerank_mapi_ms_per_iter']:.0f} ms, RPI {out['pagerank_rpi_ms_per_iter']:.0f} ms "
        f"per iteration")
    # the generated mix (n log-uniform in [64, 8192]): one float32 MAPI solve (tol 1e-6) at the
    # geometric middle of each quarter of the range; the mean is the expected time per request
    ns = [int(round(64 * 128 ** ((k + 0.5) / 4))) for k in range(4)]
    per = []
    for k, nk in enumerate(ns):
        A, w0 = synth.generated_dense(nk, 90000 + k)
        t0 = time.perf_counter()
        r = oracle.mapi(A, w0, 1000, tol=1e-6)
        per.append(time.perf_counter() - t0)
        out[f"mix_n{nk}_ms_per_solve"] = per[-1] * 1e3
        out[f"mix_n{nk}_iters"] = r.iters
    out["mix_solves_s_estimate"] = 1.0 / (sum(per) / len(per))
    out["mix_sample"] = f"one solve per quarter of log-uniform [64, 8192] (n = {ns}), equal weights"
    log(f"oracle mix: {out['mix_solves_s_estimate']:.2f} solves/s")
    return out


def bench_serving(mp, torch, n_req=20000, rate=2000.0, seed=11, budget=64 << 30, n_sat=8000):
    """Poisson arrivals; 70 % dense generated problems (n log-uniform 64..8192, BF16/F32, MAPI/RPI),
    30 % PageRank on power-law graphs with 2^10..2^20 nodes (a resident pool of 11 graphs, one per
    power of two, in pinned host memory), tolerance 1e-6 each; compared with the one-at-a-time
    plain path (FIFO, float32) run on the same arrivals."""
    import synth
    rng = np.random.default_rng(seed)
    log("serving: building the graph pool")
    pool = {}
    for e in range(10, 21):
        g = synth.powerlaw_graph(1 << e, seed=900 + e)
        pinned = {}
        for key in ("row_ptr", "col", "val"):
            t = torch.empty(g[key].shape, dtype=torch.from_numpy(g[key][:1]).dtype, pin_memory=True)
            t.numpy()[...] = g[key]
            pinned[key] = t
        pool[e] = pinned
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    reqs = []
    for i in range(n_req):
        if rng.uniform() < 0.7:
            n = int(round(float(np.exp(rng.uniform(np.log(64), np.log(8192))))))
            reqs.append(("gen", n, ["f32", "bf16"][rng.integers(2)], ["mapi", "rpi"][rng.integers(2)], 10_000_000 + i))
        else:
            e = int(rng.integers(10, 21))
            reqs.append(("csr", 1 << e, "f32", ["mapi", "rpi"][rng.integers(2)], e))

    def make(r):
        kind, n, dt, meth, s = r
        if kind == "gen":
            return mp.request_generated(n, s, dt, meth, max_iters=1000, tol=1e-6, stall_iters=STALL)
        p = pool[s]
        return mp.request_csr_host(p["row_ptr"], p["col"], p["val"], 0.85, meth,
                                   max_iters=1000, tol=1e-6, stall_iters=STALL)

    log(f"serving: {n_req} requests at {rate:.0f}/s")
    srv = mp.Server(budget_bytes=budget)
    tickets = []
    t_start = time.perf_counter()
    for i, r in enumerate(reqs):
        wait = arrivals[i] - (time.perf_counter() - t_start)
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(make(r), np.empty(r[1], np.float32)))
        if i % 2000 == 0:
            log(f"serving: submitted {i}")
    res = [srv.wait(t, timeout_us=120_000_000) for t in tickets]
    st = srv.stats()
    srv.close()
    ok = sum(1 for x in res if x is not None and x["status"] == "OK")
    out = {"requests": n_req, "rate_per_s": rate, "completed_ok": ok, "solves_s": st["solves_per_s"],
           "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "peak_pool_bytes": st["peak_bytes"],
           "budget_bytes": budget, "kernel_launches": st["kernel_launches"],
           "converged": int(sum(1 for x in res if x and x["converged"]))}
    # capacity: the first n_sat requests of the same mix submitted back to back
    n_sat = min(n_sat, n_req)
    log(f"serving: capacity run, {n_sat} requests submitted at once")
    srv = mp.Server(budget_bytes=budget)
    tickets = [srv.submit(make(r), np.empty(r[1], np.float32)) for r in reqs[:n_sat]]
    res_sat = [srv.wait(t, timeout_us=120_000_000) for t in tickets]
    st = srv.stats()
    srv.close()
    out["saturated_requests"] = n_sat
    out["saturated_completed_ok"] = sum(1 for x in res_sat if x is not None and x["status"] == "OK")
    out["saturated_solves_s"] = st["solves_per_s"]
    out["saturated_p50_ms"] = st["p50_ms"]
    out["saturated_p99_ms"] = st["p99_ms"]
    out["saturated_kernel_launches"] = st["kernel_launches"]
    out["saturated_peak_pool_bytes"] = st["peak_bytes"]
    # the one-at-a-time plain path on the same arrival process: float32, FIFO, one solve after
    # another on one stream, each request started at its arrival time or when the previous one
    # is done; latency from arrival to the result in host memory
    log(f"serving: one-at-a-time path on the same {n_req} arrivals")
    ctx = mp.Context()
    lat = np.empty(n_req)
    t_start = time.perf_counter()
    for i, (kind, n, dt, meth, s) in enumerate(reqs):
        wait = arrivals[i] - (time.perf_counter() - t_start)
        if wait > 0:
            time.sleep(wait)
        if kind == "gen":
            A, w0 = mp.mapi_generate_dense(n, s, ctx=ctx)
            fn = mp.mapi_solve if meth == "mapi" else mp.rpi_solve
            w, _ = fn(A, w0, max_iters=1000, tol=1e-6, check_every=4, stall_iters=STALL, ctx=ctx)
        else:
            p = pool[s]
            rp, col, val = (p[k].cuda(non_blocking=True) for k in ("row_ptr", "col", "val"))
            w, _ = mp.mapi_pagerank(rp, col, val, 0.85, meth, max_iters=1000, tol=1e-6, check_every=4,
                                    stall_iters=STALL, ctx=ctx)
        w.cpu()
        lat[i] = (time.perf_counter() - t_start) - arrivals[i]
        if i % 2000 == 0:
            log(f"serving: one-at-a-time {i} done")
    total = time.perf_counter() - t_start
    ctx.close()
    out["plain_f32_solves_s"] = n_req / (total - float(arrivals[0]))
    out["plain_f32_p50_ms"] = float(np.percentile(lat, 50) * 1e3)
    out["plain_f32_p99_ms"] = float(np.percentile(lat, 99) * 1e3)
    return out


# ------------------------------------------------------------------ benchmark
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="bench", choices=["bench", "kernels"])
    ap.add_argument("--sections", default="small,hybrid,minibatch,image,batched,pca,pagerank,serving,oracle",
                    help="other workloads reported under detail (comma list; empty for none)")
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-sections", metavar="STATS_DIR",
                    help="write the kernel summary of the pca, small and minibatch sections (first --commands entry)")
    ap.add_argument("--commands", nargs="+", default=["", "", ""], help="commands that produced the dirs")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="write the limiter counter summary from rocprofv3 --pmc directories (with --commands)")
    ap.add_argument("--bench-json", default=None, help="JSON line printed by the profiled benchmark command")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.commands)
        return
    if args.summarize_sections:
        summarize_sections(args.summarize_sections, args.commands[0], bench_json=args.bench_json)
        return
    if args.summarize:
        summarize(*args.summarize, *args.commands, bench_json=args.bench_json)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    if args.mode == "kernels":
        run_kernels_mode()
        return

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

    # Attainable read bandwidth on the same matrices: a plain streaming read.
    reads = {}
    for dt, (A, _) in mats.items():
        nbytes = A.numel() * A.element_size()
        ms = mp.mapi_read_reference(A, reps=READ_REPS, ctx=ctx)
        reads[dt] = {"bytes": nbytes, "us": ms * 1e3, "gbs": nbytes / (ms * 1e-3) / 1e9}
        log(f"read reference {dt}: {ms * 1e3:.1f} us, {reads[dt]['gbs']:.0f} GB/s")
    detail["read_reference"] = reads
    detail["launch_cost"] = bench_launch_cost(mp, ctx, mats, w0, detail)

    sections = [x for x in args.sections.split(",") if x]
    for name, fn in (("small", lambda: bench_small(mp, ctx, torch)), ("hybrid", lambda: bench_hybrid(mp, ctx, torch)),
                     ("minibatch", lambda: bench_minibatch(mp, ctx, torch)), ("image", lambda: bench_image(mp, ctx, torch)),
                     ("batched", lambda: bench_batched(mp, ctx, torch)), ("pca", lambda: bench_pca(mp, ctx, torch)),
                     ("pagerank", lambda: bench_pagerank(mp, ctx, torch)), ("serving", lambda: bench_serving(mp, torch)),
                     ("oracle", bench_oracle)):
        if name in sections:
            log(f"section {name}")
            t0 = time.perf_counter()
            detail[name] = fn()
            detail[name]["section_wall_s"] = time.perf_counter() - t0
            log(f"section {name} done in {detail[name]['section_wall_s']:.1f} s")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the FP64 CPU oracle on a bounded sample")
        Ch = C.cpu().numpy().astype(np.float64)
        w = w0.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        its = 0
        while its < ITERS:        # one whole step: the result is also the accuracy reference below
            y = oracle.mavp(Ch, w)
            w = y / np.abs(y).sum()
            its += 1
        dt_s = time.perf_counter() - t0
        cpu = {"value": its * float(N) * N / dt_s / 1e9, "unit": "Gelem/s", "cores": 1, "kind": "oracle",
               "sample": f"{its} full MAPI iterations (min1 product + l1 normalisation) of the n=16384 FP64 "
                         f"oracle, numpy, one thread, {dt_s:.1f} s"}
        # each storage mode's 20-iteration GPU iterate against this FP64 oracle on the float32 matrix
        # (for BF16 / FP8 the error of storing the matrix in 2 or 1 bytes: reported, not bounded)
        acc = {}
        for dt in ("f32", "bf16", "fp8"):
            A, rs = mats[dt]
            wg, _ = mp.mapi_solve(A, w0, max_iters=ITERS, row_scale=rs, check_every=ITERS, ctx=ctx)
            g = wg.double().cpu().numpy()
            acc[dt] = {"rel_l1": float(np.abs(g - w).sum() / np.abs(w).sum()),
                       "cosine": float(abs(g @ w) / (np.linalg.norm(g) * np.linalg.norm(w)))}
        detail["accuracy_vs_fp64_oracle"] = acc
        log("accuracy against the FP64 oracle: " + ", ".join(f"{k} rel-l1 {v['rel_l1']:.2e}" for k, v in acc.items()))
        # the same oracle product over blocks of rows on all usable host CPUs (at most 16)
        nw = oracle_workers()
        its_p, dt_p = oracle_parallel_iterations(Ch, w0.cpu().numpy(), 8.0, 40, nw)
        detail.setdefault("oracle", {})["headline_rows_parallel"] = {
            "processes": nw, "iterations": its_p, "seconds": dt_p,
            "gelem_s": its_p * float(N) * N / dt_p / 1e9, **_cpu_info()}
        log(f"oracle on {nw} processes: {its_p * float(N) * N / dt_p / 1e9:.2f} Gelem/s")
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
                     "algorithmic_bytes_per_launch": product_bytes("f32"), "avg_launch_us": k_ms * 1e3,
                     "read_reference_gbs": reads["f32"]["gbs"], "frac_of_read_reference": achieved / reads["f32"]["gbs"]},
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
