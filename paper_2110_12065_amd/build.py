"""Build libmapi.so (HIP, gfx950 only) in-tree with hipcc.

    python -m paper_2110_12065_amd.build [--no-checked]

Objects go to paper_2110_12065_amd/_build/, the library to
paper_2110_12065_amd/libmapi.so.  Every call recompiles.  Unless --no-checked, the same
call also links libmapi_checked.so (its checked objects in _build/checked/, compiled with
MAPI_DEVICE_CHECKS: device-side index checks that record the first failure in the solve
state, for debugging).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmapi.so")
LIB_CHECKED = os.path.join(HERE, "libmapi_checked.so")

SOURCES = ["k_dense_f32.hip", "k_dense_bf16.hip", "k_dense_fp8.hip", "k_dense.hip", "k_quant.hip", "k_csr.hip", "k_csr_split.hip",
           "k_gram.hip", "k_factored.hip", "k_small.hip", "k_minibatch.hip", "k_image.hip", "k_batched.hip", "batch.hip", "serve.hip", "api.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for device code; the host pass reports the
# feature as unknown, which is harmless.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
    "-Wno-unused-command-line-argument",
]


def _compile(src, checked=False):
    obj = os.path.join(BUILD, "checked" if checked else "", os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DMAPI_DEVICE_CHECKS"] if checked else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    return obj, errs


# Translation units with device checks (MAPI_DCHECK); the checked library takes every
# other object from the ordinary build (the macro does not occur in them).
CHECKED_SOURCES = ["k_dense_f32.hip", "k_dense_bf16.hip", "k_dense_fp8.hip", "k_dense.hip", "k_csr.hip",
                   "k_csr_split.hip", "k_batched.hip"]


def _link(lib_path, objs):
    tmp = lib_path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, lib_path)
    return lib_path


def build(verbose=False, checked=True):
    """Compile every source and link libmapi.so, and with `checked` also libmapi_checked.so
    (the checked objects compile in the same pool).  Returns the ordinary library's path."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(os.path.join(BUILD, "checked"), exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + ([(src, True) for src in CHECKED_SOURCES] if checked else [])
    # the largest units first, so that they do not start last
    jobs.sort(key=lambda j: -os.path.getsize(os.path.join(CSRC, j[0])) - (1 << 20) * j[0].startswith("k_dense_"))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        done = dict(zip(jobs, ex.map(lambda j: _compile(*j), jobs)))
    for obj, msg in done.values():
        if verbose and msg.strip():
            print(msg)
    _link(LIB, [done[(src, False)][0] for src in SOURCES])
    if checked:
        _link(LIB_CHECKED, [done[(src, src in CHECKED_SOURCES)][0] for src in SOURCES])
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, checked="--no-checked" not in sys.argv))
