"""The device-checked build (libmapi_checked.so, MAPI_DEVICE_CHECKS): the same workloads run
clean through it and give the results of the ordinary build; a check that is made to fail
(MAPI_DCHECK_SELFTEST=1, no out-of-bounds access involved) reaches the caller as
MAPI_ERR_DEVICE_CHECK.  Each case runs in a child process, since the binding loads one
library per process."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

WORK = r'''
import json, sys
import numpy as np
import torch
sys.path.insert(0, ROOT)
import synth
import paper_2110_12065_amd as mp
out = {"lib": mp.LIB_PATH}
A32, _, _ = synth.planted_symmetric(1008, [0.4], seed=3)
w0 = torch.from_numpy(synth.start_vector(1008, 4)).cuda()
for dt in ("f32", "bf16", "fp8"):
    A, rs = (torch.from_numpy(A32).cuda(), None) if dt == "f32" else mp.mapi_quantize(torch.from_numpy(A32).cuda(), dt)
    w, info = mp.mapi_solve(A, w0, max_iters=25, row_scale=rs)
    out[dt] = w.cpu().numpy().tolist()
g = synth.powerlaw_graph(6000, seed=9)
rp, col, val = (torch.from_numpy(g[k]).cuda() for k in ("row_ptr", "col", "val"))
ctx = mp.Context()
mp.mapi_pagerank_split_config(1024, ctx=ctx)                   # the column-split product at this size
w, _ = mp.mapi_pagerank(rp, col, val, 0.85, "mapi", max_iters=6, ctx=ctx)
out["pr_split"] = w.cpu().numpy().tolist()
w, _ = mp.mapi_pagerank(rp, col, val, 0.85, "rpi", max_iters=6)
out["pr_plain"] = w.cpu().numpy().tolist()
probs = [mp.problem_generated(n, 40 + n, "bf16", "mapi", max_iters=12) for n in (100, 700, 3000)]
mp.mapi_solve_batched(probs)
out["batched"] = [p.out.cpu().numpy().tolist() for p in probs]
print("RESULT " + json.dumps(out), flush=True)
'''


def _run(env_extra, code):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, "-u", "-c", "ROOT = %r\n" % ROOT + code], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    return r


def _result(r):
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


@pytest.fixture(scope="module")
def checked_built():
    if not os.path.exists(os.path.join(ROOT, "paper_2110_12065_amd", "libmapi_checked.so")):
        pytest.skip("libmapi_checked.so not built")


def test_checked_build_runs_clean_and_matches(checked_built):
    print("[case] device-checked build: dense f32/bf16/fp8, PageRank split and plain, batched", flush=True)
    plain = _result(_run({"MAPI_CHECKED": "0"}, WORK))
    checked = _result(_run({"MAPI_CHECKED": "1"}, WORK))
    assert checked["lib"].endswith("libmapi_checked.so") and plain["lib"].endswith("libmapi.so")
    for k in ("f32", "bf16", "fp8", "pr_split", "pr_plain"):
        np.testing.assert_array_equal(np.array(checked[k]), np.array(plain[k]), err_msg=k)
    for a, b in zip(checked["batched"], plain["batched"]):
        np.testing.assert_array_equal(np.array(a), np.array(b))


SELFTEST = r'''
import sys
import torch
sys.path.insert(0, ROOT)
import synth
import paper_2110_12065_amd as mp
A = torch.from_numpy(synth.dense_cov(300, 700, seed=3)).cuda()
w0 = torch.from_numpy(synth.start_vector(300, 4)).cuda()
mp.mapi_tuning_set(mp.MAPI_F32, 300, 300, dict(rows_per_wave=1, waves=4, blocks_per_cu=1, unroll=2, w_in_lds=1,
                                                nontemporal=0))
try:
    mp.mapi_solve(A, w0, max_iters=5)
    print("RESULT none", flush=True)
except mp.MapiError as e:
    print("RESULT %d %s" % (e.status, e), flush=True)
'''


def test_failed_device_check_reaches_the_caller(checked_built):
    print("[case] device-checked build: self-test check", flush=True)
    r = _run({"MAPI_CHECKED": "1", "MAPI_DCHECK_SELFTEST": "1"}, SELFTEST)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    assert line.startswith("RESULT 9 ") and "file id 15" in line, line
    # the ordinary build compiles the check out: the same request succeeds
    r = _run({"MAPI_CHECKED": "0", "MAPI_DCHECK_SELFTEST": "1"}, SELFTEST)
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    assert line == "RESULT none", line
