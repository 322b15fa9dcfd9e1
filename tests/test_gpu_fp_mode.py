"""The forward kernels run in a relaxed floating-point mode (FP32 denormals
flushed, IEEE mode off, no NaN or signed-zero semantics; see SOURCE_FLAGS in
the build).  No value their outputs depend on may be a denormal, a NaN or a
signed zero, so the product build must give the same output planes, bit for
bit, as the strict build of the same sources (libfrt_strict.so, every kernel
in strict IEEE semantics).  The strict build is loaded in a child process."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRICT = os.path.join(ROOT, "paper_2102_01747_amd", "libfrt_strict.so")

# job sets covering every forward variant: the n = 8 Mandelbulb with shadows
# (central and analytic normals), the degree-2 and degree-p Julia batches,
# the real-power sweep frames with a cut plane, the differentiable set
SETS = '''
import workloads as W
sets = {
    "bulb8": W.bulb_views(width=480, height=270),
    "bulb8_analytic": W.bulb_views(n_views=2, width=320, height=180, normal_mode="analytic"),
    "julia": W.julia_batch(n_jobs=16),
    "degree": W.julia_degree_batch(n_jobs=8, sizes=(256,)),
    "sweep": [W.with_size(W.stress_frame(f), 480, 270) for f in (0, 20, 45, 63)],
    "diff": W.diff_set(width=256, height=256)[0],
}
'''

HASH = '''
import hashlib, json, sys, torch
sys.path.insert(0, ROOT)
import paper_2102_01747_amd as frt
out = {}
for name, jobs in sets.items():
    frames = frt.render_batch(jobs, "cuda", counters=True)
    torch.cuda.synchronize()
    h = hashlib.sha256()
    for f in frames:
        for k in ("depth", "normal", "colour", "status", "counters"):
            h.update(f[k].cpu().numpy().tobytes())
    out[name] = h.hexdigest()
print(json.dumps({"lib": frt.LIB_PATH, "hashes": out}))
'''


def _hashes(env, lib):
    code = "ROOT = %r\nimport sys\nsys.path.insert(0, ROOT)\n" % ROOT + SETS + HASH
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-3000:]
    rec = json.loads(res.stdout.strip().splitlines()[-1])
    assert os.path.realpath(rec["lib"]) == os.path.realpath(lib), rec["lib"]
    return rec["hashes"]


def test_relaxed_fp_mode_changes_no_output_bit():
    if not os.path.exists(STRICT):
        pytest.skip("libfrt_strict.so not built")
    env = dict(os.environ)
    env.pop("FRT_LIB_PATH", None)
    product = _hashes(env, os.path.join(ROOT, "paper_2102_01747_amd", "libfrt.so"))
    env["FRT_LIB_PATH"] = STRICT
    strict = _hashes(env, STRICT)
    print(json.dumps({"product": product, "strict": strict}, indent=1))
    assert product == strict
