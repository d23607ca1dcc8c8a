"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on a
machine without a GPU: model creation validates the description, derives every tree's
parameters in FP64, renumbers, packs and orders the trees on the host before its first
device allocation, which then fails (out of memory: no device).  A build with both
sanitizers on the host pass only (any finding aborts) runs that whole path for several
mappings, variants and tree shapes in a child process.  CPU only; skipped where a GPU is
present or hipcc / clang's ASan runtime is missing."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_06337_amd", "csrc")

CHILD = r'''
import sys
from orchard_inputs import assemble, chain_tree, gen_tree, step_constants
from paper_2607_06337_amd.orchard import load_library
load_library(sys.argv[1])
from paper_2607_06337_amd import Model, OrchardError
assert any(sys.argv[1] in l for l in open("/proc/self/maps"))
trees = [gen_tree(s, n, a) for s, n, a in ((1, 40, 5), (2, 300, 20), (3, 1500, 100), (4, 1, 0), (5, 5000, 60))]
trees.append(chain_tree(300, length=0.1, radius=0.02))
b = assemble(trees)
tunings = [None, dict(threads=256, lds_width=240, steps_per_launch=50),
           dict(threads=128, lds_width=64, wave_width=32, big_threads=256),
           dict(threads=64, lds_width=64, pack_skew=1), dict(threads=512, lds_width=0, persistent=1),
           dict(threads=256, lds_width=240, adjoint_ckpt_max=20, big_threads=512)]
consts = [step_constants(), step_constants(fruit_dof=3, stiffness_k0=50.0, stiffness_gamma=0.7, drag_lin=0.1,
                                           friction_base=0.2, friction_speed=0.5, event_band=1e-3)]
n = 0
for t in tunings:
    for c in consts:
        try:
            Model(b, c, t)
            raise SystemExit("a model was created: a device is present")
        except OrchardError as e:
            assert e.code == 3 and "hipMalloc" in str(e), (t, e)
            n += 1
# rejected descriptions leave through the error paths
bad = assemble([gen_tree(1, 20, 3)])
bad.seg_parent[5] = 7
try:
    Model(bad, step_constants())
    raise SystemExit("an invalid topology was accepted")
except OrchardError as e:
    assert e.code == 2, e
print("host paths:", n)
'''


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_model_construction_host_code_under_sanitizers(tmp_path):
    try:
        import torch
        if torch.cuda.device_count() > 0:   # counts devices without initialising one
            pytest.skip("a GPU is present: model creation would not stop at its first device allocation")
    except ImportError:
        pass
    runtime = _asan_runtime()
    if shutil.which("hipcc") is None or runtime is None:
        pytest.skip("hipcc or clang's ASan runtime is not available")
    lib = tmp_path / "liborchard.so"
    sources = [os.path.join(CSRC, f) for f in ("orchard_api.hip", "orchard_step.hip", "orchard_adjoint.hip",
                                               "orchard_build.hip", "orchard_sphere.hip")]
    subprocess.run(["hipcc", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
                    "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-o", str(lib), *sources],
                   check=True, timeout=900, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD, str(lib)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "host paths: 12" in r.stdout, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
