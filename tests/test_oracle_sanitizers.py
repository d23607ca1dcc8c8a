"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the same sources
built with both (any finding aborts), and every oracle pin suite run against that build in
a child process.  CPU only; skipped where g++ or its ASan runtime is missing."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_SUITES = ["tests/test_oracle_pins.py", "tests/test_oracle_apple_pins.py", "tests/test_oracle_extras_pins.py",
              "tests/test_oracle_structure_pins.py", "tests/test_oracle_rebuild_pins.py",
              "tests/test_oracle_adjoint.py"]


def _asan_runtime():
    if shutil.which("g++") is None:
        return None
    path = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_pass_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("g++ with an ASan runtime is not available")
    lib = tmp_path / "liboracle.so"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "oracle.cpp"), "-lpthread"], check=True, timeout=600)
    env = dict(os.environ, ORACLE_LIB=str(lib), LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    # a child with this environment maps the sanitized build, not the regular one
    probe = subprocess.run([sys.executable, "-c", "from oracle import oracle as o; o.lib(); "
                            "print(''.join(l for l in open('/proc/self/maps') if 'liboracle' in l))"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0 and str(lib) in probe.stdout, probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        *PIN_SUITES], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
