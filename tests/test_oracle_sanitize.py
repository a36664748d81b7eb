"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

`tests/pins/oracle_sanitize.c` drives every path of the oracle once at the
largest design it accepts (L = OR_MAX_L = 8 coefficients, 8 distinct rows):
slice sweeps through burn-in, the shift step, the exact conjugate draws, the
independence-MH step with a network (and fallback genes), the network's
forward pass and gradients, contrast events, the three-level hooks and
top-level draws, the slice sampler's test targets and every read-out.  It also
checks that or_create rejects L = 9 and more than OR_MAX_ROWS distinct rows of
X, the bounds of the oracle's fixed work arrays.  Any out-of-bounds access,
leak or undefined operation aborts the run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_paths_are_memory_safe(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    src = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "mlp.c"),
           os.path.join(HERE, "pins", "oracle_sanitize.c")]
    cmd = ["gcc", "-std=gnu11", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"), *src, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip(f"sanitizer runtime not available: {r.stderr[-300:]}")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and run.stdout.strip() == "ok", (run.stdout[-2000:], run.stderr[-4000:])
