"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is the reference every GPU result is checked against, so its own
memory and arithmetic must be sound: out-of-bounds accesses, leaks, integer
overflow in index arithmetic and other undefined behaviour would make its
answers unreliable without failing its pins.  The test program
(tests/oracle_sanitize_driver.c) calls every entry point on small inputs:
each line length class of the transform, both start rules, linear and
nonlinear runs with and without the 2/3 truncation, a blow-up, the complex
field, the per-mode first step and rejected arguments.  Any sanitizer report
aborts the run.  Host code only; no GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "kg_oracle.c"),
       os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")]


def build(tmp_path, sanitizers):
    exe = str(tmp_path / f"driver_{sanitizers.replace(',', '_')}")
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           f"-fsanitize={sanitizers}", "-fno-sanitize-recover=all", *SRC, "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in r.stderr:
        pytest.skip(f"sanitizer runtime not installed: {r.stderr.strip()[:200]}")
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
@pytest.mark.parametrize("sanitizers", ["address,undefined"])
def test_oracle_is_clean_under_sanitizers(tmp_path, sanitizers):
    exe = build(tmp_path, sanitizers)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "all checks passed" in r.stdout
