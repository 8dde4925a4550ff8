"""The C code of the CPU oracle and of the input generators built with
AddressSanitizer and UndefinedBehaviorSanitizer, and the oracle's CPU pins
run against those builds in a child process (ASan runtime preloaded): any
out-of-bounds access, use after free or undefined behaviour (signed
overflow, misaligned or null access, bad shift) aborts the child and fails
this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# pins that exercise every oracle entry point and generator; the exhaustive
# n = 6 part of the sampler pin is left to the plain build (it only repeats
# the smaller cases' code paths)
PINS = ["tests/test_oracle_closed_forms.py", "tests/test_oracle_invariants.py", "tests/test_oracle_bruteforce.py",
        "tests/test_oracle_sampling.py", "tests/test_oracle_scaled_edge.py", "tests/test_oracle_directed.py",
        "tests/test_oracle_weighted.py", "tests/test_oracle_closeness.py", "tests/test_golden.py",
        "tests/test_graphgen.py", "tests/test_oracle_sampler_exact.py"]
DESELECT = ["tests/test_oracle_sampler_exact.py::test_every_labelled_graph_n6"]


def _asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], stdout=subprocess.PIPE, text=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    return out


def test_oracle_pins_under_sanitizers():
    env = dict(os.environ, NK_SANITIZE="1", LD_PRELOAD=_asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    subprocess.check_call([sys.executable, "-c", "import graphgen, oracle; graphgen.build(True); oracle.build(True)"],
                          env=env, cwd=ROOT)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + PINS
    for d in DESELECT:
        cmd += ["--deselect", d]
    res = subprocess.run(cmd, env=env, cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert res.returncode == 0, res.stdout[-4000:]
    assert " passed" in res.stdout and "failed" not in res.stdout
