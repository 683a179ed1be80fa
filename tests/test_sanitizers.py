"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
a driver exercises every entry point, ragged block lengths, the threaded
batch driver and the error conventions; the sanitized run must be clean and
print the same numbers as an unsanitized build of the same driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "hmm_oracle.c")]


def _build_and_run(tmp_path, name, flags):
    exe = str(tmp_path / name)
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", *flags, "-o", exe, *SRC,
                    "-lm", "-lpthread"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    plain = _build_and_run(tmp_path, "plain", [])
    assert plain.returncode == 0, plain.stderr
    san = _build_and_run(tmp_path, "san", ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                           "-fno-sanitize-recover=undefined"])
    assert san.returncode == 0, san.stderr[-4000:]
    assert "runtime error" not in san.stderr and "AddressSanitizer" not in san.stderr, san.stderr[-4000:]
    assert san.stdout == plain.stdout
    lines = dict(l.split(" ", 1) for l in plain.stdout.splitlines() if not l.startswith("blocked"))
    assert lines["empty"].strip() == "0"          # ln(sum delta) with sum delta = 1
    assert lines["invalid"].strip() == "nan"
