"""Host C++ of the library under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): the exact solvers of the reduced instance (integer and real
weights) on random instances against brute force, on malformed CSR input,
on instances large enough for the threaded reductions and on one whose
augmenting searches exhaust their budget; and the serving scheduler's
admission policy driven by a mock executor (tests/host/sched_sim.cpp). Both
programs are built with g++ from the library's own sources."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1104_3830_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
FLAGS = ["-std=c++17", "-O1", "-g", "-Wall", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")


def build_and_run(tmp_path, name, sources):
    exe = tmp_path / name
    subprocess.run(["g++", *FLAGS, f"-I{CSRC}", *sources, "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout[-4000:] + out.stderr[-4000:]
    assert out.stdout.strip().startswith("ok"), out.stdout
    return out.stdout


def test_exact_solvers_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "solver_check",
                  [os.path.join(HOST, "solver_check.cpp"), os.path.join(CSRC, "sk_solver.cpp"),
                   os.path.join(CSRC, "sk_solver_real.cpp")])


def test_serving_admission_policy_with_mock_executor(tmp_path):
    out = build_and_run(tmp_path, "sched_sim", [os.path.join(HOST, "sched_sim.cpp")])
    # every branch was taken: refusals, regions at submission, at admission
    fields = dict(kv.split("=") for kv in out.split()[1:])
    assert int(fields["refused"]) > 0 and int(fields["placed_at_submit"]) > 0
