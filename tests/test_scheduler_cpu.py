"""The serving runtime's scheduler on the CPU: runtime.cpp built against a
host-only stand-in of the HIP runtime (tests/cpu_sched: streams are worker
threads, kernels are no-op executors that write a checkable pattern) and
driven by several client threads, plain and under AddressSanitizer +
UndefinedBehaviorSanitizer and ThreadSanitizer.  The harness checks every
request's results, admission under arena and pinned-staging pressure, model
reuse, the pending-queue bound, and destroy with requests outstanding."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = "/opt/rocm/llvm/bin/clang++"
SRC = [os.path.join(ROOT, "paper_2401_04068_amd", "csrc", "runtime.cpp"),
       os.path.join(ROOT, "tests", "cpu_sched", "fake_device.cpp"),
       os.path.join(ROOT, "tests", "cpu_sched", "harness.cpp")]
INC = ["-I" + os.path.join(ROOT, "tests", "cpu_sched", "fake_hip"), "-I" + os.path.join(ROOT, "include"),
       "-I" + os.path.join(ROOT, "paper_2401_04068_amd", "csrc")]

# (name, extra flags, client threads, requests per thread)
VARIANTS = [
    ("plain", [], 4, 60),
    ("asan_ubsan", ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"], 4, 60),
    ("tsan", ["-fsanitize=thread"], 4, 30),
]


@pytest.mark.skipif(not os.path.exists(CXX), reason="needs the ROCm clang++ (host build)")
@pytest.mark.parametrize("name,flags,threads,nreq", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_scheduler_under_sanitizers(tmp_path, name, flags, threads, nreq):
    exe = tmp_path / f"sched_{name}"
    cmd = [CXX, "-std=c++17", "-O1", "-g", *flags, *INC, *SRC, "-lpthread", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    res = subprocess.run([str(exe), str(threads), str(nreq)], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "WARNING" not in res.stderr, res.stderr[-4000:]
    assert "scheduler harness:" in res.stdout
