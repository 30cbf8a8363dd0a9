"""The batch runtime (apo_api.cpp) compiled for the host with
AddressSanitizer and UndefinedBehaviorSanitizer against stand-ins for the
HIP calls and the kernel launchers (tests/helpers/batch_host.cpp): batches
of the 512-run batched configuration, its subsets and a mixed batch are
created, tuned over every launch schedule, run and destroyed one after
another in one process; every batched launch's (run, block) table must
name each member's workgroups exactly once, with one kernel shape and
enough LDS per launch, every capture must join its forked streams back,
and nothing may leak."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_14982_amd", "csrc")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def test_batch_runtime_under_sanitizers(tmp_path):
    cxx = _clang()
    if not cxx or not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("no clang++ with the HIP headers")
    flags = ["-x", "c++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g", "-O1", "-Wno-c++20-extensions"]
    objs = []
    for src in (os.path.join(CSRC, "apo_api.cpp"),
                os.path.join(ROOT, "tests", "helpers", "batch_host.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([cxx] + flags + ["-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    exe = str(tmp_path / "batch_host")
    subprocess.run([cxx, "-fsanitize=address,undefined", "-o", exe] + objs, check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok"), r.stdout[-2000:]
    assert "all again: 512 runs, schedule 3" in r.stdout
