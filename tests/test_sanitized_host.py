"""Host code of the C ABI and the planner (argument checks, plan building, operator packing,
the device-memory cap) under AddressSanitizer and UndefinedBehaviorSanitizer: the library is
rebuilt with both sanitizers on its host pass, and the CPU tests of the ABI run against it in a
child process with the ASan runtime preloaded.  No GPU is needed or used."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_pass_under_asan_and_ubsan():
    from paper_1103_5391_amd import build as B
    lib = B.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=B.asan_runtime(), DMRG_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES="")
    env.pop("DMRG_MAX_WORKSPACE", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in out and "runtime error" not in out
