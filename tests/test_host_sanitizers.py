"""The host half of the library (argument checks, exclusion-key numbering, error paths)
run under AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: the C-ABI tests of
test_abi.py against a build whose host code is instrumented (build.py --sanitize; device
code is compiled as usual), in a child process with the sanitizer runtime preloaded.  Any
sanitizer report aborts the child, which fails this test."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_pass_under_address_and_ub_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2501_11962_amd import build as B
    lib = B.SANITIZED_LIB
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + \
        [os.path.join(B.CSRC, h) for h in os.listdir(B.CSRC) if h.endswith(".h")] + \
        [os.path.join(ROOT, "include", "mop.h")]
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(s) for s in srcs):
        B.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=B.asan_runtime(), MOP_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
