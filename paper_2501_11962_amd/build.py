"""Build libmop.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2501_11962_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmop.so")
SOURCES = ["kernels_bin.hip", "kernels_pair.hip", "kernels_path.hip", "kernels_pmd.hip", "kernels_bias.hip",
           "kernels_pme.hip", "mop_api.hip"]
ARCH = os.environ.get("MOP_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are switched off (the compiler may otherwise form
# v_pk_fma_f32 / v_pk_mul_f32 / v_pk_add_f32 from scalar float code).
FLAGS = ["-O3", "-fPIC", "-std=c++20", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# Host-side sanitizers: the host half of every source (argument checks, exclusion-key
# numbering, plan geometry and workspace layout, launch set-up) instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer; device code is compiled as usual.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-shared-libasan", "-g"]
SANITIZED_LIB = os.path.join(HERE, "_build", "asan", "libmop.so")


def asan_runtime():
    """Path of the shared AddressSanitizer runtime of hipcc's clang (to LD_PRELOAD into a
    process that loads the sanitized library)."""
    out = subprocess.check_output([os.path.join(os.path.dirname(hipcc()), "amdclang++"),
                                   "-print-file-name=libclang_rt.asan-x86_64.so"]).decode().strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        raise RuntimeError("AddressSanitizer runtime not found")
    return out


def build(verbose=False, jobs=None, sanitize=False):
    """Compile every source and link libmop.so in-tree; with sanitize, the host-sanitized
    variant at _build/asan/libmop.so instead."""
    cc = hipcc()
    bdir = os.path.join(HERE, "_build", "asan") if sanitize else os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    objs = []
    flags = FLAGS + SANITIZE if sanitize else FLAGS
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(bdir, s.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc, *flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0 or (verbose and out):
            sys.stderr.write(out.decode(errors="replace"))
        if p.returncode != 0:
            failed.append(s)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    lib = SANITIZED_LIB if sanitize else LIB
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lrocfft"]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-shared-libasan"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
