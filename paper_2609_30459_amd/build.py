"""Builds the gfx950 frontend library (libvio_frontend.so) with hipcc, in-tree."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libvio_frontend.so")
# host code built with AddressSanitizer and UndefinedBehaviorSanitizer (device code as usual); loaded
# instead of LIB when VIO_SANITIZE=1 (tests/sanitize.py)
LIB_SAN = os.path.join(PKG, "libvio_frontend_san.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# Per-file flags. k_track.hip: LLVM's sinking of common trailing code merges
# the stores that end the two chunk layouts of the two-keypoint level sums into
# one store through a pointer phi, which keeps two floats of the odd-level
# kernels in scratch memory; without it every array stays in registers (the
# one-keypoint kernels' code hardly changes: a few instructions).
FILE_FLAGS = {"k_track.hip": ["-mllvm", "-simplifycfg-sink-common=false"]}

# host-only sanitizer flags: each -fsanitize= right after -Xarch_host
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False) -> str:
    """Compiles every translation unit to an object, then links the shared library (sanitize: the
    host-sanitized variant LIB_SAN, objects in their own folder)."""
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    objdir = os.path.join(PKG, "_build_san" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []),
               *(SAN_HOST_FLAGS if sanitize else []), *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text, flush=True)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"--- {src}\n{text}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(os.path.basename(s) for s, _ in failed))
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    subprocess.run([hipcc, f"--offload-arch={ARCH}", *(SAN_HOST_FLAGS if sanitize else []), "-shared", "-fPIC", "-o",
                    tmp, *objs], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
