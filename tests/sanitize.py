"""Runs the CPU test suite (``-m "not gpu"``) under AddressSanitizer and
UndefinedBehaviorSanitizer.

Builds the oracle, the scene renderer and the host side of the frontend
library with ROCm's clang and both sanitizers (``VIO_SANITIZE=1`` makes each
package load its ``*_san.so`` variant; device code is built as usual), then
runs pytest with clang's sanitizer runtime preloaded into the interpreter.
Leak checking is off (the interpreter itself keeps allocations to exit);
undefined behaviour aborts. Usage, from the repository root::

    python tests/sanitize.py [extra pytest arguments]
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def runtime() -> str:
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/*/libclang_rt.asan*x86_64*.so"))
    libs = [p for p in libs if "preinit" not in p] or sorted(glob.glob(
        "/opt/rocm/llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"))
    if not libs:
        raise SystemExit("clang's AddressSanitizer runtime not found under /opt/rocm/llvm")
    return libs[0]


def main(argv) -> int:
    env = dict(os.environ, VIO_SANITIZE="1")
    # the builds run without the runtime preloaded (the compilers are not instrumented); the package's
    # build script runs on its own (importing the package would load the library being built)
    subprocess.run([sys.executable, "-c", "import oracle, synthgen; synthgen.build(); oracle.build()"], env=env,
                   check=True, cwd=ROOT)
    subprocess.run([sys.executable, os.path.join(ROOT, "paper_2609_30459_amd", "build.py"), "--sanitize"], env=env,
                   check=True, cwd=ROOT)
    env.update(LD_PRELOAD=runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:protect_shadow_gap=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x", "-q",
           "-p", "no:cacheprovider", *argv]
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
