"""Host-code sanitizer run (CPU only): builds libmistencil with AddressSanitizer
and UndefinedBehaviorSanitizer on its host code (argument validation, the
planner, tuning tables, the stencil-program parser and code generator) and
runs the host-side test files against that build.

    python paper_2310_01882_amd/sanitize.py [pytest args...]

Device code is compiled exactly as in build.py: the sanitizer flags reach
the host pass only (-Xarch_host). The library is written to
_build/sanitize/libmistencil.so and selected through MS_LIB_PATH; the
sanitizer runtime is preloaded into the (uninstrumented) Python process.
Any report aborts the run with a non-zero status.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import build as B  # noqa: E402

OUTDIR = os.path.join(HERE, "_build", "sanitize")
LIB = os.path.join(OUTDIR, "libmistencil.so")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-g"]
TESTS = [os.path.join(ROOT, "tests", "test_abi_host.py"),
         os.path.join(ROOT, "tests", "test_jit_host.py"),
         os.path.join(ROOT, "tests", "test_batch_plan_host.py")]


def _compile(src):
    obj = os.path.join(OUTDIR, os.path.basename(src) + ".o")
    cmd = [B.hipcc(), *B.HIPCC_FLAGS, *SAN, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build():
    os.makedirs(OUTDIR, exist_ok=True)
    srcs = B.sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = [B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *SAN, "-shared-libsan",
           *objs, "-lhiprtc", "-o", LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return LIB


def runtime():
    r = subprocess.run([B.hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError(f"AddressSanitizer runtime not found ({path!r})")
    return path


def main(argv):
    lib = build()
    env = dict(os.environ)
    env["MS_LIB_PATH"] = lib
    env["LD_PRELOAD"] = " ".join(p for p in (runtime(), env.get("LD_PRELOAD", "")) if p)
    # the interpreter and torch are not instrumented: their allocations are
    # not leaks of this library; halt on the first report of any kind
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:protect_shadow_gap=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
           *TESTS, *argv]
    print("sanitized library:", lib, flush=True)
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
