"""Build step of the CPU oracle: gcc, FP64, OpenMP over particles.

No fast-math and no FMA contraction: the oracle evaluates each formula as
written, in IEEE double precision.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


# Instrumented build for the sanitizer run of the CPU tests (host code only):
# AddressSanitizer and UndefinedBehaviorSanitizer, every finding fatal.  The
# Python process must preload the runtimes, e.g.
#   LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)" \
#   ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu"
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def build(force: bool = True, sanitize: bool = False) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "gc_oracle.h"))):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    opt = SANITIZE if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv, sanitize="--sanitize" in sys.argv))
