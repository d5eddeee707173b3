"""Build libgcpush.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, at -O3, without fast-math, and with
packed FP32 instructions disabled (the compiler would otherwise form
v_pk_* FP32 operations from scalar float code).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgcpush.so")
SOURCES = ["gc_api.cpp", "gc_push.hip", "gc_push_mlp.hip", "gc_kernels.hip", "gc_moments.hip", "gc_order.hip", "gc_mlp.hip", "gc_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-ffp-contract=fast"]
# Matrix-core sources: MFMA results in ordinary VGPRs (the activation code reads
# every accumulator; with AGPR results each read is an extra v_accvgpr_read).
EXTRA = {"gc_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"], "gc_push_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         # The push kernels of every form must give the same bits: multiply-adds
         # are contracted only within one source expression, never across
         # statements, where the choice would follow each kernel's block layout.
         "gc_push.hip": ["-ffp-contract=on"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC] + CFLAGS + EXTRA.get(src, []) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        futs = {ex.submit(_compile, s): s for s in SOURCES}
        objs = []
        for fu in cf.as_completed(futs):
            try:
                objs.append(fu.result())
            except subprocess.CalledProcessError as e:
                sys.stderr.write(e.stdout.decode(errors="replace"))
                raise
    objs.sort()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
