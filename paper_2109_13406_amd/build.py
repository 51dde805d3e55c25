"""Build libmpdd.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_2109_13406_amd.build        # or build() from Python

Every source is compiled by hipcc with:
  --offload-arch=gfx950 -O3          the MI355X target only;
  -ffp-contract=off                  no implicit multiply-add fusion: the dd
                                     error-free transformations rely on each
                                     add and multiply being rounded as written;
  -target-feature -packed-fp32-ops   no packed FP32 instructions are emitted.
Objects go to _build/ (untracked); the library lands next to this file.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build", "mpdd")
LIB = os.path.join(PKG, "libmpdd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["mpdd.cpp", "tuner.cpp", "server.cpp", "host_api.cpp", "gemm_plain.hip", "ozaki.hip",
           "complex.hip", "potrf.hip", "qd.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


# Per-source extra flags.  The plain dd kernels keep their FP64 MFMA
# accumulators (the cross terms) in ordinary VGPRs: with AGPRs the compiler
# copied them out and back every k-tile (64 v_accvgpr moves per 2 100 FP64
# ops), and the register budget (two waves per SIMD) has room for them.
EXTRA_FLAGS = {"gemm_plain.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src):
    out = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA_FLAGS.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, out, r


def build(verbose=False, jobs=None):
    """Compile every HIP / C++ source and link libmpdd.so.  Raises on error."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, out, r in ex.map(_compile, SOURCES):
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
            if verbose and r.stderr.strip():
                sys.stderr.write(r.stderr)
            objs.append(out)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
