"""Build libnphase_lbm.so in-tree with hipcc for gfx950.

    python -m paper_2306_06983_amd.build [--only-n N] [-j JOBS]

Compiles the kernel translation units (FP64/FP32 x D2Q9/D3Q19, the D3Q19 ones split by
phase count; the two adjoint units) and the host C-ABI unit in parallel, then links the shared library next to this file.  `--only-n` limits
the instantiated phase counts to one value (faster development builds)."""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnphase_lbm.so")
# the D3Q19 step units are split by phase count: the longest unit sets the build time
SOURCES = ["kernels_f64_d3q19_n5.hip", "kernels_f64_d3q19_n6.hip", "kernels_f64_d3q19_n7.hip",
           "kernels_f64_d3q19_n8.hip", "kernels_f32_d3q19_n7to8.hip",
           "kernels_f32_d3q19_n2to5.hip", "kernels_f64_d3q19_n2to4.hip",
           "kernels_f64_d2q9.hip", "kernels_f32_d2q9.hip", "adjoint_d3q19.hip",
           "kernels_f32_d3q19_n6.hip", "adjoint_d2q9.hip", "nphase_lbm.hip"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed-FP32 instructions in any HIP code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(only_n=None, jobs=None, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    extra = [f"-DNPHASE_ONLY_N={int(only_n)}"] if only_n else []
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--only-n", type=int, default=None)
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args(argv)
    build(a.only_n, a.j)


if __name__ == "__main__":
    sys.exit(main())
