"""Compile the HIP sources of the library into liboz.so (gfx950 only), and the
BLAS offload layer (dgemm_ / zgemm_, host code) into liboz_blas.so, which
links liboz.so from its own directory and rocBLAS for the native mode.

Every HIP file is compiled with:
  -ffp-contract=off   FP64 epilogue products and sums rounded separately, as
                      the method's accumulation order prescribes;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions (the kernels do no FP32
                      work; the flag keeps the compiler from forming them).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liboz.so")
BLAS_LIB = os.path.join(HERE, "liboz_blas.so")
BLAS_SOURCE = "oz_blas.cpp"
SOURCES = ["oz_split.hip", "oz_gemm.hip", "oz_check.hip", "oz_api.hip", "oz_batch.hip", "oz_select.hip",
           "oz_mlp.hip", "oz_learn.hip", "oz_lu.hip", "oz_peak.hip"]
HEADERS = ["oz_internal.h", os.path.join("..", "..", "include", "oz.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-function", "-Wno-unknown-warning-option"]


def build(verbose=False, extra_flags=()):
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, *extra_flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if out and (verbose or p.returncode):
            sys.stdout.write(out.decode(errors="replace"))
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed on: " + ", ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_blas(verbose)
    return LIB


def build_blas(verbose=False):
    """liboz_blas.so: the Fortran-ABI dgemm_ / zgemm_ layer over liboz.so."""
    obj = os.path.join(BUILD, BLAS_SOURCE.replace(".cpp", ".o"))
    inc = os.path.join(HERE, "..", "include")
    cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-Wall", "-I" + inc, "-c", os.path.join(CSRC, BLAS_SOURCE), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    cmd = [HIPCC, "-shared", "-fPIC", "-o", BLAS_LIB + ".tmp", obj, "-L" + HERE, "-l:liboz.so", "-lrocblas",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(BLAS_LIB + ".tmp", BLAS_LIB)
    return BLAS_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
