"""Build the CPU oracle shared library (plain gcc, OpenMP).

Test infrastructure: the product library never builds against or loads this.

build(sanitize=True) writes liboz_oracle_san.so instead: the same source with
AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal).  A
process selects it with OZ_ORACLE_LIB=<path> and must preload the ASan
runtime (``asan_runtime()``), as tests/test_oracle_sanitized.py does.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oz_oracle.c")
LIB = os.path.join(HERE, "liboz_oracle.so")
SAN_LIB = os.path.join(HERE, "liboz_oracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def build(verbose=False, sanitize=False):
    out = SAN_LIB if sanitize else LIB
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", *opt, "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-shared", "-fPIC", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def asan_runtime():
    """Path of gcc's ASan runtime library (to preload before the sanitized oracle)."""
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()


if __name__ == "__main__":
    print(build(verbose=True))
