"""Build the oracle's shared library (plain C, single-threaded, -O2, no BLAS).

Test infrastructure: see qcqp_oracle.c's header.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qcqp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_from(src_path: str, out_path: str) -> str:
    """Build another copy of the oracle's source (the tests' planted-mistake copies) with the
    flags of build()."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", out_path, src_path, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def build_sanitized(out_path: str) -> str:
    """AddressSanitizer + UndefinedBehaviorSanitizer build of the oracle (host code only), for
    running the CPU pins under the sanitizers; any report aborts the process."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", out_path, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
