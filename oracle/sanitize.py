"""Sanitizer build of the oracle (test infrastructure, like the oracle).

Compiles msrep_oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
using ROCm's clang, so that it shares one sanitizer runtime with the
library's sanitizer build, into oracle/liboracle_san.so.  Load it with
ORACLE_LIB pointing at it in a process that preloads that runtime.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "msrep_oracle.c")
SAN_LIB = os.path.join(_HERE, "liboracle_san.so")


def build_sanitized() -> str:
    cc = os.environ.get("SAN_CC", "/opt/rocm/llvm/bin/clang")
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-shared-libasan", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build_sanitized())
