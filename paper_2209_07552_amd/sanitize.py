"""Sanitizer build of libmsrep for CPU testing of the host code.

python -m paper_2209_07552_amd.sanitize builds libmsrep_san.so: the same
sources with the *host* code instrumented by AddressSanitizer and
UndefinedBehaviorSanitizer (each -fsanitize= passed to the host compilation
only; the gfx950 device code is built as usual), linked against the shared
sanitizer runtime of ROCm's clang.  Load it in a process that preloads that
runtime, with MSREP_LIB pointing at it (see tests/test_sanitizers.py).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from .build import CSRC, HERE, HIPCC, SOURCES, _compile, _link

SAN_BUILD = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(HERE, "libmsrep_san.so")
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """The shared AddressSanitizer runtime of ROCm's clang (to preload into a
    Python process that loads the sanitizer builds)."""
    out = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    if out and os.path.isabs(out) and os.path.exists(out):
        return out
    cand = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cand:
        raise RuntimeError("no libclang_rt.asan-x86_64.so found")
    return cand[-1]


def build_sanitized(verbose: bool = False) -> str:
    """libmsrep_san.so: host code under ASan + UBSan (shared runtime)."""
    os.makedirs(SAN_BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, SAN_BUILD, SAN_FLAGS), SOURCES))
    _link(objs, SAN_LIB, ["-Xarch_host", "-fsanitize=address", "-Xarch_host",
                          "-fsanitize=undefined", "-shared-libasan"])
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


def sources():
    return glob.glob(os.path.join(CSRC, "*")) + glob.glob(
        os.path.join(os.path.dirname(HERE), "include", "*"))


if __name__ == "__main__":
    build_sanitized(verbose=True)
    sys.exit(0)
