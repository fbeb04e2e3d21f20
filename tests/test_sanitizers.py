"""The host-side code under AddressSanitizer and UndefinedBehaviorSanitizer:
the library's sanitizer build (host code instrumented, device code as usual)
and the oracle's run the CPU tests of the host logic (argument checks, the
serving scheduler, arena and admission through msrep_serve_simulate, struct
layouts) and the oracle's pins in a child process with the sanitizer runtime
preloaded.  A planted out-of-bounds write shows that the instrumentation is
live."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2209_07552_amd import build as hipbuild  # noqa: E402
from paper_2209_07552_amd import sanitize  # noqa: E402
from oracle import sanitize as osan  # noqa: E402

pytestmark = pytest.mark.slow

HOST_TESTS = ["tests/test_serve_sim.py", "tests/test_abi_cpu.py", "tests/test_oracle_partition.py",
              "tests/test_oracle_spmv.py", "tests/test_oracle_convert.py", "tests/test_oracle_spmm.py"]


def _newer(target, sources):
    return os.path.exists(target) and all(os.path.getmtime(target) >= os.path.getmtime(s)
                                          for s in sources)


@pytest.fixture(scope="module")
def san_env():
    if not os.path.exists(hipbuild.HIPCC):
        pytest.skip("hipcc not available")
    try:
        rt = sanitize.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    if not _newer(sanitize.SAN_LIB, sanitize.sources()):
        sanitize.build_sanitized()
    if not _newer(osan.SAN_LIB, [osan.SRC]):
        osan.build_sanitized()
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               MSREP_LIB=sanitize.SAN_LIB, ORACLE_LIB=osan.SAN_LIB)
    return env


def test_host_logic_and_oracle_under_sanitizers(san_env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *HOST_TESTS], cwd=ROOT, env=san_env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    # the child really ran the sanitizer builds
    probe = ("import os, oracle, paper_2209_07552_amd as pk; pk.load_library(); oracle._load(); "
             "maps = open('/proc/self/maps').read(); "
             "print('libmsrep_san.so' in maps, 'liboracle_san.so' in maps, 'asan' in maps)")
    p = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=san_env, capture_output=True,
                       text=True, timeout=120)
    assert p.stdout.split() == ["True", "True", "True"], p.stdout + p.stderr


def test_planted_overflow_is_reported(san_env):
    """The oracle's CSR-to-COO expansion writes ptr[m] entries; given a
    shorter output buffer, the sanitizer must stop the process."""
    code = ("import ctypes, numpy as np, oracle; L = oracle._load(); "
            "ptr = np.array([0, 3, 7], np.int32); out = np.zeros(5, np.int32); "
            "L.oracle_csr_to_coo(2, ptr.ctypes.data, out.ctypes.data)")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=san_env, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0 and "AddressSanitizer" in p.stderr, p.stderr[-2000:]
