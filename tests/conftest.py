import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size configuration")


def load_golden(name):
    """Parse a tests/golden/*.txt fixture into {key: [tokens]} plus partition
    records {(fmt, np): {i: (fields, lptr)}}."""
    path = os.path.join(ROOT, "tests", "golden", name)
    kv, parts = {}, {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if "|" in line:
                head, tail = line.split("|")
                t = head.split()
                fmt, np_, i = t[0], int(t[1]), int(t[2])
                fields = [int(v) for v in t[3:]]
                lp = [int(v) for v in tail.split()]
                parts.setdefault((fmt, np_), {})[i] = (fields, lp)
            else:
                t = line.split()
                kv[t[0]] = t[1:]
    return kv, parts


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
