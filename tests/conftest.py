import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def _oracle_stale():
    so = os.path.join(ROOT, "oracle", "liblbref.so")
    src = os.path.join(ROOT, "oracle", "lbref.c")
    return (not os.path.exists(so)) or os.path.getmtime(so) < os.path.getmtime(src)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if _oracle_stale():
        oracle.build(force=True)
    yield


def read_golden(name):
    """Parse a golden text fixture: 'key = value  # citation' lines or
    whitespace-separated rows; '#' starts a comment."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line)
    return rows


def golden_values(name):
    out = {}
    for row in read_golden(name):
        k, v = (t.strip() for t in row.split("=", 1))
        out[k] = float(v)
    return out
