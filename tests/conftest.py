import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def load_golden(name="paper_values.txt"):
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val, _src = [p.strip() for p in line.split("|", 2)]
            vals = [float(v) for v in val.split()]
            out[key] = vals if len(vals) > 1 else vals[0]
    return out


@pytest.fixture(scope="session")
def golden():
    return load_golden()
