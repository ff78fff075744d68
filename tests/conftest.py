import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


def read_golden(name):
    """Parse a golden file: 'case <ints> | <numbers>' followed by rows of 're im' expressions."""
    import math

    env = {"sqrt": math.sqrt, "__builtins__": {}}
    cases = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("case"):
                head, data = line[4:].split("|")
                cases.append(([int(v) for v in head.split()], [float(v) for v in data.split()], []))
            else:
                re_s, im_s = line.split()
                cases[-1][2].append(complex(eval(re_s, env), eval(im_s, env)))
    return cases


@pytest.fixture
def golden():
    return read_golden
