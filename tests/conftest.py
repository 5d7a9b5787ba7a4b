import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# The mutation tests run the oracle pins against a planted-mistake copy of the
# oracle package: OBK_ORACLE_PKG names the folder holding that copy.
if os.environ.get("OBK_ORACLE_PKG"):
    sys.path.insert(0, os.environ["OBK_ORACLE_PKG"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library on the device)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def parse_golden(name):
    """Parse a golden text fixture into a list of dict cases (see the files)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    cases, cur = [], None
    with open(path) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(" ")
            if key in ("case", "name"):
                cur = {"name": rest.strip(), "row": []}
                cases.append(cur)
            elif key == "row":
                cur["row"].append([float(t) for t in rest.split()])
            else:
                cur[key] = rest.strip()
    return cases
