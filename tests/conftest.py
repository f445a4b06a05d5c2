import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and libllhmm.so")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", "paper_values.txt")
    for line in open(path):
        if line.startswith(name + " "):
            parts = line.split()
            vals = []
            for p in parts[1:]:
                try:
                    vals.append(float(p))
                except ValueError:
                    break
            return vals
    raise KeyError(name)
