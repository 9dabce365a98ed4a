import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture
def golden():
    """Load a whitespace-separated numeric fixture from tests/golden/ ('#' starts a comment)."""

    def load(name):
        rows = []
        with open(os.path.join(GOLDEN, name)) as fh:
            for line in fh:
                line = line.split("#", 1)[0].strip()
                if line:
                    rows.append(tuple(int(t) if t.lstrip("-").isdigit() else float(t) for t in line.split()))
        return rows

    return load
