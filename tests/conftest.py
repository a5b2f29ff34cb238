import os
import sys

# Before numpy loads: the seeded pairs are drawn with one fixed OpenBLAS
# kernel family, so they are bitwise the same on every host.
os.environ.setdefault("OPENBLAS_CORETYPE", "Haswell")

import pytest  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")
