import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")

# the first `import torch` on a fresh machine can take a minute: do it at
# collection, outside any per-test time limit
try:
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    pass
