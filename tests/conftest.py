import os
import sys
import warnings

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# scipy.integrate.quad warns about round-off when the requested 1e-14
# relative tolerance sits at the double-precision floor; the results are
# pinned against closed forms in test_oracle_bath.py.
warnings.filterwarnings("ignore", message=".*roundoff error.*")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")
    warnings.filterwarnings("ignore", message=".*roundoff error.*")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
