import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running test")


def load_product():
    """Import the solver package for a GPU test module.  Where a GPU is
    visible a missing or broken libss.so is an error (never a skip); on a
    machine without one the module is skipped at collection."""
    import pytest
    try:
        import paper_1504_06768_amd as ssl
        return ssl
    except Exception:
        import torch
        if torch.cuda.is_available():
            raise
        pytest.skip("no GPU and no loadable libss.so", allow_module_level=True)
