import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running test")


_TORCH_READY = False


def _torch_gpu_first():
    """Some GPU tests hand torch device tensors to the library.  torch ships
    its own HIP runtime; it comes up reliably only when it initialises the
    device before the library's runtime does, so do that once per session
    (a no-op without a GPU)."""
    global _TORCH_READY
    if _TORCH_READY:
        return
    _TORCH_READY = True
    import torch
    if torch.cuda.is_available():
        torch.zeros(1, device="cuda")
        torch.cuda.synchronize()


def load_product():
    """Import the solver package for a GPU test module.  Where a GPU is
    visible a missing or broken libss.so is an error (never a skip); on a
    machine without one the module is skipped at collection."""
    import pytest
    _torch_gpu_first()
    try:
        import paper_1504_06768_amd as ssl
        return ssl
    except Exception:
        import torch
        if torch.cuda.is_available():
            raise
        pytest.skip("no GPU and no loadable libss.so", allow_module_level=True)
