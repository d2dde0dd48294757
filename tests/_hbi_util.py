import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2210_02698_amd", "libhbi.so")


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2210_02698_amd import build
        build.build()
    return LIB


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


requires_gpu = pytest.mark.skipif(not gpu_available(), reason="no GPU")
