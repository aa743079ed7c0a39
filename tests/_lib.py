"""Shared helpers of the test suite: locate (and if needed build) libnls."""
import os

import pytest

import paper_2410_24138_amd.nls as nls


def ensure_built():
    if not os.path.exists(nls.LIB_PATH):
        from paper_2410_24138_amd.build import build
        build()
    return nls.load()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


requires_gpu = pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
