"""Helpers shared by the GPU tests (no method arithmetic here)."""
import os
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_10657_amd import hfe
    if not os.path.exists(hfe.LIB_PATH):
        raise RuntimeError("libhfe.so is not built: the GPU path has no fallback")
    return torch


def announce(*parts):
    """Print what names the case before a GPU step (flushed)."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    if nb == 0.0:
        return float(np.linalg.norm(a.ravel()))
    return float(np.linalg.norm((a - b).ravel()) / nb)
