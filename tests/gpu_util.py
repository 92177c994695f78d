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


def _as_arrays(a, b):
    """Both as float64, or both as complex128 if either is complex (so that
    imaginary parts are compared too)."""
    a, b = np.asarray(a), np.asarray(b)
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    return a.astype(dt), b.astype(dt)


def rel_err(a, b):
    """Relative L2 error ||a - b|| / ||b|| (real or complex)."""
    a, b = _as_arrays(a, b)
    nb = np.linalg.norm(b.ravel())
    if nb == 0.0:
        return float(np.linalg.norm(a.ravel()))
    return float(np.linalg.norm((a - b).ravel()) / nb)


def max_err(a, b):
    """Element-wise max |a - b| / max |b| (real or complex)."""
    a, b = _as_arrays(a, b)
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    md = float(np.max(np.abs(a - b))) if a.size else 0.0
    return md if mb == 0.0 else md / mb
