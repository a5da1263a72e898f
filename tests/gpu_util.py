"""Helpers shared by the GPU tests (no solver arithmetic)."""
import numpy as np


def need_torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def unpack(flat, offsets, rows, cols):
    """Split a packed buffer into per-element (rows_k x cols_k) column-major arrays (as N x m)."""
    out = []
    for k in range(len(rows)):
        seg = flat[offsets[k]:offsets[k + 1]]
        out.append(seg.reshape(cols[k], rows[k]).T)
    return out
