"""Helpers for the GPU tests (device check, window extraction on the device)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_10292_amd import gs
    gs.load()  # raises if libgs.so is missing: no fallback
    return torch


def window_from_device(t, x0, y0, z0, w):
    """w^3 periodic window of a (nz, ny, nx) CUDA tensor, as float64 numpy."""
    import torch
    nz, ny, nx = t.shape
    dev = t.device
    zi = (torch.arange(w, device=dev) + z0) % nz
    yi = (torch.arange(w, device=dev) + y0) % ny
    xi = (torch.arange(w, device=dev) + x0) % nx
    sub = t.index_select(0, zi).index_select(1, yi).index_select(2, xi)
    return sub.double().cpu().numpy()


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
