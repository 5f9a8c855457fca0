"""Helpers for the GPU tests: host <-> device column-major conversion.

A column-major n x s device matrix is a contiguous float64 tensor of shape
(s, n).  Nothing here does any of the method's arithmetic.
"""

import numpy as np


def to_dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(X, dtype=np.float64).T)).to("cuda")


def to_host(T):
    return np.ascontiguousarray(T.detach().cpu().numpy().T)


def kappa_after_projection(N, X):
    """kappa_j = ||X||_2 * ||N^{-1}||_2 (condition of the projected block)."""
    return float(np.linalg.norm(X, 2) * np.linalg.norm(np.linalg.inv(N), 2))
