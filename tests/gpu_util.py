"""Helpers for GPU tests: column-major device copies of numpy matrices."""
import numpy as np


def dev(A: np.ndarray):
    """Device buffer holding A column-major (leading dimension = rows)."""
    import torch
    A = np.asarray(A, dtype=np.float64)
    if A.ndim == 1:
        return torch.from_numpy(A.copy()).cuda()
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda()


def host(T, rows, cols):
    """numpy (rows x cols) from a column-major device buffer with leading dimension rows."""
    import torch
    torch.cuda.synchronize()
    return T.detach().cpu().numpy().reshape(-1)[: rows * cols].reshape(cols, rows).T.copy()


def empty(rows, cols):
    import torch
    return torch.zeros(max(rows * cols, 1), dtype=torch.float64, device="cuda")
