"""Host <-> device array marshalling for the library's two layouts.

Host arrays are node-major NumPy arrays of shape (N, ...).  NODE_MAJOR keeps
that order on the device; ELEM_MAJOR stores one array per matrix entry,
i.e. the (N, ...) array transposed to (..., N).
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import LAYOUT_ELEM_MAJOR, LAYOUT_NODE_MAJOR


def to_device(a, layout, device="cuda"):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if layout == LAYOUT_ELEM_MAJOR and a.ndim > 1:
        n = a.shape[0]
        a = np.ascontiguousarray(a.reshape(n, -1).T)
    return torch.from_numpy(a.copy()).to(device)


def from_device(t, shape, layout):
    a = t.detach().cpu().numpy()
    if layout == LAYOUT_ELEM_MAJOR and len(shape) > 1:
        n = shape[0]
        a = a.reshape(-1, n).T
    return np.ascontiguousarray(a).reshape(shape)


def empty(shape, device="cuda"):
    return torch.zeros(int(np.prod(shape)), dtype=torch.float64, device=device)


__all__ = ["to_device", "from_device", "empty", "LAYOUT_NODE_MAJOR", "LAYOUT_ELEM_MAJOR"]
