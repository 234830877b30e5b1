"""Helpers for the GPU parity tests: move column-major numpy arrays to the
device and back."""
from __future__ import annotations

import numpy as np
import torch


def dev(a: np.ndarray) -> torch.Tensor:
    """Column-major device copy of a 2-D (or 1-D) numpy array."""
    t = torch.from_numpy(np.array(a, order="F", copy=True))
    t = t.to("cuda:0")
    if t.dim() == 2 and t.stride(0) != 1:
        t = t.mT.contiguous().mT
    return t


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def log(msg: str) -> None:
    print(msg, flush=True)
