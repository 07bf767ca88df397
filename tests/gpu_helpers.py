"""Shared helpers of the GPU parity tests (host side only; no method arithmetic here)."""
from __future__ import annotations

import sys

import numpy as np
import torch


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def padded(a: np.ndarray, extra_px: int) -> torch.Tensor:
    """Device copy of an image whose rows carry `extra_px` pixels of padding (pitch > W*C)."""
    H, W, C = a.shape
    t = torch.full((H, W + extra_px, C), 0xAB, dtype=torch.uint8, device="cuda")
    t[:, :W] = dev(a)
    return t[:, :W]


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()
