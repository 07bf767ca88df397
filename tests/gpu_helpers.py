"""Shared helpers of the GPU parity tests (host side only; no method arithmetic here)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
import pins


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


def remove_np(cur: np.ndarray, s: np.ndarray) -> np.ndarray:
    H, w, C = cur.shape
    keep = np.ones((H, w), bool)
    keep[np.arange(H), s] = False
    return cur[keep].reshape(H, w - 1, C)


def check_carve_sampled(img: np.ndarray, out: np.ndarray, seams: np.ndarray, costs: np.ndarray, sample):
    """Exact check of a long carve without running the oracle on every seam.

    Every seam is checked for validity (in range, 8-connected) and the final image must be the
    input with the recorded seams deleted in order.  For every seam index in `sample`, the
    image state before that seam is rebuilt by deleting the earlier recorded seams, and the
    oracle's minimum seam and cost of that state must equal the recorded ones.
    """
    cur = img.copy()
    H = img.shape[0]
    sample = set(int(k) for k in sample)
    for k in range(seams.shape[0]):
        s = seams[k]
        pins.check_seam_valid(s, H, cur.shape[1])
        if k in sample:
            e = oracle.energy(cur)
            os_, oc = oracle.dp_seam(e)
            assert np.array_equal(s, os_), f"seam {k} differs from the oracle"
            assert int(costs[k]) == oc, f"cost {k}: {int(costs[k])} != {oc}"
        cur = remove_np(cur, s)
    assert np.array_equal(out, cur), "final image != input with the recorded seams deleted"
