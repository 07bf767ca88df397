"""Seeded synthetic inputs for seam carving.

This module only makes input bytes and job lists; it holds none of the
method's arithmetic.  Both the oracle and the HIP path consume what it makes,
so parity never depends on its floating-point internals: both sides always see
the same stored uint8 bytes.

The paper measures on one AI-generated square image and one photograph, neither
of which is available; the distributions below stand in for them:

* ``uniform_image``: i.i.d. uniform bytes (the correctness configuration).
* ``blob_image``: a smooth field of 32 Gaussian blobs plus small integer noise,
  i.e. large low-energy regions broken by soft edges, like a photograph.
* ``batch_jobs``: many blob images of uneven size, each removing 10-40 % of its
  width (the batched configuration).
* ``serving_requests``: Poisson arrivals of blob images with log-uniform sides
  (the serving configuration).
* ``object_mask``: a filled axis-aligned ellipse (the object of the object-removal
  application), optionally with a few stray pixels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["uniform_image", "blob_image", "batch_jobs", "serving_requests", "Job", "Request",
           "canvas_crop", "object_mask", "ellipse_mask"]


def uniform_image(h: int, w: int, c: int = 3, seed: int = 0) -> np.ndarray:
    """i.i.d. uniform uint8 pixels in 0..255, shape [h, w, c]."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(h, w, c), dtype=np.uint8)


def blob_image(h: int, w: int, c: int = 3, seed: int = 1, n_blobs: int = 32,
               sigma=(20.0, 200.0), amp: float = 96.0, noise: int = 8, base: float = 128.0) -> np.ndarray:
    """Sum of ``n_blobs`` Gaussian blobs plus uniform integer noise, uint8 [h, w, c].

    Recipe (float64, ``np.random.default_rng(seed)``, draws in this order):
      centres cx ~ U[0, w), cy ~ U[0, h); sigma ~ U[sigma0, sigma1] px;
      per-blob, per-channel amplitude ~ U[-amp, amp];
      value = base + sum_b a_bc * exp(-((x-cx_b)^2 + (y-cy_b)^2) / (2 sigma_b^2));
      noise ~ U{-noise..noise} per pixel and channel, added;
      rounded half away from zero, clipped to 0..255.
    Each blob is separable, so the sum is one (h x B) @ (B x w) product per channel.
    """
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, w, n_blobs)
    cy = rng.uniform(0.0, h, n_blobs)
    sg = rng.uniform(sigma[0], sigma[1], n_blobs)
    a = rng.uniform(-amp, amp, (n_blobs, c))
    xs = np.arange(w, dtype=np.float64)
    ys = np.arange(h, dtype=np.float64)
    gx = np.exp(-((xs[None, :] - cx[:, None]) ** 2) / (2.0 * sg[:, None] ** 2))  # [B, w]
    gy = np.exp(-((ys[None, :] - cy[:, None]) ** 2) / (2.0 * sg[:, None] ** 2))  # [B, h]
    out = np.empty((h, w, c), np.uint8)
    nz = rng.integers(-noise, noise + 1, size=(h, w, c), dtype=np.int16)
    for ch in range(c):
        v = base + gy.T @ (a[:, ch, None] * gx)  # [h, w]
        v += nz[:, :, ch]
        v = np.sign(v) * np.floor(np.abs(v) + 0.5)
        np.clip(v, 0, 255, out=v)
        out[:, :, ch] = v.astype(np.uint8)
    return out


@dataclass(frozen=True)
class Job:
    """One image of a batch: shape, target width and the seed of its pixels."""
    h: int
    w: int
    target_w: int
    seed: int

    @property
    def seams(self) -> int:
        return self.w - self.target_w

    @property
    def pixel_seams(self) -> int:
        """Sum over removed seams of the pixels of the image the seam was found in."""
        k = self.seams
        return self.h * (k * self.w - k * (k - 1) // 2)

    def image(self, c: int = 3) -> np.ndarray:
        return blob_image(self.h, self.w, c, seed=self.seed)


def batch_jobs(n: int = 256, seed: int = 3, side=(240, 2160), frac=(0.10, 0.40)) -> list[Job]:
    """Batched workload: H, W ~ U{side0..side1} independently; k = floor(r*W), r ~ U[frac0, frac1)."""
    rng = np.random.default_rng(seed)
    hs = rng.integers(side[0], side[1] + 1, n)
    ws = rng.integers(side[0], side[1] + 1, n)
    rs = rng.uniform(frac[0], frac[1], n)
    seeds = rng.integers(0, 2**31 - 1, n)
    jobs = []
    for h, w, r, s in zip(hs, ws, rs, seeds):
        k = int(math.floor(r * int(w)))
        jobs.append(Job(int(h), int(w), int(w) - k, int(s)))
    return jobs


@dataclass(frozen=True)
class Request:
    """One served carve request: arrival time (s), shape, target width, crop of a canvas."""
    t: float
    h: int
    w: int
    target_w: int
    canvas: int
    y0: int
    x0: int

    @property
    def pixel_seams(self) -> int:
        k = self.w - self.target_w
        return self.h * (k * self.w - k * (k - 1) // 2)


def serving_requests(rate: float = 300.0, duration: float = 60.0, seed: int = 4, side=(128, 4096),
                     keep=(0.5, 0.9), n_canvases: int = 16, canvas_side: int = 4096) -> list[Request]:
    """Poisson arrivals; sides log-uniform in [side0, side1]; target_w = floor(u*W), u ~ U[keep0, keep1).

    Pixels are crops of ``n_canvases`` blob canvases of canvas_side^2 (see ``canvas_crop``).
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    lo, hi = math.log(side[0]), math.log(side[1])
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        h = int(round(math.exp(rng.uniform(lo, hi))))
        w = int(round(math.exp(rng.uniform(lo, hi))))
        h = min(max(h, side[0]), side[1])
        w = min(max(w, side[0]), side[1])
        u = rng.uniform(keep[0], keep[1])
        tw = max(1, int(math.floor(u * w)))
        cv = int(rng.integers(0, n_canvases))
        y0 = int(rng.integers(0, canvas_side - h + 1))
        x0 = int(rng.integers(0, canvas_side - w + 1))
        out.append(Request(t, h, w, tw, cv, y0, x0))
    return out


def canvas_crop(canvases, req: Request) -> np.ndarray:
    """Pixels of a request: a crop of one of the pre-generated canvases."""
    return np.ascontiguousarray(canvases[req.canvas][req.y0:req.y0 + req.h, req.x0:req.x0 + req.w])


def resized(img: np.ndarray, n: int, m: int | None = None) -> np.ndarray:
    """Nearest-neighbour resampling of an image to n rows and m (default n) columns: the
    different-sized versions of one image used by the size sweep."""
    m = n if m is None else m
    H, W = img.shape[:2]
    ys = (np.arange(n) * H) // n
    xs = (np.arange(m) * W) // m
    return np.ascontiguousarray(img[ys][:, xs])


def ellipse_mask(h: int, w: int, cy: float, cx: float, ry: float, rx: float) -> np.ndarray:
    """uint8 [h, w] mask, 1 inside the axis-aligned ellipse ((y-cy)/ry)^2 + ((x-cx)/rx)^2 <= 1."""
    y = (np.arange(h, dtype=np.float64)[:, None] - cy) / max(ry, 1e-9)
    x = (np.arange(w, dtype=np.float64)[None, :] - cx) / max(rx, 1e-9)
    return ((y * y + x * x) <= 1.0).astype(np.uint8)


def object_mask(h: int, w: int, seed: int, size=(0.05, 0.25), stray: int = 0) -> np.ndarray:
    """A seeded object: a filled ellipse with semi-axes uniform in size * (h, w), centred uniformly
    where it fits, plus `stray` isolated masked pixels anywhere (values 1..255)."""
    rng = np.random.default_rng(seed)
    ry = max(0.5, rng.uniform(*size) * h)
    rx = max(0.5, rng.uniform(*size) * w)
    cy = rng.uniform(min(ry, h / 2), max(h - ry, h / 2))
    cx = rng.uniform(min(rx, w / 2), max(w - rx, w / 2))
    m = ellipse_mask(h, w, cy, cx, ry, rx)
    for _ in range(stray):
        m[int(rng.integers(0, h)), int(rng.integers(0, w))] = int(rng.integers(1, 256))
    return m
