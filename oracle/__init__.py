"""Seam-carving oracle: a plain, slow CPU reference of the method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2410_21207_amd``) never imports, links or runs it, and this package
never imports the product.  The two meet only at the seeded input bytes made by
``synth``.

The arithmetic lives in ``sco.c`` (plain C, integer only, each function citing
the passage of arXiv 2410.21207 it follows); this module compiles it with gcc
into ``liboracle.so`` next to the source and wraps it with ctypes for numpy
arrays.  Parity pins: ``tests/test_oracle.py`` (brute force, hand-worked grids,
closed forms, invariants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sco.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_default = None


def compile_source(src_path: str, out_path: str) -> str:
    """Compile one oracle C source into a shared library (gcc -O2, single-threaded)."""
    tmp = out_path + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                           src_path, "-o", tmp])
    os.replace(tmp, out_path)
    return out_path


def build(force: bool = False) -> str:
    """Compile sco.c into liboracle.so next to it (when missing or stale)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _img(img):
    img = np.asarray(img)
    if img.dtype != np.uint8 or img.ndim != 3:
        raise ValueError("image must be uint8 [H, W, C]")
    return np.ascontiguousarray(img)


class Oracle:
    """ctypes view of one compiled oracle library (the default one, or a test variant)."""

    def __init__(self, libpath: str):
        lib = ctypes.CDLL(libpath)
        P, I = ctypes.c_void_p, ctypes.c_int
        sig = {
            "sco_energy": [P, I, I, I, I, P],
            "sco_dp": [P, I, I, P, P, P, P],
            "sco_remove_seam": [P, I, I, I, I, P],
            "sco_carve": [P, I, I, I, I, I, P, P],
            "sco_transpose": [P, I, I, I, I, P, I],
            "sco_carve_hv": [P, I, I, I, I, I, I, P, I, P, P, P, P],
            "sco_seam_origins": [P, I, I, I, P],
            "sco_insert_seams": [P, I, I, I, I, I, P, I, P],
            "sco_greedy_seam": [P, I, I, P, P],
            "sco_brute_seam": [P, I, I, P, P],
            "sco_forward_dp": [P, I, I, I, I, P, P, P, P],
            "sco_carve_forward": [P, I, I, I, I, I, P, P],
            "sco_object_direction": [P, I, I, I],
            "sco_masked_seam": [P, P, I, I, I, I, I, ctypes.c_int32, P, P],
            "sco_remove_object": [P, P, I, I, I, I, I, I, I, P, I, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.sco_mask_bias.argtypes = [I, I]
        lib.sco_mask_bias.restype = ctypes.c_int32
        self.lib = lib

    def energy(self, img) -> np.ndarray:
        """e1 energy of a uint8 [H, W, C] image -> int32 [H, W]."""
        img = _img(img)
        H, W, C = img.shape
        e = np.empty((H, W), np.int32)
        _check(self.lib.sco_energy(_p(img), H, W, C, W * C, _p(e)), "energy")
        return e

    def dp_seam(self, e, full: bool = False):
        """Minimum vertical seam of an int32 [H, W] energy map.

        Returns (seam int32 [H], cost int) or, with ``full``, also the cumulative
        table M (int64 [H, W]) and the direction map D (uint8 [H, W], 0/1/2).
        """
        e = np.ascontiguousarray(np.asarray(e, dtype=np.int32))
        H, W = e.shape
        seam = np.empty(H, np.int32)
        cost = np.zeros(1, np.int64)
        M = np.empty((H, W), np.int64) if full else None
        D = np.empty((H, W), np.uint8) if full else None
        _check(self.lib.sco_dp(_p(e), H, W, _p(M), _p(D), _p(seam), _p(cost)), "dp")
        if full:
            return seam, int(cost[0]), M, D
        return seam, int(cost[0])

    def remove_seam(self, img, seam) -> np.ndarray:
        """Image with one vertical seam removed -> uint8 [H, W-1, C] (a copy)."""
        img = _img(img).copy()
        H, W, C = img.shape
        seam = np.ascontiguousarray(np.asarray(seam, dtype=np.int32))
        _check(self.lib.sco_remove_seam(_p(img), H, W, C, W * C, _p(seam)), "remove_seam")
        return np.ascontiguousarray(img[:, : W - 1])

    def carve(self, img, target_w: int):
        """Remove W-target_w vertical seams -> (image [H,target_w,C], seams [k,H], costs [k])."""
        img = _img(img).copy()
        H, W, C = img.shape
        k = W - target_w
        seams = np.empty((max(k, 0), H), np.int32)
        costs = np.empty(max(k, 0), np.int64)
        _check(self.lib.sco_carve(_p(img), H, W, C, W * C, target_w, _p(seams), _p(costs)), "carve")
        return np.ascontiguousarray(img[:, :target_w]), seams, costs

    def transpose(self, img) -> np.ndarray:
        img = _img(img)
        H, W, C = img.shape
        out = np.empty((W, H, C), np.uint8)
        _check(self.lib.sco_transpose(_p(img), H, W, C, W * C, _p(out), H * C), "transpose")
        return out

    def carve_hv(self, img, target_w: int, target_h: int):
        """Vertical seams to target_w, then horizontal seams (via transpose) to target_h.

        Returns (image [target_h, target_w, C], vseams, vcosts, hseams, hcosts).
        """
        img = _img(img).copy()
        H, W, C = img.shape
        out = np.empty((target_h, target_w, C), np.uint8)
        vs = np.empty((W - target_w, H), np.int32)
        vc = np.empty(W - target_w, np.int64)
        hs = np.empty((H - target_h, target_w), np.int32)
        hc = np.empty(H - target_h, np.int64)
        _check(self.lib.sco_carve_hv(_p(img), H, W, C, W * C, target_w, target_h, _p(out), target_w * C,
                                     _p(vs), _p(vc), _p(hs), _p(hc)), "carve_hv")
        return out, vs, vc, hs, hc

    def seam_origins(self, seams, W: int) -> np.ndarray:
        """Original columns of seams recorded in current coordinates ([k, H] int32)."""
        seams = np.ascontiguousarray(seams, dtype=np.int32)
        k, H = seams.shape
        orig = np.zeros((k, H), dtype=np.int32)
        _check(self.lib.sco_seam_origins(_p(seams), k, H, W, _p(orig)), "seam_origins")
        return orig

    def insert_seams(self, img, k: int):
        """Widen img by k seams: (out [H, W + k, C], original seam columns [k, H])."""
        img = _img(img)
        H, W, C = img.shape
        out = np.zeros((H, W + k, C), dtype=np.uint8)
        orig = np.zeros((max(k, 1), H), dtype=np.int32)
        _check(self.lib.sco_insert_seams(_p(img), H, W, C, W * C, k, _p(out), (W + k) * C, _p(orig)), "insert_seams")
        return out, orig[:k]

    def forward_seam(self, img, full: bool = False):
        """Minimum forward-energy seam of a uint8 [H, W, C] image.

        Returns (seam int32 [H], cost int) or, with ``full``, also the cumulative
        table M (int64 [H, W]) and the direction map D (uint8 [H, W], 0/1/2).
        """
        img = _img(img)
        H, W, C = img.shape
        seam = np.empty(H, np.int32)
        cost = np.zeros(1, np.int64)
        M = np.empty((H, W), np.int64) if full else None
        D = np.empty((H, W), np.uint8) if full else None
        _check(self.lib.sco_forward_dp(_p(img), H, W, C, W * C, _p(M), _p(D), _p(seam), _p(cost)), "forward_dp")
        if full:
            return seam, int(cost[0]), M, D
        return seam, int(cost[0])

    def carve_forward(self, img, target_w: int):
        """Forward-energy carve -> (image [H,target_w,C], seams [k,H], costs [k])."""
        img = _img(img).copy()
        H, W, C = img.shape
        k = W - target_w
        seams = np.empty((max(k, 0), H), np.int32)
        costs = np.empty(max(k, 0), np.int64)
        _check(self.lib.sco_carve_forward(_p(img), H, W, C, W * C, target_w, _p(seams), _p(costs)), "carve_forward")
        return np.ascontiguousarray(img[:, :target_w]), seams, costs

    def mask_bias(self, h: int, C: int) -> int:
        """The bias B subtracted under the mask for an h-row image of C channels (R20)."""
        return int(self.lib.sco_mask_bias(h, C))

    def object_direction(self, mask) -> int:
        """0 (vertical seams) or 1 (horizontal seams) for a uint8 [H, W] mask (R21)."""
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        H, W = mask.shape
        d = self.lib.sco_object_direction(_p(mask), H, W, W)
        _check(0 if d >= 0 else d, "object_direction")
        return int(d)

    def masked_seam(self, img, mask, B: int):
        """Minimum vertical seam of img with B subtracted from the e1 energy under the mask (R20)
        -> (seam int32 [H], cost int)."""
        img = _img(img)
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        H, W, C = img.shape
        assert mask.shape == (H, W)
        seam = np.empty(H, np.int32)
        cost = np.zeros(1, np.int64)
        _check(self.lib.sco_masked_seam(_p(img), _p(mask), H, W, C, W * C, W, int(B), _p(seam), _p(cost)),
               "masked_seam")
        return seam, int(cost[0])

    def remove_object(self, img, mask, direction: int = -1, restore: bool = False):
        """Remove the object under `mask` (R20-R24).

        Returns (out uint8 [oh, ow, C], info dict, seams int32 [k, h], costs int64 [k]); seams are
        in the carved frame (h = H for vertical seams, W for horizontal ones)."""
        img = _img(img)
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        H, W, C = img.shape
        assert mask.shape == (H, W)
        out = np.zeros((H, W, C), np.uint8)
        info = np.zeros(5, np.int32)
        seams = np.zeros(H * W, np.int32)
        costs = np.zeros(max(H, W), np.int64)
        _check(self.lib.sco_remove_object(_p(img), _p(mask), H, W, C, W * C, W, int(direction), int(bool(restore)),
                                          _p(out), W * C, _p(info), _p(seams), _p(costs)), "remove_object")
        d, k, oh, ow, left = (int(v) for v in info)
        h = H if d == 0 else W
        res = np.ascontiguousarray(out.reshape(-1)[: oh * W * C].reshape(oh, W, C)[:, :ow])
        return res, {"direction": d, "k": k, "rows": oh, "cols": ow, "left": left}, \
            seams[: k * h].reshape(k, h), costs[:k]

    def greedy_seam(self, e):
        """Alg. 2 greedy seam of an int32 [H, W] energy map -> (seam, cost)."""
        e = np.ascontiguousarray(np.asarray(e, dtype=np.int32))
        H, W = e.shape
        seam = np.empty(H, np.int32)
        cost = np.zeros(1, np.int64)
        _check(self.lib.sco_greedy_seam(_p(e), H, W, _p(seam), _p(cost)), "greedy_seam")
        return seam, int(cost[0])

    def brute_seam(self, e):
        """Alg. 1 exhaustive seam (tiny maps only) -> (seam, cost)."""
        e = np.ascontiguousarray(np.asarray(e, dtype=np.int32))
        H, W = e.shape
        seam = np.empty(H, np.int32)
        cost = np.zeros(1, np.int64)
        _check(self.lib.sco_brute_seam(_p(e), H, W, _p(seam), _p(cost)), "brute_seam")
        return seam, int(cost[0])


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def energy(img):
    return default().energy(img)


def dp_seam(e, full: bool = False):
    return default().dp_seam(e, full)


def remove_seam(img, seam):
    return default().remove_seam(img, seam)


def carve(img, target_w: int):
    return default().carve(img, target_w)


def transpose(img):
    return default().transpose(img)


def carve_hv(img, target_w: int, target_h: int):
    return default().carve_hv(img, target_w, target_h)


def seam_origins(seams, W: int):
    return default().seam_origins(seams, W)


def insert_seams(img, k: int):
    return default().insert_seams(img, k)


def greedy_seam(e):
    return default().greedy_seam(e)


def mask_bias(h: int, C: int):
    return default().mask_bias(h, C)


def object_direction(mask):
    return default().object_direction(mask)


def masked_seam(img, mask, B: int):
    return default().masked_seam(img, mask, B)


def remove_object(img, mask, direction: int = -1, restore: bool = False):
    return default().remove_object(img, mask, direction, restore)


def brute_seam(e):
    return default().brute_seam(e)


def forward_seam(img, full: bool = False):
    return default().forward_seam(img, full)


def carve_forward(img, target_w: int):
    return default().carve_forward(img, target_w)
