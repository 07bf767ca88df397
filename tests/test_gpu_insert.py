"""GPU parity of seam insertion (image enlargement) against the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log, padded

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import _lib, api  # noqa: E402


def rng_img(seed, H, W, C=3, alpha=256):
    return np.random.default_rng(seed).integers(0, alpha, size=(H, W, C), dtype=np.uint8)


def _check(img, k, pad=0, **kw):
    src = padded(img, pad) if pad else dev(img)
    before = host(src).copy()
    out, seams = api.insert_seams(src, k, **kw)
    o_out, o_orig = oracle.insert_seams(img, k)
    assert np.array_equal(host(out), o_out), "widened image differs"
    if k:
        assert np.array_equal(host(seams), o_orig), "original seam columns differ"
    assert np.array_equal(host(src), before), "the source must not be modified"


@pytest.mark.parametrize("H,W,C,k,alpha,pad", [(1, 4, 1, 1, 256, 0), (2, 3, 1, 1, 256, 0), (1, 9, 3, 8, 256, 0),
                                               (37, 120, 3, 40, 256, 0), (61, 333, 1, 150, 4, 3),
                                               (45, 200, 4, 199, 256, 0), (70, 97, 3, 0, 256, 5),
                                               (33, 130, 2, 64, 2, 7)])
def test_insert_parity(H, W, C, k, alpha, pad):
    log("insert", H, W, C, k, alpha, pad)
    img = synth.blob_image(H, W, 3, seed=H * W) if (C == 3 and alpha == 256) else rng_img(H + W + k, H, W, C, alpha)
    _check(img, k, pad)


def test_insert_hand_grids():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "insert_grids.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        img = np.array(c["img"], dtype=np.uint8)
        out, seams = api.insert_seams(dev(img), c["k"])
        assert np.array_equal(host(out), np.array(c["out"], np.uint8)), c["name"]
        assert np.array_equal(host(seams), np.array(c["orig"], np.int32)), c["name"]


@pytest.mark.parametrize("team,variant", [(1, 1), (4, 7), (8, 5)])
def test_insert_launch_shapes(team, variant):
    img = synth.blob_image(150, 400, 3, seed=91)
    _check(img, 120, team=team, variant=variant)


def test_insert_wide_team_path():
    """W > 4096: the seams come from the team carve path."""
    img = synth.blob_image(24, 4200, 3, seed=93)
    _check(img, 30, team=2)


def test_insert_errors():
    img = dev(rng_img(1, 5, 8, 3))
    with pytest.raises(ValueError):
        api.insert_seams(img, 8)  # k must be < W
    out = torch.empty((5, 9, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.ScError):
        lib = _lib.load()
        ws = api.workspace(lib.sc_insert_workspace_bytes(5, 8, 3, 24, 1), "cuda")
        import ctypes
        _lib.call("sc_insert_seams", ctypes.c_void_p(img.data_ptr()), 5, 8, 3, 24, 1,
                  ctypes.c_void_p(img.data_ptr()), 27, None, None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))  # out overlaps img
    del out
