"""GPU parity of object removal with a mask (sc_remove_object) against the oracle: the output
image, the direction, the number of seams, the masked pixels left, every seam and every masked
cost, bit-exact.  Sizes span several 60-row phases and thread column ranges with ragged tails,
both directions, C = 1..4, masks with stray pixels, the restore rounds, frames wider than half the
workgroup's column range, the 8-column-per-thread path (frames wider than 4096) and phase
ancestors spilled from LDS to the workspace."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import _lib, api  # noqa: E402  (a missing library fails these tests)


def _compare(img, mask, direction=-1, restore=False, where=""):
    o_out, o_info, o_seams, o_costs = oracle.remove_object(img, mask, direction, restore)
    g_out, g_info, g_seams, g_costs = api.remove_object(dev(img), dev(mask), direction, restore)
    g_out, g_seams, g_costs = host(g_out), host(g_seams), host(g_costs)
    for key in ("direction", "k", "rows", "cols", "left"):
        assert g_info[key] == o_info[key], f"{where}: {key} {g_info[key]} != {o_info[key]}"
    assert np.array_equal(g_seams, o_seams), f"{where}: seams differ"
    assert np.array_equal(g_costs, o_costs), f"{where}: costs differ"
    assert np.array_equal(g_out, o_out), f"{where}: pixels differ"
    return g_info


CASES = [
    # H, W, C, seed, mask size range, stray pixels
    (37, 45, 3, 1, (0.1, 0.3), 0),
    (61, 130, 3, 2, (0.05, 0.2), 2),
    (130, 61, 1, 3, (0.05, 0.2), 0),
    (121, 257, 2, 4, (0.1, 0.2), 3),
    (250, 300, 4, 5, (0.05, 0.15), 1),
    (301, 199, 3, 6, (0.05, 0.2), 0),
]


@pytest.mark.parametrize("H,W,C,seed,size,stray", CASES)
def test_object_auto_direction(H, W, C, seed, size, stray):
    img = synth.blob_image(H, W, C, seed=seed) if C == 3 else synth.uniform_image(H, W, C, seed=seed)
    mask = synth.object_mask(H, W, seed=100 + seed, size=size, stray=stray)
    info = _compare(img, mask, where=f"{W}x{H}x{C}")
    log("object", W, "x", H, "x", C, "->", info["direction"], info["k"], "seams", f"{info['carve_ms']:.2f} ms")


@pytest.mark.parametrize("H,W,C,seed,size,stray", CASES[:4])
def test_object_forced_direction_and_restore(H, W, C, seed, size, stray):
    img = synth.uniform_image(H, W, C, seed=seed)
    mask = synth.object_mask(H, W, seed=200 + seed, size=size, stray=stray)
    for direction in (_lib.SC_OBJ_VERTICAL, _lib.SC_OBJ_HORIZONTAL):
        _compare(img, mask, direction=direction, restore=True, where=f"{W}x{H}x{C} dir {direction} restore")


def test_object_edge_cases():
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, size=(33, 70, 3), dtype=np.uint8)
    # no mask: nothing removed, the image comes back
    for restore in (False, True):
        info = _compare(img, np.zeros((33, 70), np.uint8), restore=restore, where="empty mask")
        assert info["k"] == 0
    # whole columns masked, more than the rest: the restore needs several insertion rounds
    m = np.zeros((33, 70), np.uint8)
    m[:, 5:45] = 1
    info = _compare(img, m, direction=0, restore=True, where="wide block")
    assert info["k"] >= 40
    # everything masked: the carve stops at one column with pixels left, and cannot be restored
    full = np.ones((33, 70), np.uint8)
    info = _compare(img, full, direction=0, where="full mask")
    assert info["cols"] == 1 and info["left"] == 33
    with pytest.raises(_lib.ScError):
        api.remove_object(dev(img), dev(full), 0, True)
    # one row and one column
    _compare(img[:1], np.ones((1, 70), np.uint8) * (np.arange(70) % 9 == 0), direction=0, where="one row")
    _compare(img[:, :1].copy(), (np.arange(33) % 5 == 0).astype(np.uint8)[:, None].copy(), direction=1,
             where="one column")


def test_object_wide_and_spilled_ancestors():
    # frames wider than 2048 and than 4096 columns (8 columns per thread), and one whose phase
    # ancestors (phases x width bytes) exceed the LDS share and go to the workspace
    img = synth.blob_image(64, 2600, 3, seed=10)
    m = synth.ellipse_mask(64, 2600, 30, 2100, 28, 5)
    _compare(img, m, direction=0, where="2600 wide")
    img = synth.blob_image(70, 4500, 3, seed=8)
    m = synth.ellipse_mask(70, 4500, 35, 3000, 30, 6)
    _compare(img, m, direction=0, where="4500 wide")
    img = synth.blob_image(1250, 900, 3, seed=9)
    m = synth.ellipse_mask(1250, 900, 600, 450, 500, 5)
    _compare(img, m, direction=0, where="1250 rows x 900")


def test_object_rejects_bad_arguments():
    img = dev(synth.uniform_image(20, 30, 3, seed=1))
    with pytest.raises(ValueError):
        api.remove_object(img, dev(np.zeros((20, 29), np.uint8)))
    with pytest.raises(_lib.ScError):
        api.remove_object(img, dev(np.zeros((20, 30), np.uint8)), direction=2)
    # 5483 rows of 3 channels exceed the 23-bit seam energy for vertical seams
    tall = torch.zeros((5483, 4, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.ScError):
        api.remove_object(tall, torch.ones((5483, 4), dtype=torch.uint8, device="cuda"), direction=0)


def test_object_1080p_workload():
    """The measured workload: 1920x1080 blob+noise (seed 1) with an elliptical object of semi-axes
    100 x 200 px at the centre, removed by vertical seams and the size restored."""
    img = synth.blob_image(1080, 1920, 3, seed=1)
    mask = synth.ellipse_mask(1080, 1920, 540, 960, 200, 100)
    info = _compare(img, mask, restore=True, where="1080p object")
    assert info["direction"] == 0 and info["left"] == 0 and info["k"] >= 201
    log("1080p object:", info)
