"""GPU parity of the forward-energy carve against the oracle, bit for bit.

Sizes span several 4-column lane groups and 240-column wave cores, ragged row tails of the
56-row phases, images wider than one workgroup's 968 exact columns (teams of 2 to 9 DP members
exchanging keys at phase ends), tall images with many phases, every channel count, padded
pitches, tie-heavy pixels and the degenerate shapes; the full batched workload is checked on
sampled seams.
"""
import numpy as np
import pytest
import torch

import oracle
import pins
import synth
from gpu_helpers import dev, host, log, padded

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import api  # noqa: E402


def rng_img(seed, H, W, C=3, alpha=256):
    return np.random.default_rng(seed).integers(0, alpha, size=(H, W, C), dtype=np.uint8)


def _check(img, tw, pad=0, in_place=False):
    t = padded(img, pad) if pad else dev(img)
    if in_place:
        out, seams, costs = api.carve_forward(t, tw)
    else:
        dst = padded(np.zeros_like(img), pad) if pad else torch.empty_like(t)
        out, seams, costs = api.carve_forward(dst, tw, src=t)
    o_out, o_seams, o_costs = oracle.carve_forward(img, tw)
    if tw < img.shape[1]:
        assert np.array_equal(host(seams), o_seams), "seams differ"
        assert np.array_equal(host(costs), o_costs), "costs differ"
    assert np.array_equal(host(out), o_out), "carved image differs"


@pytest.mark.parametrize("H,W,C,tw,alpha,pad", [
    (1, 2, 1, 1, 256, 0), (1, 9, 3, 2, 256, 0), (7, 2, 3, 1, 256, 0), (5, 5, 4, 5, 256, 0),
    (61, 97, 3, 40, 256, 0), (121, 300, 1, 150, 4, 3), (130, 257, 4, 100, 256, 0),
    (64, 1030, 2, 1000, 3, 5), (180, 120, 3, 1, 256, 0), (59, 4096, 3, 4090, 256, 0),
])
def test_forward_parity(H, W, C, tw, alpha, pad):
    log("forward", H, W, C, tw, alpha, pad)
    img = synth.blob_image(H, W, 3, seed=H * W) if (C == 3 and alpha == 256) else rng_img(H + W + tw, H, W, C, alpha)
    _check(img, tw, pad)


def test_forward_in_place():
    _check(rng_img(1, 40, 77, 3, 5), 30, in_place=True)


def test_forward_wide_path():
    """W > 4096: teams of five to nine DP members."""
    log("forward wide")
    _check(synth.blob_image(70, 4500, 3, seed=5), 4494)
    _check(rng_img(2, 9, 8192, 1, 3), 8189)


def test_forward_ancestors_in_workspace():
    """A tall image: 54 phases, a team of 14 workgroups."""
    log("forward tall")
    _check(synth.blob_image(3000, 1600, 3, seed=6), 1597)


def test_forward_hand_grids():
    for g in pins.load_golden("forward_grids.json")["grids"]:
        img = np.array(g["image"], np.uint8)
        _, seams, costs = api.carve_forward(dev(img), img.shape[1] - 1)
        assert host(seams)[0].tolist() == g["seam"] and int(host(costs)[0]) == g["cost"], g["name"]


def test_forward_repeatable_and_ws_reuse():
    img = synth.blob_image(150, 333, 3, seed=9)
    src = dev(img)
    ws = api.workspace(1 << 24, "cuda")
    outs = []
    for _ in range(3):
        out, seams, costs = api.carve_forward(torch.empty_like(src), 200, src=src, ws=ws)
        outs.append((host(out), host(seams), host(costs)))
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(outs[0], o))


def _forward_jobs(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        H, W = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        C = [3, 1, 4, 3, 2][i % 5]
        tw = W if i == 3 else max(1, W - int(rng.integers(1, max(2, W // 3))))
        jobs.append((synth.blob_image(H, W, 3, seed=seed * 100 + i) if C == 3 else rng_img(i, H, W, C, 4), tw))
    return jobs


@pytest.mark.parametrize("wide", [False, True])
def test_forward_batch_parity(wide):
    jobs = _forward_jobs(11, 10, 20, 300)
    if wide:  # one image above 4096 columns moves the whole batch to eight columns per thread
        jobs.append((rng_img(3, 12, 4200, 3, 5), 4195))
    srcs = [dev(img) for img, _ in jobs]
    imgs = [torch.empty_like(s) for s in srcs]
    log("forward batch", len(jobs), "wide", wide)
    fb = api.ForwardBatch(imgs, [tw for _, tw in jobs], srcs=srcs)
    for _ in range(2):  # a second launch carves again from src
        fb.launch()
        for (img, tw), (out, seams, costs) in zip(jobs, fb.results()):
            o_out, o_seams, o_costs = oracle.carve_forward(img, tw)
            if tw < img.shape[1]:
                assert np.array_equal(host(seams), o_seams)
                assert np.array_equal(host(costs), o_costs)
            assert np.array_equal(host(out), o_out)


def _check_sampled(img, out, seams, costs, sample):
    """Exact check of a long forward carve: every seam valid, the output equal to the input with
    the recorded seams deleted in order, and the oracle's seam and cost at sampled states."""
    H, W, _ = img.shape
    idx = np.broadcast_to(np.arange(W, dtype=np.int32), (H, W)).copy()
    rows = np.arange(H)[:, None]
    sample = set(sample)
    for k in range(seams.shape[0]):
        s = seams[k]
        pins.check_seam_valid(s, H, idx.shape[1])
        if k in sample:
            cur = img[rows, idx]
            os_, oc = oracle.forward_seam(cur)
            assert np.array_equal(s, os_), f"seam {k} differs from the oracle"
            assert int(costs[k]) == oc, f"cost {k}: {int(costs[k])} != {oc}"
        keep = np.ones(idx.shape, bool)
        keep[np.arange(H), s] = False
        idx = idx[keep].reshape(H, idx.shape[1] - 1)
    assert np.array_equal(out, img[rows, idx]), "output != input with the recorded seams deleted"


def test_forward_batch_full_workload_sampled():
    """The batched workload at full size (256 images, H, W ~ U[240, 2160], 10-40 % of the width
    removed) in the launch the benchmark times: the heaviest image checked exactly on sampled
    seams, the eight lightest against the full oracle carve, every seam of every image valid."""
    jobs = synth.batch_jobs(n=256)
    log("forward full workload: images")
    imgs_np = [j.image() for j in jobs]
    srcs = [dev(a) for a in imgs_np]
    imgs = [torch.empty_like(s) for s in srcs]
    fb = api.ForwardBatch(imgs, [j.target_w for j in jobs], srcs=srcs)
    log("forward full workload: launch")
    fb.launch()
    torch.cuda.synchronize()
    res = fb.results()
    order = sorted(range(len(jobs)), key=lambda i: jobs[i].pixel_seams)
    for i in range(len(jobs)):
        seams = host(res[i][1])
        assert seams.shape == (jobs[i].seams, jobs[i].h)
        assert seams.min() >= 0 and np.all(seams.max(axis=1) < jobs[i].w - np.arange(jobs[i].seams))
        assert np.all(np.abs(np.diff(seams.astype(np.int64), axis=1)) <= 1)
    big = order[-1]
    log("forward full workload: heaviest image", jobs[big])
    k = jobs[big].seams
    _check_sampled(imgs_np[big], host(res[big][0]), host(res[big][1]), host(res[big][2]), [0, 1, k // 2, k - 1])
    for i in order[:8]:
        o_out, o_seams, o_costs = oracle.carve_forward(imgs_np[i], jobs[i].target_w)
        assert np.array_equal(host(res[i][1]), o_seams) and np.array_equal(host(res[i][2]), o_costs)
        assert np.array_equal(host(res[i][0]), o_out)
