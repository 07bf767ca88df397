"""GPU parity: every step of the HIP path against the CPU oracle, element by element (bit-exact).

All arithmetic of the method is integer, so the bar is equality of energies, directions,
seams, costs and output bytes.  Inputs are seeded and synthetic (``synth``); the oracle and
the GPU see the same bytes.  Sizes span several DP strips (S = 192 or 416 columns per wave)
and several DP phases (32 or 48 rows) with ragged tails.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log, padded

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import _lib, api  # noqa: E402  (a missing library fails these tests)

VARIANTS = list(range(len(api.variants()))) if torch.cuda.is_available() else []


def rng_img(seed, H, W, C=3, alpha=256):
    rng = np.random.default_rng(seed)
    return rng.integers(0, alpha, size=(H, W, C), dtype=np.uint8)


# ----------------------------------------------------------------------------------------- a1
@pytest.mark.parametrize("H,W,C", [(1, 1, 3), (1, 7, 3), (9, 1, 1), (37, 301, 3), (64, 48, 3), (130, 517, 4),
                                   (200, 1000, 1), (33, 2049, 2)])
def test_energy(H, W, C):
    log("energy", H, W, C)
    img = rng_img(H * 7 + W, H, W, C)
    got = host(api.energy(padded(img, 5)))
    assert np.array_equal(got, oracle.energy(img))


# ----------------------------------------------------------------------------------------- a3-a5
DP_SHAPES = [(1, 1), (1, 9), (7, 1), (2, 2), (32, 192), (33, 193), (64, 384), (31, 191), (100, 700),
             (161, 1000), (47, 416), (49, 833), (250, 130)]


@pytest.mark.parametrize("H,W", DP_SHAPES)
@pytest.mark.parametrize("alpha", [2, 5, 2041])
def test_dp_seam(H, W, alpha):
    log("dp", H, W, alpha)
    rng = np.random.default_rng(H * 1000 + W + alpha)
    e = rng.integers(0, alpha, size=(H, W)).astype(np.int32)
    seam, cost, dirs = api.dp_seam(dev(e), dirs=True)
    os_, oc, _, D = oracle.dp_seam(e, full=True)
    assert np.array_equal(host(dirs)[1:], D[1:]), "direction map differs"
    assert np.array_equal(host(seam), os_)
    assert int(host(cost)[0]) == oc


def test_dp_max_energy_tall():
    """Largest column cost the key format allows: H = 5482 rows of the maximum RGB energy."""
    H, W = 5482, 64
    e = np.full((H, W), 1530, np.int32)
    e[:, 17] = 1529
    seam, cost = api.dp_seam(dev(e))
    os_, oc = oracle.dp_seam(e)
    assert np.array_equal(host(seam), os_) and int(host(cost)[0]) == oc == 1529 * H


# ----------------------------------------------------------------------------------------- a6
@pytest.mark.parametrize("H,W,C", [(1, 1, 3), (5, 2, 3), (40, 333, 3), (17, 1200, 4), (70, 97, 1), (9, 64, 2)])
def test_remove_seam(H, W, C):
    log("remove", H, W, C)
    img = rng_img(H + W, H, W, C)
    rng = np.random.default_rng(W)
    s = [int(rng.integers(0, W))]
    for _ in range(H - 1):
        s.append(int(np.clip(s[-1] + rng.integers(-1, 2), 0, W - 1)))
    s = np.array(s, np.int32)
    t = padded(img, 3)
    api.remove_seam(t, dev(s))
    got = host(t)
    exp = oracle.remove_seam(img, s)
    assert np.array_equal(got[:, : W - 1], exp)
    assert np.array_equal(got[:, W - 1], img[:, W - 1]), "the old last column must stay as it was"


# ----------------------------------------------------------------------------------------- a7
@pytest.mark.parametrize("H,W,C", [(1, 1, 3), (64, 64, 3), (65, 130, 3), (200, 3, 4), (7, 300, 1), (129, 66, 2)])
def test_transpose(H, W, C):
    img = rng_img(H * W, H, W, C)
    got = host(api.transpose(padded(img, 2)))
    assert np.array_equal(got, oracle.transpose(img))


# ----------------------------------------------------------------------------------------- a8
def _carve_and_compare(img, target_w, **kw):
    t = dev(img)
    out, seams, costs = api.carve(t, target_w, **kw)
    o_out, o_seams, o_costs = oracle.carve(img, target_w)
    assert np.array_equal(host(seams), o_seams), "seams differ"
    assert np.array_equal(host(costs), o_costs), "costs differ"
    assert np.array_equal(host(out), o_out), "output pixels differ"


def test_carve_small_uniform_config():
    """64x48 (W x H) i.i.d. uniform RGB, seed 0, 16 vertical seams."""
    img = synth.uniform_image(48, 64, 3, seed=0)
    _carve_and_compare(img, 48)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("team", [1, 2, 3, 8])
def test_carve_variants_and_teams(variant, team):
    log("carve variant", variant, "team", team)
    img = synth.blob_image(130, 500, 3, seed=21)
    _carve_and_compare(img, 440, variant=variant, team=team)


@pytest.mark.parametrize("H,W,C,tw,alpha,team", [(50, 301, 3, 240, 2, 1), (97, 211, 1, 150, 3, 2), (33, 450, 4, 400, 256, 3),
                                                 (1, 50, 3, 10, 256, 1), (40, 2, 3, 1, 256, 1), (65, 193, 3, 1, 4, 4),
                                                 (120, 1030, 3, 900, 3, 8)])
def test_carve_two_columns_per_lane(H, W, C, tw, alpha, team):
    """The variant whose lanes own two columns (their direction bits share a byte with the next
    lane's): tie-heavy and ragged images, widths that end inside a lane pair and inside a strip,
    single workgroups and teams; seams, costs and pixels equal to the oracle's."""
    v = api.variants().index("cpl2_k48_t512")
    log("carve cpl2", H, W, C, tw, alpha, team)
    _carve_and_compare(rng_img(H * W + alpha + 7, H, W, C, alpha), tw, variant=v, team=team)


@pytest.mark.parametrize("H,W,C,tw,alpha", [(50, 300, 3, 250, 2), (97, 211, 1, 150, 3), (33, 450, 4, 400, 256),
                                            (1, 50, 3, 10, 256), (40, 2, 3, 1, 256), (65, 193, 3, 1, 4)])
def test_carve_tie_heavy_and_edges(H, W, C, tw, alpha):
    log("carve edges", H, W, C, tw, alpha)
    _carve_and_compare(rng_img(H * W + alpha, H, W, C, alpha), tw)


@pytest.mark.parametrize("minside", [True, False])
@pytest.mark.parametrize("H,W,C,tw,team", [(61, 333, 3, 250, 1), (45, 260, 1, 100, 2), (70, 419, 4, 300, 4),
                                           (33, 129, 2, 1, 1), (130, 500, 3, 440, 8)])
def test_carve_removal_side(H, W, C, tw, team, minside):
    """Min-side removal (shift the shorter side of each row, rows re-based at the end) and
    right-side removal give the oracle's result; row padding beyond W is never written."""
    log("carve removal side", H, W, C, tw, team, minside)
    img = synth.blob_image(H, W, C, seed=H + W) if C == 3 else rng_img(H * W, H, W, C, 8)
    t = padded(img, 5)
    out, seams, costs = api.carve(t, tw, team=team, minside=minside)
    o_out, o_seams, o_costs = oracle.carve(img, tw)
    assert np.array_equal(host(seams), o_seams) and np.array_equal(host(costs), o_costs)
    assert np.array_equal(host(out), o_out)
    full = host(t.as_strided((H, W + 5, C), t.stride()))
    assert (full[:, W:] == 0xAB).all(), "padding written"


def test_carve_wider_than_lds_row():
    """W > 4096: the phase exchange row no longer fits LDS, so even one workgroup uses the team path."""
    img = synth.blob_image(40, 4500, 3, seed=31)
    _carve_and_compare(img, 4470, team=1)


def test_carve_hv_small():
    img = synth.blob_image(90, 160, 3, seed=33)
    out, vs, vc, hs, hc = api.carve_hv(dev(img), 120, 70)
    o_out, o_vs, o_vc, o_hs, o_hc = oracle.carve_hv(img, 120, 70)
    assert np.array_equal(host(vs), o_vs) and np.array_equal(host(vc), o_vc)
    assert np.array_equal(host(hs), o_hs) and np.array_equal(host(hc), o_hc)
    assert np.array_equal(host(out), o_out)


def test_carve_identity_and_src_pitch():
    img = synth.blob_image(70, 260, 3, seed=5)
    t = padded(img, 7)
    out, seams, costs = api.carve(t, 260)
    assert seams is None and np.array_equal(host(out), img)
    src = padded(img, 7)
    dst = padded(np.zeros_like(img), 7)
    ws = api.workspace(_lib.load().sc_workspace_bytes(70, 260, 3), "cuda")
    out, seams, costs = api.carve(dst, 200, src=src, ws=ws)
    o_out, o_seams, o_costs = oracle.carve(img, 200)
    assert np.array_equal(host(out), o_out) and np.array_equal(host(seams), o_seams)
    assert np.array_equal(host(src), img), "src must not be modified"
    assert api.read_status(ws, 1) == [0]


def test_carve_repeatable():
    img = synth.blob_image(120, 600, 3, seed=6)
    outs = []
    for _ in range(3):
        out, seams, costs = api.carve(dev(img), 500)
        outs.append((host(out), host(seams), host(costs)))
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(outs[0], o))


def test_carve_full_1080p():
    """1920x1080 blob+noise RGB, 480 vertical seams (to 1440 wide): full oracle parity."""
    img = synth.blob_image(1080, 1920, 3, seed=1)
    log("c2 gpu carve")
    t = dev(img)
    out, seams, costs = api.carve(t, 1440)
    g_out, g_seams, g_costs = host(out), host(seams), host(costs)
    log("c2 oracle carve")
    o_out, o_seams, o_costs = oracle.carve(img, 1440)
    assert np.array_equal(g_seams, o_seams)
    assert np.array_equal(g_costs, o_costs)
    assert np.array_equal(g_out, o_out)


# ----------------------------------------------------------------------------------------- batch
def _batch_jobs(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        H, W = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        tw = max(1, W - int(rng.integers(1, max(2, W // 3))))
        jobs.append((synth.blob_image(H, W, 3, seed=seed * 100 + i) if i % 3 else rng_img(i, H, W, 3, 4), tw))
    return jobs


@pytest.mark.parametrize("minside", [True, False])
@pytest.mark.parametrize("team", [1, 2, 4])
def test_batch_parity(team, minside):
    jobs = _batch_jobs(7, 14, 20, 420)
    srcs = [dev(img) for img, _ in jobs]
    imgs = [torch.empty_like(s) for s in srcs]
    log("batch team", team, "minside", minside)
    bc = api.BatchCarver(imgs, [tw for _, tw in jobs], srcs=srcs, team=team, minside=minside)
    bc.launch()
    res = bc.results()
    for (img, tw), (out, seams, costs) in zip(jobs, res):
        o_out, o_seams, o_costs = oracle.carve(img, tw)
        assert np.array_equal(host(seams), o_seams)
        assert np.array_equal(host(costs), o_costs)
        assert np.array_equal(host(out), o_out)
    assert bc.status() == [0] * len(jobs)


def test_batch_graph_replay_matches_eager():
    jobs = _batch_jobs(8, 9, 30, 300)
    srcs = [dev(img) for img, _ in jobs]
    imgs = [torch.empty_like(s) for s in srcs]
    bc = api.BatchCarver(imgs, [tw for _, tw in jobs], srcs=srcs)
    bc.launch()
    eager = [(host(o), host(s), host(c)) for o, s, c in bc.results()]
    bc.capture()
    for rep in range(3):
        for im in imgs:
            im.zero_()
        bc.replay()
        torch.cuda.synchronize()
        got = [(host(o), host(s), host(c)) for o, s, c in bc.results()]
        for a, b in zip(eager, got):
            assert all(np.array_equal(x, y) for x, y in zip(a, b)), f"replay {rep} differs"


def test_batch_alone_vs_in_mix():
    """Each image's result is the same carved alone (sc_carve) and inside a batch."""
    jobs = _batch_jobs(9, 6, 40, 260)
    srcs = [dev(img) for img, _ in jobs]
    imgs = [torch.empty_like(s) for s in srcs]
    bc = api.BatchCarver(imgs, [tw for _, tw in jobs], srcs=srcs)
    bc.launch()
    for (img, tw), (out, seams, costs) in zip(jobs, bc.results()):
        a_out, a_seams, a_costs = api.carve(dev(img), tw)
        assert np.array_equal(host(out), host(a_out)) and np.array_equal(host(seams), host(a_seams))


def test_abi_errors_on_device():
    img = dev(rng_img(0, 10, 10))
    with pytest.raises(_lib.ScError):
        api.carve(img, 0)
    with pytest.raises(_lib.ScError):
        api.carve(img, 11)
