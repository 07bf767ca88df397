"""Full-size GPU parity: the batched configuration (256 images, the launch shape the benchmark
times) and the 3840x2160 configuration (960 vertical then 540 horizontal seams), every seam,
every cost and every output pixel compared with the CPU oracle.

The oracle runs one image per host thread (its ctypes calls release the GIL), longest first, so
the whole comparison takes about a minute on 16 host cores.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import api  # noqa: E402  (a missing library fails these tests)


def _cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def test_batch_full_workload_parity():
    """256 blob+noise images, H,W ~ U[240,2160], 10-40 % of the width removed (seed 3), carved in one
    launch with the autotuned shape the benchmark uses (its largest team on the critical image),
    eagerly and by HIP-graph replay; all results bit-exact against the oracle."""
    jobs = synth.batch_jobs(n=256)
    imgs_np = [j.image() for j in jobs]
    srcs = [dev(a) for a in imgs_np]
    dsts = [torch.empty_like(s) for s in srcs]
    bc = api.BatchCarver(dsts, [j.target_w for j in jobs], srcs=srcs)
    log("batch full: variant", api.variants()[bc.info.variant], "team", bc.info.team, "teams used",
        bc.info.teams_used, "tuned", bc.tuned)
    bc.launch()
    eager = [(host(o), host(s), host(c)) for o, s, c in bc.results()]  # results() checks the device status
    bc.capture()
    for im in dsts:
        im.zero_()
    bc.replay()
    torch.cuda.synchronize()
    replay = [(host(o), host(s), host(c)) for o, s, c in bc.results()]
    for i, (a, b) in enumerate(zip(eager, replay)):
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), f"image {i}: graph replay differs from eager"

    order = sorted(range(len(jobs)), key=lambda i: -jobs[i].pixel_seams)
    log("batch full: oracle on", _cores(), "threads")
    with ThreadPoolExecutor(max_workers=_cores()) as ex:
        futs = {i: ex.submit(oracle.carve, imgs_np[i], jobs[i].target_w) for i in order}
        for n, i in enumerate(order):
            o_out, o_seams, o_costs = futs[i].result()
            g_out, g_seams, g_costs = eager[i]
            where = f"image {i} ({jobs[i].w}x{jobs[i].h}, {jobs[i].seams} seams)"
            assert np.array_equal(g_seams, o_seams), f"{where}: seams differ"
            assert np.array_equal(g_costs, o_costs), f"{where}: costs differ"
            assert np.array_equal(g_out, o_out), f"{where}: pixels differ"
            if n % 64 == 0:
                log("batch full: checked", n + 1, "of", len(order))


def test_carve_hv_4k_full():
    """3840x2160 blob+noise RGB (seed 2): 960 vertical seams, then 540 horizontal seams via a
    transpose.  Every seam, cost and pixel of both passes against the oracle.  The horizontal
    pass of the oracle starts from the GPU's intermediate image, which must equal the oracle's
    own, so the two oracle passes run at the same time."""
    img = synth.blob_image(2160, 3840, 3, seed=2)
    log("c3 gpu carve_hv")
    out, vs, vc, hs, hc = api.carve_hv(dev(img), 2880, 1620)
    g_out, g_vs, g_vc, g_hs, g_hc = host(out), host(vs), host(vc), host(hs), host(hc)
    assert g_out.shape == (1620, 2880, 3)
    mid_t, mid_s, _ = api.carve(dev(img), 2880)  # the vertical pass alone: the intermediate image
    g_mid = host(mid_t)
    assert np.array_equal(host(mid_s), g_vs), "the vertical pass is not deterministic"
    log("c3 oracle, both passes")
    with ThreadPoolExecutor(max_workers=2) as ex:
        fv = ex.submit(oracle.carve, img, 2880)
        fh = ex.submit(oracle.carve, np.ascontiguousarray(np.transpose(g_mid, (1, 0, 2))), 1620)
        o_mid, o_vs, o_vc = fv.result()
        o_hout, o_hs, o_hc = fh.result()
    assert np.array_equal(g_vs, o_vs), "vertical seams differ"
    assert np.array_equal(g_vc, o_vc), "vertical costs differ"
    assert np.array_equal(g_mid, o_mid), "intermediate image differs"
    assert np.array_equal(g_hs, o_hs), "horizontal seams differ"
    assert np.array_equal(g_hc, o_hc), "horizontal costs differ"
    assert np.array_equal(g_out, np.transpose(o_hout, (1, 0, 2))), "output pixels differ"
