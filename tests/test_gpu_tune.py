"""GPU: the autotuner times real launches, and every candidate shape gives identical results."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import api, tune  # noqa: E402


def test_autotune_batch_candidates_agree(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_cache", None)
    path = str(tmp_path / "cache.json")
    rng = np.random.default_rng(11)
    jobs = []
    for i in range(6):
        H, W = int(rng.integers(20, 300)), int(rng.integers(30, 420))
        jobs.append((synth.blob_image(H, W, 3, seed=500 + i), max(1, W - int(rng.integers(1, W // 3 + 2)))))
    srcs = [dev(img) for img, _ in jobs]
    imgs = [torch.empty_like(s) for s in srcs]
    cands = [(1, 1), (7, 2), (5, 4), (9, 4)]
    log("autotune batch", cands)
    best, timings = tune.autotune_batch(imgs, [tw for _, tw in jobs], srcs=srcs, candidates=cands, reps=1, path=path)
    assert best in cands and set(timings) == set(cands)
    key = tune.key_batch(tune.device_arch(0), [(s.shape[0], s.shape[1]) for s in srcs])
    assert tune.lookup(key, path) == best
    expect = [oracle.carve(img, tw) for img, tw in jobs]
    for v, g in cands:  # every candidate: the oracle's seams, costs and pixels
        bc = api.BatchCarver(imgs, [tw for _, tw in jobs], srcs=srcs, team=g, variant=v)
        bc.launch()
        for (o_out, o_seams, o_costs), (out, seams, costs) in zip(expect, bc.results()):
            assert np.array_equal(host(seams), o_seams) and np.array_equal(host(costs), o_costs)
            assert np.array_equal(host(out), o_out)


def test_autotune_single_records_choice(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_cache", None)
    path = str(tmp_path / "cache.json")
    img = synth.blob_image(70, 300, 3, seed=77)
    src = dev(img)
    best, timings = tune.autotune_single(torch.empty_like(src), 250, src=src, candidates=[(1, 1), (7, 2)], reps=1,
                                         path=path)
    assert tune.lookup(tune.key_single(tune.device_arch(0), 70, 300), path) == best
    monkeypatch.setenv("SC_TUNE_CACHE", path)
    out, seams, costs = api.carve(dev(img), 250)  # takes the recorded shape
    o_out, o_seams, o_costs = oracle.carve(img, 250)
    assert np.array_equal(host(seams), o_seams) and np.array_equal(host(out), o_out)
