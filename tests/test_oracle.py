"""CPU pins of the oracle (no GPU): hand-worked grids, brute force, closed forms, invariants."""
import numpy as np
import pytest

import oracle
import pins
import synth


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(o, pin):
    pin(o)


def test_bruteforce_up_to_paper_sizes(o):
    """DP == exhaustive search up to 12x12, the largest size the paper runs brute force on."""
    pins.pin_bruteforce_large(o)


def test_config_small_uniform(o):
    """64x48 (W x H) i.i.d. uniform RGB, seed 0, 16 vertical seams; every seam checked
    against every invariant; brute-force cross-check on 6x5 (W x H) crops."""
    img = synth.uniform_image(48, 64, 3, seed=0)
    seams, costs = pins.carve_invariants(o, img, 48)
    assert seams.shape == (16, 48)
    e = o.energy(img)
    rng = np.random.default_rng(0)
    offsets = [(0, 0)] + [(int(rng.integers(0, 48 - 5)), int(rng.integers(0, 64 - 6))) for _ in range(3)]
    for (y0, x0) in offsets:
        # the 6x5 window of the full image's energy map
        win = e[y0:y0 + 5, x0:x0 + 6]
        bs, bc = pins.py_brute_seam(win)
        s, c = o.dp_seam(win)
        assert s.tolist() == bs.tolist() and c == bc
        # the crop as a standalone image, carved 6 -> 1 with brute force on every seam
        crop = np.ascontiguousarray(img[y0:y0 + 5, x0:x0 + 6])
        pins.carve_invariants(o, crop, 1, check_brute=True)


def test_blob_generator_is_deterministic():
    a = synth.blob_image(40, 50, 3, seed=3)
    b = synth.blob_image(40, 50, 3, seed=3)
    assert a.dtype == np.uint8 and a.shape == (40, 50, 3) and np.array_equal(a, b)
    assert not np.array_equal(a, synth.blob_image(40, 50, 3, seed=4))


def test_batch_jobs_recipe():
    jobs = synth.batch_jobs()
    assert len(jobs) == 256
    for j in jobs:
        assert 240 <= j.h <= 2160 and 240 <= j.w <= 2160
        assert 0.10 * j.w - 1 <= j.seams < 0.40 * j.w
    assert jobs == synth.batch_jobs()


def test_serving_requests_recipe():
    reqs = synth.serving_requests(duration=5.0)
    assert 1000 < len(reqs) < 2000
    ts = [r.t for r in reqs]
    assert ts == sorted(ts) and ts[-1] < 5.0
    for r in reqs:
        assert 128 <= r.h <= 4096 and 128 <= r.w <= 4096
        assert 0.5 * r.w - 1 <= r.target_w < 0.9 * r.w
