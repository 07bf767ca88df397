"""GPU serving: requests carved together by the continuous-batching server equal the same
images carved alone (sc_carve) and the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log
from paper_2410_21207_amd import api
from paper_2410_21207_amd.serve import GPUExecutor, Server

pytestmark = pytest.mark.gpu


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = int(rng.integers(30, 300)), int(rng.integers(30, 420))
        img = synth.blob_image(h, w, 3, seed=seed * 1000 + i) if i % 4 else \
            rng.integers(0, 3, size=(h, w, 3), dtype=np.uint8)
        out.append((img, max(1, int(w * rng.uniform(0.5, 0.9)))))
    return out


@pytest.mark.parametrize("seams_per_step", [1, 7])
def test_served_in_mix_equals_alone(seams_per_step):
    reqs = _requests(24, seed=seams_per_step)
    log("serve mix", seams_per_step)
    budget = 6 * max(2 * img.nbytes for img, _ in reqs) + 8 * (1 << 20)
    srv = Server(GPUExecutor(16), budget_bytes=budget, max_slots=16, seams_per_step=seams_per_step)
    ts = [srv.submit(img.shape[0], img.shape[1], 3, tw, dev(img)) for img, tw in reqs]
    while not srv.idle():
        srv.step()
    assert srv.peak_active >= 2
    for i, (t, (img, tw)) in enumerate(zip(ts, reqs)):
        assert t.status == "done", (t.status, t.error)
        out, seams, costs = t.result
        a_out, a_seams, a_costs = api.carve(dev(img), tw)
        assert np.array_equal(host(out), host(a_out)), f"request {i}: pixels differ from the alone carve"
        if a_seams is not None:
            assert np.array_equal(host(seams), host(a_seams)) and np.array_equal(host(costs), host(a_costs))
        if i % 6 == 0:
            assert np.array_equal(host(out), oracle.carve(img, tw)[0])


def test_open_loop_serving_short():
    reqs = synth.serving_requests(rate=200.0, duration=0.5, seed=9, side=(64, 512), canvas_side=512)
    canvases = [dev(synth.blob_image(512, 512, 3, seed=2000 + i)) for i in range(16)]
    srv = Server(GPUExecutor(64), budget_bytes=4 << 30, max_slots=64, seams_per_step=16)
    st = srv.run(reqs, lambda r: canvases[r.canvas][r.y0:r.y0 + r.h, r.x0:r.x0 + r.w].contiguous())
    log(st)
    assert st["done"] == len(reqs) and st["errors"] == 0
    for t, r in list(zip(srv.tickets, reqs))[:10]:
        crop = synth.canvas_crop([host(c) for c in canvases[r.canvas:r.canvas + 1]] * 16, r)
        assert np.array_equal(host(t.result[0]), oracle.carve(crop, r.target_w)[0])
