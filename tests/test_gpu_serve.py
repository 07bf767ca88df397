"""GPU serving: requests carved together by the continuous-batching server equal the same
images carved alone (sc_carve) and the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host, log
from paper_2410_21207_amd import api
from paper_2410_21207_amd.serve import GPUExecutor, Server, team_by_work

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


def _teams_for_tests(t):
    """Team slots for the small test requests: 2 to 4 workgroups by width, changing as they shrink."""
    wc = t.w - t.seams_done
    return 1 if wc < 120 else min(4, 2 + wc // 200)


@pytest.mark.parametrize("seams_per_step,step_us,teams", [(1, 0, False), (7, 0, False), (1 << 20, 300, False),
                                                          (3, 0, True), (1 << 20, 300, True)])
def test_served_in_mix_equals_alone(seams_per_step, step_us, teams):
    reqs = _requests(24, seed=seams_per_step % 1000 + step_us + (7 if teams else 0))
    log("serve mix", seams_per_step, step_us, "teams" if teams else "")
    budget = 6 * max(2 * img.nbytes for img, _ in reqs) + 8 * (1 << 20)
    srv = Server(GPUExecutor(16), budget_bytes=budget, max_slots=16, seams_per_step=seams_per_step,
                 step_budget_us=step_us, team_policy=_teams_for_tests if teams else None)
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


def test_team_steps_leave_empty_slots_empty():
    """A team step over the first few slots, then a step over more slots that include emptied ones:
    the block plan of the first step must not have touched any slot's descriptor (the emptied slots
    report -2 and the live ones carve correctly)."""
    from paper_2410_21207_amd.serve import Ticket
    ex = GPUExecutor(12)
    imgs = [synth.blob_image(60 + 7 * i, 150 + 11 * i, 3, seed=300 + i) for i in range(8)]
    tickets = [Ticket(i, im.shape[0], im.shape[1], 3, im.shape[1] - 20, 0.0, dev(im)) for i, im in enumerate(imgs)]
    for i in range(6):
        ex.start(i, tickets[i])
    for i in range(2, 6):  # four slots emptied again
        ex.release(i)
    p = ex.advance(2, 3, 0, [3, 2])  # the plan of this step lies beyond all 12 descriptors
    assert p[0] == 3 and p[1] == 3
    ex.start(7, tickets[7])
    p = ex.advance(8, 1 << 20, 0, [2, 1, 1, 1, 1, 1, 1, 4])
    assert p[2:7] == [-2] * 5 and p[0] == 20 and p[1] == 20 and p[7] == 20
    for i in (0, 1, 7):
        out, seams, costs = ex.result(i)
        a_out, a_seams, a_costs = api.carve(dev(imgs[i]), imgs[i].shape[1] - 20)
        assert np.array_equal(host(out), host(a_out)) and np.array_equal(host(seams), host(a_seams))


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


@pytest.mark.parametrize("xcd", [0, 5])
def test_carve_on_chosen_xcd(xcd):
    img = synth.blob_image(120, 500, 3, seed=23)
    a_out, a_seams, _ = api.carve(dev(img), 430, team=4, variant=7)
    import ctypes
    from paper_2410_21207_amd import _lib
    t = dev(img)
    lib = _lib.load()
    ws = api.workspace(lib.sc_workspace_bytes(120, 500, 3), "cuda")
    seams = torch.empty((70, 120), dtype=torch.int32, device="cuda")
    _lib.call("sc_carve", ctypes.c_void_p(t.data_ptr()), 120, 500, 3, 430, t.stride(0),
              ctypes.c_void_p(seams.data_ptr()), None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), None, api._tune(4, 7, True, xcd=xcd))
    assert api.read_status(ws, 1) == [0]
    assert np.array_equal(host(t[:, :430]), host(a_out)) and np.array_equal(host(seams), host(a_seams))
