"""CPU tests of the serving scheduler: admission by budget and slots, FIFO order, continuous
batching, failure isolation, latency statistics.  The executor here is a fake that carves with
the oracle step by step (test infrastructure only); the real one drives the HIP library."""
import numpy as np
import pytest

import oracle
import synth
from paper_2410_21207_amd.serve import Server, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class OracleExecutor:
    """Carves each slot's image `seams_per_step` seams at a time with the oracle."""

    def __init__(self, clock, step_seconds=0.01, fail_start=(), fail_device=()):
        self.clock, self.dt = clock, step_seconds
        self.slots = {}
        self.fail_start, self.fail_device = set(fail_start), set(fail_device)
        self.advance_calls = []

    def state_bytes(self, h, w, c, target_w):
        return 2 * h * w * c

    def start(self, slot, t):
        if t.id in self.fail_start:
            raise RuntimeError("injected allocation failure")
        self.slots[slot] = {"t": t, "img": np.array(t.payload), "seams": [], "costs": []}

    def advance(self, n, max_seams):
        self.advance_calls.append(sorted(self.slots))
        prog = [-2] * n
        for slot, st in self.slots.items():
            t = st["t"]
            if t.id in self.fail_device:
                prog[slot] = -1
                continue
            w = st["img"].shape[1]
            tw = max(t.target_w, w - max_seams)
            out, s, c = oracle.carve(st["img"], tw)
            st["img"] = out
            st["seams"] += list(s)
            st["costs"] += list(c)
            prog[slot] = len(st["seams"])
        self.clock.t += self.dt
        return prog

    def result(self, slot):
        st = self.slots[slot]
        return st["img"], np.array(st["seams"]), np.array(st["costs"])

    def release(self, slot):
        del self.slots[slot]


def make_reqs(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = int(rng.integers(8, 24)), int(rng.integers(10, 40))
        img = synth.blob_image(h, w, 3, seed=100 + i, sigma=(2.0, 8.0))
        out.append((img, int(rng.integers(max(1, w // 2), w))))
    return out


def drain(srv):
    while not srv.idle():
        srv.step()


def test_results_equal_one_shot_carve():
    clk = FakeClock()
    srv = Server(OracleExecutor(clk), budget_bytes=1 << 30, max_slots=4, seams_per_step=3, clock=clk)
    reqs = make_reqs(6)
    ts = [srv.submit(img.shape[0], img.shape[1], 3, tw, img) for img, tw in reqs]
    drain(srv)
    for t, (img, tw) in zip(ts, reqs):
        assert t.status == "done"
        o_out, o_s, o_c = oracle.carve(img, tw)
        out, s, c = t.result
        assert np.array_equal(out, o_out) and np.array_equal(s, o_s) and np.array_equal(c, o_c)


def test_budget_and_slots_bound_admission_and_fifo_order():
    clk = FakeClock()
    ex = OracleExecutor(clk)
    reqs = make_reqs(8, seed=1)
    # budget for about two requests at a time
    budget = 2 * max(2 * img.shape[0] * img.shape[1] * 3 for img, _ in reqs)
    srv = Server(ex, budget_bytes=budget, max_slots=3, seams_per_step=2, clock=clk)
    ts = [srv.submit(img.shape[0], img.shape[1], 3, tw, img, arrival=0.0) for img, tw in reqs]
    while not srv.idle():
        srv.step()
        assert srv.in_use <= budget and len(srv.active) <= 3
    admits = [t.admit for t in ts]
    assert admits == sorted(admits), "admission must follow arrival order"
    assert all(t.status == "done" for t in ts)
    assert srv.peak_active >= 2
    # continuous batching: some step advanced requests admitted at different times together
    assert any(len(a) >= 2 for a in ex.advance_calls)


def test_rejection_and_failures_are_isolated():
    clk = FakeClock()
    reqs = make_reqs(5, seed=2)
    ex = OracleExecutor(clk, fail_start={1}, fail_device={3})
    srv = Server(ex, budget_bytes=1 << 30, max_slots=4, seams_per_step=4, clock=clk)
    ts = [srv.submit(img.shape[0], img.shape[1], 3, tw, img) for img, tw in reqs]
    big = srv.submit(30000, 30000, 3, 15000, None)  # 5.4 GB of state > 1 GiB budget
    bad = srv.submit(10, 10, 3, 11, None)
    drain(srv)
    assert big.status == "rejected" and bad.status == "rejected"
    assert ts[1].status == "error" and "injected" in ts[1].error
    assert ts[3].status == "error"
    for i in (0, 2, 4):
        img, tw = reqs[i]
        assert ts[i].status == "done" and np.array_equal(ts[i].result[0], oracle.carve(img, tw)[0])
    assert srv.in_use == 0 and len(srv.free_slots) == 4


def test_latency_statistics():
    clk = FakeClock()
    srv = Server(OracleExecutor(clk, step_seconds=0.5), budget_bytes=1 << 30, max_slots=1, seams_per_step=100,
                 clock=clk)
    reqs = make_reqs(4, seed=3)
    ts = [srv.submit(img.shape[0], img.shape[1], 3, tw, img, arrival=0.0) for img, tw in reqs]
    drain(srv)
    lat = [t.latency for t in ts]
    assert lat == [0.5, 1.0, 1.5, 2.0]  # one slot: served one after another, one step each
    st = srv.stats()
    assert st["latency_s"]["p50"] == pytest.approx(np.percentile(lat, 50))
    assert st["latency_s"]["p99"] == pytest.approx(np.percentile(lat, 99))
    assert percentile([3, 1, 2], 50) == 2


def test_open_loop_run_with_virtual_time():
    clk = FakeClock()
    srv = Server(OracleExecutor(clk, step_seconds=0.01), budget_bytes=1 << 30, max_slots=8, seams_per_step=4,
                 clock=clk)
    reqs = make_reqs(10, seed=4)

    class R:
        def __init__(self, t, img, tw):
            self.t, self.h, self.w, self.target_w, self.img = t, img.shape[0], img.shape[1], tw, img

    arrivals = [R(0.013 * i, img, tw) for i, (img, tw) in enumerate(reqs)]

    def sleep(dt):
        clk.t += max(dt, 1e-4)

    st = srv.run(arrivals, lambda r: r.img, sleep=sleep)
    assert st["done"] == 10 and st["errors"] == 0
    for t, r in zip(srv.tickets, arrivals):
        assert np.array_equal(t.result[0], oracle.carve(r.img, r.target_w)[0])


def test_team_policy_sizes():
    from paper_2410_21207_amd.serve import Ticket, team_by_work
    pol = team_by_work(min_pixel_seams=1e6, max_team=16)
    assert pol(Ticket(0, 100, 100, 3, 90, 0.0)) == 1                     # little work left
    assert pol(Ticket(1, 4096, 4096, 3, 2048, 0.0)) == 8                 # 29 strips: 4 x 2
    assert pol(Ticket(2, 2000, 1000, 3, 500, 0.0)) == 2
