"""Continuous-batching carve server (serving configuration of the seam-carving path).

Requests of different sizes arrive over time.  The server admits them in arrival order as soon
as a slot and enough of the HBM budget are free, keeps every admitted image and its carve state
on the device between seams, and advances ALL admitted images together: one step is one launch
of the step kernel (``sc_slots_step_timed``), one workgroup per image, in which every active
image removes seams until the step's time budget is spent (or ``seams_per_step`` seams): small
requests finish within a step and no workgroup waits for the largest one.  With a team policy
(``sc_slots_step_teams``) a request with much work left advances with a team of workgroups on
one XCD instead of one, so the largest requests no longer set the tail latency.  A request that
arrives while others are mid-carve joins at the next step; its work overlaps theirs on the
device.  Latency is arrival to completion.

The executor is an interface: ``GPUExecutor`` drives the C ABI; tests drive the same scheduler
with a fake executor on the CPU.

    python -m paper_2410_21207_amd.serve [--rate 300] [--duration 60] [--budget-gb 64] [--step-us 20000]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys
import time
from collections import deque
from dataclasses import dataclass, field

__all__ = ["Ticket", "Server", "GPUExecutor", "percentile", "team_by_work"]


@dataclass
class Ticket:
    """One request's life: arrival -> admission -> completion (times in seconds of the server clock)."""
    id: int
    h: int
    w: int
    c: int
    target_w: int
    arrival: float
    payload: object = None
    admit: float | None = None
    done: float | None = None
    status: str = "queued"   # queued | running | done | error | rejected
    slot: int = -1
    seams_done: int = 0
    state_bytes: int = 0
    result: object = None
    error: str = ""

    @property
    def seams(self) -> int:
        return self.w - self.target_w

    @property
    def pixel_seams(self) -> int:
        k = self.seams
        return self.h * (k * self.w - k * (k - 1) // 2)

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


def team_by_work(min_pixel_seams: float = 4e8, max_team: int = 16):
    """A team policy: a request with at least `min_pixel_seams` of work left gets one workgroup per
    eight 144-column DP strips of its current width, doubled for the removal (2 .. max_team);
    every other request one workgroup."""
    def policy(t: "Ticket") -> int:
        r = t.seams - t.seams_done
        wc = t.w - t.seams_done
        left = t.h * r * (wc - (r - 1) / 2.0)
        if left < min_pixel_seams:
            return 1
        strips = -(-wc // 144)
        return int(min(max_team, max(2, 2 * -(-strips // 8))))
    return policy


def percentile(xs, q):
    """Linear-interpolated percentile of a non-empty list (q in [0, 100])."""
    xs = sorted(xs)
    if not xs:
        return float("nan")
    pos = (len(xs) - 1) * q / 100.0
    lo = math.floor(pos)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (pos - lo)


class Server:
    """FIFO admission by HBM budget and free slots; continuous batching of the carve steps."""

    def __init__(self, executor, budget_bytes: int = 64 << 30, max_slots: int = 256, seams_per_step: int = 16,
                 clock=time.perf_counter, step_budget_us: int = 0, team_policy=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.seams_per_step = int(seams_per_step)
        self.step_budget_us = int(step_budget_us)  # > 0: steps end on time, seams_per_step is a cap
        self.team_policy = team_policy  # ticket -> workgroups carving it in the next step, or None
        self.clock = clock
        self.queue: deque[Ticket] = deque()
        self.active: dict[int, Ticket] = {}
        self.free_slots = list(range(self.max_slots - 1, -1, -1))
        self.in_use = 0
        self.tickets: list[Ticket] = []
        self.steps = 0
        self.peak_active = 0
        self.peak_bytes = 0

    # ------------------------------------------------------------------ requests
    def submit(self, h: int, w: int, c: int, target_w: int, payload=None, arrival: float | None = None) -> Ticket:
        t = Ticket(len(self.tickets), int(h), int(w), int(c), int(target_w),
                   self.clock() if arrival is None else float(arrival), payload)
        t.state_bytes = self.ex.state_bytes(t.h, t.w, t.c, t.target_w)
        self.tickets.append(t)
        if t.state_bytes > self.budget or not (1 <= t.target_w <= t.w):
            t.status = "rejected"
            t.error = "larger than the whole budget" if t.state_bytes > self.budget else "bad target width"
            t.done = t.arrival
            return t
        self.queue.append(t)
        return t

    def _admit(self, now: float):
        while self.queue and self.free_slots and self.in_use + self.queue[0].state_bytes <= self.budget:
            t = self.queue.popleft()
            slot = self.free_slots.pop()
            try:
                self.ex.start(slot, t)
            except Exception as ex:  # this request fails alone; the others go on
                t.status, t.error, t.done = "error", str(ex), now
                self.free_slots.append(slot)
                continue
            t.slot, t.status, t.admit = slot, "running", now
            self.active[slot] = t
            self.in_use += t.state_bytes
            self.peak_bytes = max(self.peak_bytes, self.in_use)
        self.peak_active = max(self.peak_active, len(self.active))

    def _retire(self, t: Ticket, now: float, status: str, error: str = ""):
        t.status, t.error, t.done = status, error, now
        if status == "done":
            t.result = self.ex.result(t.slot)
        self.ex.release(t.slot)
        del self.active[t.slot]
        self.free_slots.append(t.slot)
        self.in_use -= t.state_bytes
        t.payload = None

    def step(self) -> list[Ticket]:
        """Admit what fits, advance every active image by up to seams_per_step seams, retire the done."""
        self._admit(self.clock())
        if not self.active:
            return []
        n = max(self.active) + 1
        if self.team_policy is not None:
            teams = [1] * n
            for slot, t in self.active.items():
                teams[slot] = max(1, int(self.team_policy(t)))
            progress = self.ex.advance(n, self.seams_per_step, self.step_budget_us, teams)
        elif self.step_budget_us:
            progress = self.ex.advance(n, self.seams_per_step, self.step_budget_us)
        else:
            progress = self.ex.advance(n, self.seams_per_step)
        self.steps += 1
        now = self.clock()
        finished = []
        for slot, t in list(self.active.items()):
            p = progress[slot]
            if p >= 0:
                t.seams_done = p
            if p < 0:
                self._retire(t, now, "error", f"device status {p}")
                finished.append(t)
            elif p >= t.seams:
                self._retire(t, now, "done")
                finished.append(t)
        return finished

    def idle(self) -> bool:
        return not self.queue and not self.active

    # ------------------------------------------------------------------ open-loop run
    def run(self, arrivals, make_payload, horizon: float | None = None, sleep=time.sleep, progress=None,
            progress_every: float = 5.0):
        """Serve `arrivals` (objects with .t, .h, .w, .target_w) released at their arrival times.

        make_payload(req) builds a request's pixels when it arrives.  progress(text), when given,
        is called about every `progress_every` seconds.  Returns self.stats().
        """
        arrivals = sorted(arrivals, key=lambda r: r.t)
        t0 = self.clock()
        i = 0
        next_report = progress_every
        while i < len(arrivals) or not self.idle():
            now = self.clock() - t0
            if progress is not None and now >= next_report:
                next_report += progress_every
                done = sum(t.status == "done" for t in self.tickets)
                progress(f"t={now:.1f}s arrived {i}/{len(arrivals)} active {len(self.active)} "
                         f"queued {len(self.queue)} done {done} steps {self.steps}")
            while i < len(arrivals) and arrivals[i].t <= now:
                r = arrivals[i]
                self.submit(r.h, r.w, getattr(r, "c", 3), r.target_w, make_payload(r), arrival=t0 + r.t)
                i += 1
            if self.idle():
                if i < len(arrivals):
                    sleep(max(0.0, min(arrivals[i].t - now, 0.005)))
                continue
            self.step()
            if horizon is not None and now > horizon:
                break
        return self.stats(t0)

    def stats(self, t0: float | None = None) -> dict:
        done = [t for t in self.tickets if t.status == "done"]
        lat = [t.latency for t in done]
        t0 = min((t.arrival for t in self.tickets), default=0.0) if t0 is None else t0
        t_end = max((t.done for t in done), default=t0)
        span = max(t_end - t0, 1e-9)
        ps = sum(t.pixel_seams for t in done)
        return {
            "requests": len(self.tickets), "done": len(done),
            "errors": sum(t.status == "error" for t in self.tickets),
            "rejected": sum(t.status == "rejected" for t in self.tickets),
            "latency_s": {"p50": round(percentile(lat, 50), 4) if lat else None,
                          "p99": round(percentile(lat, 99), 4) if lat else None,
                          "max": round(max(lat), 4) if lat else None},
            "pixel_seams": ps, "pixel_seams_per_s": round(ps / span, 1), "span_s": round(span, 3),
            "steps": self.steps, "peak_active": self.peak_active, "peak_state_gb": round(self.peak_bytes / 1e9, 3),
        }


class GPUExecutor:
    """Device side of the server: one slot table, per-request device image + workspace.

    Every admitted request is stepped in the slot table (one workgroup per image in each step
    launch); a device failure of a slot comes back as a negative progress value, which the server
    turns into an error for that request alone.
    """

    def __init__(self, max_slots: int, device="cuda"):
        import torch

        from . import _lib, api
        self.torch, self._lib, self.lib, self.api = torch, _lib, _lib.load(), api
        self.device = torch.device(device)
        self.max_slots = max_slots
        self.table = torch.zeros(self.lib.sc_slot_table_bytes(max_slots), dtype=torch.uint8, device=self.device)
        self.progress = torch.zeros(max_slots, dtype=torch.int32, device=self.device)
        self.progress_host = torch.zeros(max_slots, dtype=torch.int32).pin_memory()
        self.state = [None] * max_slots
        # a stream of its own for the steps (default priority)
        self.stream = torch.cuda.Stream(self.device)

    def state_bytes(self, h, w, c, target_w):
        """HBM a request holds while admitted: source and image, workspace, seam log and costs."""
        k = max(w - target_w, 1)
        return 2 * h * w * c + int(self.lib.sc_workspace_bytes(h, w, c)) + 4 * k * h + 8 * k

    def start(self, slot, t: Ticket):
        torch, api, _lib = self.torch, self.api, self._lib
        src = t.payload
        if not isinstance(src, torch.Tensor) or not src.is_cuda:
            src = torch.as_tensor(src).to(self.device, non_blocking=True)
        caller = torch.cuda.current_stream(self.device)  # where the payload was written
        if tuple(src.shape) != (t.h, t.w, t.c):
            raise ValueError(f"payload shape {tuple(src.shape)} != request ({t.h}, {t.w}, {t.c})")
        img = torch.empty_like(src)
        ws = api.workspace(self.lib.sc_workspace_bytes(t.h, t.w, t.c), self.device)
        k = t.seams
        seams = torch.empty((max(k, 1), t.h), dtype=torch.int32, device=self.device)
        costs = torch.empty(max(k, 1), dtype=torch.int64, device=self.device)
        self.state[slot] = (src, img, ws, seams, costs, t.target_w, k)
        job = _lib.sc_job(img.data_ptr(), t.h, t.w, t.c, src.stride(0), t.target_w, seams.data_ptr(),
                          costs.data_ptr(), src.data_ptr())
        # every payload written on the caller's stream is awaited by the step stream
        self.stream.wait_stream(caller)
        _lib.call("sc_slot_start", ctypes.byref(job), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                  ctypes.c_void_p(self.table.data_ptr()), self.max_slots, slot,
                  ctypes.c_void_p(self.stream.cuda_stream))

    def advance(self, n, max_seams, budget_us: int = 0, teams=None):
        if teams is None:
            self._lib.call("sc_slots_step_timed", ctypes.c_void_p(self.table.data_ptr()), n, max_seams,
                           int(budget_us), ctypes.c_void_p(self.progress.data_ptr()),
                           ctypes.c_void_p(self.stream.cuda_stream))
        else:
            arr = (ctypes.c_int32 * n)(*[int(g) for g in teams[:n]])
            self._lib.call("sc_slots_step_teams", ctypes.c_void_p(self.table.data_ptr()), self.max_slots, n, arr,
                           max_seams,
                           int(budget_us), ctypes.c_void_p(self.progress.data_ptr()),
                           ctypes.c_void_p(self.stream.cuda_stream))
        with self.torch.cuda.stream(self.stream):  # ordered after the step on the same stream
            self.progress_host[:n].copy_(self.progress[:n], non_blocking=True)
        self.stream.synchronize()
        return self.progress_host.tolist()

    def result(self, slot):
        src, img, ws, seams, costs, tw, k = self.state[slot]
        return img[:, :tw], (seams if k > 0 else None), (costs if k > 0 else None)

    def release(self, slot):
        self._lib.call("sc_slot_clear", ctypes.c_void_p(self.table.data_ptr()), self.max_slots, slot,
                       ctypes.c_void_p(self.stream.cuda_stream))
        self.state[slot] = None


def main():
    ap = argparse.ArgumentParser(description="serve Poisson carve requests on one GPU")
    ap.add_argument("--rate", type=float, default=300.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=512)
    ap.add_argument("--seams-per-step", type=int, default=1 << 20, help="cap on the seams a slot removes per step")
    ap.add_argument("--step-us", type=int, default=20000,
                    help="time budget of a step in microseconds (0: every slot removes seams-per-step seams)")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--teams", action="store_true",
                    help="requests with much work left advance with a team of workgroups (team_by_work)")
    args = ap.parse_args()

    import torch

    import synth
    reqs = synth.serving_requests(rate=args.rate, duration=args.duration, seed=args.seed)
    dev = torch.device("cuda")
    canvases = [torch.from_numpy(synth.blob_image(4096, 4096, 3, seed=1000 + i)).to(dev) for i in range(16)]
    torch.cuda.synchronize()

    def payload(r):  # a request's pixels: a crop of a device-resident canvas (no PCIe in the loop)
        return canvases[r.canvas][r.y0:r.y0 + r.h, r.x0:r.x0 + r.w].contiguous()

    srv = Server(GPUExecutor(args.slots, dev), budget_bytes=int(args.budget_gb * 1e9),
                 max_slots=args.slots,
                 seams_per_step=args.seams_per_step, step_budget_us=args.step_us,
                 team_policy=team_by_work() if args.teams else None)
    st = srv.run(reqs, payload, progress=lambda m: print(m, file=sys.stderr, flush=True))
    offered = sum(r.h * ((r.w - r.target_w) * r.w - (r.w - r.target_w) * (r.w - r.target_w - 1) // 2)
                  for r in reqs) / args.duration
    st.update({"workload": f"Poisson {args.rate}/s for {args.duration}s, sides log-uniform [128,4096], "
                           "target 50-90% of width, 64 GB budget",
               "offered_pixel_seams_per_s": round(offered, 1), "seams_per_step": args.seams_per_step,
               "step_us": args.step_us, "teams": bool(args.teams),
               "slots": args.slots})
    print(json.dumps(st), flush=True)


if __name__ == "__main__":
    main()
