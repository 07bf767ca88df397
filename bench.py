"""Benchmark of the seam-carving hot path on one MI355X.

Workload (one "step"): the batched configuration -- 256 RGB uint8 blob+noise images with
H and W each uniform in [240, 2160] (seed 3), each removing a uniform 10-40 % of its width --
carved in one launch: the energy pass (src -> img copy + e1 energy of every image) and the
persistent carve kernel running every image's seam loop (DP sweep, argmin, backtrack, removal,
band energy).  Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line: throughput in pixel-seams/s (one pixel-seam = one pixel of the current
image swept by one seam iteration), the HBM roofline of the carve kernel (algorithmic bytes of
the byte model / measured kernel time, against 8 TB/s), per-image completion latency p50/p99
inside the batch, the plain per-image path (sequential sc_carve calls) on a sample, and the CPU
oracle timed on the host cores on a bounded sample.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-plain] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "pixel-seams removed/sec + HBM GB/s %peak; p50/p99 carve latency, batched vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "carve_batch_c4_traffic.json")
FWD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fwt_carve_batch_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2410_21207_amd", "csrc", f)
                  for f in ("sc_kernels.hip", "sc_forward.hip", "sc_object.hip", "sc_device.h", "sc_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def byte_model(H: int, W: int, seams: np.ndarray, C: int = 3) -> int:
    """Algorithmic HBM bytes of the carve loop of one image, from its recorded seams.

    The method's loop per seam on an image of current width w: the DP reads the uint16 energy
    plane and writes a 2-bit direction per cell (2.25 B per pixel); removal shifts every pixel
    right of the seam one column left, reading and writing C image bytes and 2 energy bytes
    (10 B per shifted RGB pixel).
    """
    total = 0
    for j in range(seams.shape[0]):
        w = W - j
        total += int(2.25 * H * w) + (2 * C + 4) * int((w - 1 - seams[j].astype(np.int64)).sum())
    return total


def moved_bytes(H: int, W: int, seams: np.ndarray, minside: bool, C: int = 3) -> int:
    """Bytes the kernel itself moves for the same carve: as byte_model, but with min-side removal
    only the shorter side of each row shifts, and rows that lost pixels on their left are moved
    back to column 0 once at the end (2 C bytes per kept pixel)."""
    if not minside:
        return byte_model(H, W, seams, C)
    k = seams.shape[0]
    total = 0
    left = np.zeros(H, dtype=np.int64)
    for j in range(k):
        w = W - j
        s = seams[j].astype(np.int64)
        side = s < w - 1 - s
        left += side
        total += int(2.25 * H * w) + (2 * C + 4) * int(np.where(side, s, w - 1 - s).sum())
    if k:
        total += 2 * C * (W - k) * int((left > 0).sum())
    return total


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--team", type=int, default=None)
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--no-minside", action="store_true",
                    help="remove every seam pixel by shifting the right part (no min-side removal)")
    ap.add_argument("--n", type=int, default=256, help="images in the batch (256 = the configuration)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=24)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU oracle sample: about this many seconds of work per host core (the batch's "
                         "critical image is always in the sample)")
    ap.add_argument("--workload", choices=["batch", "1080p", "4k", "insert", "sweep", "forward", "forward1080p",
                                           "object"],
                    default="batch",
                    help="batch (default): the batched configuration; 1080p / 4k: one image on the plain "
                         "per-image path (1920x1080, 480 seams; 3840x2160, 960 vertical then 540 horizontal); "
                         "insert: 1920x1080 widened by 480 seams; sweep: the paper's size sweep of square "
                         "images, GPU DP against the CPU oracle's DP, greedy and brute force")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(images are independent: a multi-GPU run would shard the job list by work)", flush=True)
        sys.exit(2)

    import torch

    import synth
    from paper_2410_21207_amd import api

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe:
        n = 1 << 30
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 3}), flush=True)
        return
    if args.workload == "forward":
        forward(args, dev)
        return
    if args.workload == "forward1080p":
        forward_single(args, dev)
        return
    if args.workload == "object":
        object_removal(args, dev)
        return
    if args.workload != "batch":
        single(args, dev)
        return
    jobs = synth.batch_jobs(n=args.n)
    t0 = time.time()
    imgs_np = [j.image() for j in jobs]
    log(f"generated {len(jobs)} images in {time.time() - t0:.1f}s")
    srcs = [torch.from_numpy(a).to(dev) for a in imgs_np]
    dsts = [torch.empty_like(s) for s in srcs]
    targets = [j.target_w for j in jobs]
    pixel_seams = sum(j.pixel_seams for j in jobs)
    seams_total = sum(j.seams for j in jobs)
    torch.cuda.synchronize()

    minside = not args.no_minside
    bc = api.BatchCarver(dsts, targets, srcs=srcs, team=args.team, variant=args.variant, minside=minside)
    stream = torch.cuda.current_stream()

    def step(evs=None):
        if evs is not None:
            evs[0].record(stream)
        bc.launch_energy()
        if evs is not None:
            evs[1].record(stream)
        bc.launch_carve()
        if evs is not None:
            evs[2].record(stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i} done")
    status = bc.status()
    assert all(s == 0 for s in status), f"device status {status}"

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1000.0 / args.steps
    status = bc.status()  # a device failure during the timed steps voids the measurement
    assert all(s == 0 for s in status), f"device status after the timed steps {status}"
    energy_ms = [e[0].elapsed_time(e[1]) for e in events]
    carve_ms = [e[1].elapsed_time(e[2]) for e in events]
    log(f"steps: {ms_per_step:.1f} ms/step; energy pass {np.mean(energy_ms):.2f} ms; carve {np.mean(carve_ms):.1f} ms")

    # per-image completion latency inside the batch (device clock, from the first image's start)
    times = bc.times()
    t_first = min(tb for tb, _ in times)
    lat_ms = [(te - t_first) * 1000.0 for _, te in times]
    run_ms = [(te - tb) * 1000.0 for tb, te in times]

    # where the carve time goes: per-image stage clocks (first workgroup of each image)
    stages = np.array(bc.stages())  # [n, 3] seconds
    longest = int(np.argmax(run_ms))

    # algorithmic bytes of one carve launch, from the recorded seams
    res = bc.results()
    model_bytes = moved = 0
    for j, (_, seams, _) in zip(jobs, res):
        if seams is not None:
            sn = seams.cpu().numpy()
            model_bytes += byte_model(j.h, j.w, sn)
            moved += moved_bytes(j.h, j.w, sn, minside)
    carve_s = float(np.mean(carve_ms)) / 1000.0
    achieved = model_bytes / carve_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                "kernel": "carve_batch_kernel", "model_bytes_per_launch": model_bytes,
                "kernel_moved_bytes_per_launch": moved,
                "kernel_ms": round(float(np.mean(carve_ms)), 3)}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            roofline["traffic"] = tr.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": round(pixel_seams / (ms_per_step / 1000.0), 1),
        "unit": "pixel-seams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"batched carve: {len(jobs)} RGB uint8 blob+noise images, H,W~U[240,2160], "
                               "10-40% of width removed (seed 3)",
                   "images": len(jobs), "seams": seams_total, "pixel_seams": pixel_seams,
                   "team": bc.info.team, "variant": api.variants()[bc.info.variant], "minside": minside,
                   "autotuned": args.team is None and args.variant is None and bc.tuned != (None, None)},
        "roofline": roofline,
        "hbm_gbps_step": round(model_bytes / (ms_per_step / 1000.0) / 1e9, 1),
        "latency_ms": {"p50": round(pct(lat_ms, 50), 2), "p99": round(pct(lat_ms, 99), 2),
                       "max": round(max(lat_ms), 2), "per_image_run_p50": round(pct(run_ms, 50), 2)},
        "energy_pass_ms": round(float(np.mean(energy_ms)), 3),
        "stages_s_all_images": {"dp": round(float(stages[:, 0].sum()), 3),
                                "backtrack_removal": round(float(stages[:, 1].sum()), 3),
                                "band": round(float(stages[:, 2].sum()), 3)},
        "longest_image": {"h": jobs[longest].h, "w": jobs[longest].w, "seams": jobs[longest].seams,
                          "run_ms": round(run_ms[longest], 1),
                          "dp_ms": round(float(stages[longest, 0]) * 1e3, 1),
                          "backtrack_removal_ms": round(float(stages[longest, 1]) * 1e3, 1),
                          "band_ms": round(float(stages[longest, 2]) * 1e3, 1)},
        "teams": bc.info.teams_used,
    }

    # graph replay of the same launch (informative)
    replayed = False
    try:
        bc.capture()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        bc.replay()
        torch.cuda.synchronize()
        out["graph_replay_ms"] = round((time.perf_counter() - tg) * 1000.0, 3)
        replayed = True
    except Exception as ex:  # pragma: no cover - informative only
        out["graph_replay_ms"] = f"unavailable: {ex}"
    if replayed:
        status = bc.status()
        assert all(s == 0 for s in status), f"device status after the graph replay {status}"

    if not args.no_plain:
        # plain path: sequential sc_carve calls on one stream over a seeded sample of the images
        rng = np.random.default_rng(0)
        idx = sorted(rng.choice(len(jobs), size=min(args.plain_sample, len(jobs)), replace=False).tolist())
        ws = api.workspace(max(api._lib.load().sc_workspace_bytes(jobs[i].h, jobs[i].w, 3) for i in idx), dev)
        plat = []
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for i in idx:
            ti = time.perf_counter()
            api.carve(dsts[i], targets[i], src=srcs[i], record=False, team=args.team, variant=args.variant, ws=ws,
                      minside=minside)
            torch.cuda.synchronize()
            plat.append((time.perf_counter() - ti) * 1000.0)
        tp = time.perf_counter() - tp
        ps = sum(jobs[i].pixel_seams for i in idx)
        out["plain"] = {"value": round(ps / tp, 1), "unit": "pixel-seams/s", "sample_images": len(idx),
                        "per_image_ms_p50": round(pct(plat, 50), 2), "per_image_ms_p99": round(pct(plat, 99), 2),
                        "batched_speedup": round((pixel_seams / (ms_per_step / 1000.0)) / (ps / tp), 2)}
        log(f"plain: {out['plain']}")

    copy = copy_bandwidth(dev)
    out["roofline"]["copy_gbps"] = copy
    out["roofline"]["frac_of_copy"] = round(achieved / copy, 4)
    log(f"copy probe: {copy} GB/s")

    if not args.no_cpu:
        heaviest = int(np.argmax([j.pixel_seams for j in jobs]))
        out["cpu_baseline"] = cpu_baseline(jobs, imgs_np, res, args.cpu_seconds, must=(longest, heaviest))
    print(json.dumps(out), flush=True)


def single(args, dev):
    """One image on the plain path (sc_carve per image; the 4k case transposes for its horizontal seams)."""
    import torch

    import synth
    from paper_2410_21207_amd import api

    if args.workload == "insert":
        insert(args, dev)
        return
    if args.workload == "sweep":
        sweep(args, dev)
        return
    if args.workload == "1080p":
        H, W, seed, tw, th = 1080, 1920, 1, 1440, None
    else:
        H, W, seed, tw, th = 2160, 3840, 2, 2880, 1620
    src = torch.from_numpy(synth.blob_image(H, W, 3, seed=seed)).to(dev)
    dst = torch.empty_like(src)
    kv = W - tw
    ps = H * (kv * W - kv * (kv - 1) // 2)
    if th is not None:
        kh = H - th
        ps += tw * (kh * H - kh * (kh - 1) // 2)
    stream = torch.cuda.current_stream()

    def step(record=False):
        out, vs, _ = api.carve(dst, tw, src=src, record=record)
        if th is None:
            return out, vs, None
        t = api.transpose(out)                      # [tw, H, C]
        t2, hs, _ = api.carve(t, th, record=record)
        return api.transpose(t2), vs, hs

    _, vs, hs = step(record=True)                  # warm-up, and the seams for the byte model
    torch.cuda.synchronize()
    model = byte_model(H, W, vs.cpu().numpy())
    if hs is not None:
        model += byte_model(tw, H, hs.cpu().numpy())
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    gpu_s = e0.elapsed_time(e1) / 1000.0 / args.steps
    out = {"metric": METRIC, "value": round(ps / wall, 1), "unit": "pixel-seams/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1000.0, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"plain path, one {W}x{H} RGB uint8 blob+noise image (seed {seed}), "
                                  + (f"{kv} vertical seams" if th is None else
                                     f"{kv} vertical then {H - th} horizontal seams via transpose"),
                      "pixel_seams": ps, "autotuned": True},
           "roofline": {"bound": "hbm", "achieved": round(model / gpu_s / 1e9, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": round(model / gpu_s / 1e9 / HBM_PEAK_GBPS, 4), "traffic": None,
                        "kernel": "carve_single_kernel (+ energy pass, transposes)", "model_bytes_per_step": model},
           "latency_ms": round(gpu_s * 1000.0, 3)}
    print(json.dumps(out), flush=True)


def insert(args, dev):
    """Seam insertion: one 1920x1080 image widened by 480 seams (seam search by carving a copy,
    mapping to original columns, widened image)."""
    import torch

    import synth
    from paper_2410_21207_amd import api

    H, W, k = 1080, 1920, 480
    src = torch.from_numpy(synth.blob_image(H, W, 3, seed=1)).to(dev)
    out = torch.empty((H, W + k, 3), dtype=torch.uint8, device=dev)
    ps = H * (k * W - k * (k - 1) // 2)  # the seam search sweeps the same pixels as a carve to W - k
    _, seams = api.insert_seams(src, k, out=out)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        api.insert_seams(src, k, out=out, record=False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        api.insert_seams(src, k, out=out, record=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    gpu_s = e0.elapsed_time(e1) / 1000.0 / args.steps
    print(json.dumps({"metric": METRIC, "value": round(ps / wall, 1), "unit": "pixel-seams/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1000.0, 3),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                      "data": "synthetic",
                      "config": {"workload": "seam insertion: one 1920x1080 RGB uint8 blob+noise image (seed 1) "
                                             "widened by 480 seams", "pixel_seams": ps},
                      "latency_ms": round(gpu_s * 1000.0, 3)}), flush=True)


def _slope(ns, ts):
    """Least-squares slope of log(time) against log(n)."""
    x, y = np.log(np.asarray(ns, float)), np.log(np.asarray(ts, float))
    return float(np.polyfit(x, y, 1)[0])


def sweep(args, dev):
    """The paper's runtime experiment re-run on MI355X: one square blob image at 180, 360, 480, 720
    and 1080 px (nearest-neighbour versions of the 1080 px image), carved to half its width
    (s = 0.5) by the GPU DP path; the CPU legs time the oracle's DP carve and a greedy carve on one
    host core, and the oracle's brute force on 2..12 px images.  T = one seam, C = the carve."""
    import torch

    import synth
    from paper_2410_21207_amd import api

    base = synth.blob_image(1080, 1080, 3, seed=6)
    rows = []
    for n in (180, 360, 480, 720, 1080):
        img = synth.resized(base, n)
        src = torch.from_numpy(img).to(dev)
        dst = torch.empty_like(src)
        e = api.energy(src)
        api.dp_seam(e)
        api.carve(dst, n // 2, src=src)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            api.dp_seam(e)
        torch.cuda.synchronize()
        t_gpu = (time.perf_counter() - t) / args.steps
        t = time.perf_counter()
        for _ in range(args.steps):
            _, seams, _ = api.carve(dst, n // 2, src=src)
        torch.cuda.synchronize()
        c_gpu = (time.perf_counter() - t) / args.steps
        rows.append({"n": n, "gpu_T_ms": round(t_gpu * 1e3, 3), "gpu_C_ms": round(c_gpu * 1e3, 3),
                     "_img": img, "_seams": seams.cpu().numpy()})
    out = {"metric": METRIC, "value": None, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "higher_is_better": False, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "size sweep: square blob image (seed 6) at 180-1080 px, half the width removed"}}
    if not args.no_cpu:
        cpu_baseline_sweep(rows)
    for r in rows:
        r.pop("_img"), r.pop("_seams")
    out["sweep"] = rows
    ns = [r["n"] for r in rows]
    out["slopes_loglog"] = {"gpu_T": round(_slope(ns, [r["gpu_T_ms"] for r in rows]), 2),
                            "gpu_C": round(_slope(ns, [r["gpu_C_ms"] for r in rows]), 2)}
    if not args.no_cpu:
        for key in ("dp_T_ms", "dp_C_ms", "greedy_T_ms", "greedy_C_ms"):
            out["slopes_loglog"][key[:-3]] = round(_slope(ns, [r[key] for r in rows]), 2)
        out["brute_force"] = cpu_brute_sweep()
    print(json.dumps(out), flush=True)


def cpu_baseline_sweep(rows):
    """The oracle on one host core at every size of the sweep: its DP seam (T) and carve (C), and a
    greedy carve built from its greedy seam; the GPU seams must equal the oracle's."""
    import oracle

    oracle.default()
    for r in rows:
        img, n = r["_img"], r["n"]
        e = oracle.energy(img)
        t = time.perf_counter()
        oracle.dp_seam(e)
        r["dp_T_ms"] = round((time.perf_counter() - t) * 1e3, 3)
        t = time.perf_counter()
        _, seams, _ = oracle.carve(img, n // 2)
        r["dp_C_ms"] = round((time.perf_counter() - t) * 1e3, 3)
        r["seams_match_gpu"] = bool(np.array_equal(seams, r["_seams"]))
        t = time.perf_counter()
        oracle.greedy_seam(e)
        r["greedy_T_ms"] = round((time.perf_counter() - t) * 1e3, 3)
        cur = img.copy()
        t = time.perf_counter()
        for _ in range(n // 2):
            s, _ = oracle.greedy_seam(oracle.energy(cur))
            cur = oracle.remove_seam(cur, s)
        r["greedy_C_ms"] = round((time.perf_counter() - t) * 1e3, 3)


def cpu_brute_sweep():
    """Brute force (the oracle's exhaustive seam search) at the paper's sizes 2..12 px."""
    import oracle

    import synth
    out = []
    base = synth.blob_image(1080, 1080, 3, seed=6)
    for n in (2, 5, 7, 10, 12):
        img = synth.resized(base, n)
        e = oracle.energy(img)
        t = time.perf_counter()
        oracle.brute_seam(e)
        t_seam = time.perf_counter() - t
        cur = img.copy()
        t = time.perf_counter()
        for _ in range(max(1, n // 2)):
            s, _ = oracle.brute_seam(oracle.energy(cur))
            cur = oracle.remove_seam(cur, s)
        out.append({"n": n, "T_ms": round(t_seam * 1e3, 4), "C_ms": round((time.perf_counter() - t) * 1e3, 4)})
    ns = np.array([o["n"] for o in out], float)
    # T(n, n) ~ n 3^n: the slope of log(T / n) against n estimates log 3 (fitted on 10 and 12 px:
    # below that a seam takes microseconds and call overhead dominates)
    big = ns >= 10
    tt = np.array([o["T_ms"] for o in out])[big]
    out_fit = float(np.polyfit(ns[big], np.log(tt / ns[big]), 1)[0])
    return {"sizes": out, "fit_log_base_of_T_over_n_10_12": round(out_fit, 3), "log_3": round(float(np.log(3)), 3)}


def forward_byte_model(H: int, W: int, C: int, k: int) -> int:
    """Algorithmic HBM bytes of k forward-energy seams of an H x W x C image, one seam at a time:
    the DP reads the current image once (H*w*C) and writes the 2-bit direction map (H*w/4); the
    removal moves the pixels right of the seam, on average half a row each way (H*w*C)."""
    return sum(H * w * C + H * w // 4 + H * w * C for w in range(W, W - k, -1))


def forward(args, dev):
    """Forward-energy carve (sec. "Forward Energy Calculation") of the batched workload: the same
    256 images as the default benchmark, each carved by a team of 256-thread workgroups on one XCD."""
    import torch

    import synth
    from paper_2410_21207_amd import api

    jobs = synth.batch_jobs(n=args.n)
    imgs_np = [j.image() for j in jobs]
    srcs = [torch.from_numpy(a).to(dev) for a in imgs_np]
    dsts = [torch.empty_like(s) for s in srcs]
    pixel_seams = sum(j.pixel_seams for j in jobs)
    fb = api.ForwardBatch(dsts, [j.target_w for j in jobs], srcs=srcs)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        fb.launch()
        torch.cuda.synchronize()
        log(f"warmup {i} done")
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        events[i][0].record(stream)
        fb.launch_copy()
        events[i][1].record(stream)
        fb.launch_carve()
        events[i][2].record(stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    copy_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    carve_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    times = fb.times()
    t_first = min(tb for tb, _ in times)
    lat_ms = [(te - t_first) * 1000.0 for _, te in times]
    longest = int(np.argmax([te - tb for tb, te in times]))
    stages = fb.stages()
    model_bytes = sum(forward_byte_model(j.h, j.w, 3, j.seams) for j in jobs)
    fwd_traffic = None
    if os.path.exists(FWD_TRAFFIC_FILE):
        with open(FWD_TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            fwd_traffic = tr.get("bytes_per_launch")
    achieved = model_bytes / (carve_ms / 1000.0) / 1e9
    out = {
        "metric": METRIC, "value": round(pixel_seams / (ms_per_step / 1000.0), 1), "unit": "pixel-seams/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"forward-energy batched carve: {len(jobs)} RGB uint8 blob+noise images, "
                               "H,W~U[240,2160], 10-40% of width removed (seed 3)",
                   "images": len(jobs), "pixel_seams": pixel_seams},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": fwd_traffic, "kernel": "fwt_carve_kernel",
                     "model_bytes_per_launch": model_bytes, "kernel_ms": round(carve_ms, 3)},
        "copy_pass_ms": round(copy_ms, 3),
        "latency_ms": {"p50": round(pct(lat_ms, 50), 2), "p99": round(pct(lat_ms, 99), 2),
                       "max": round(max(lat_ms), 2)},
        "longest_image": {"h": jobs[longest].h, "w": jobs[longest].w, "seams": jobs[longest].seams,
                          "run_ms": round((times[longest][1] - times[longest][0]) * 1000.0, 1),
                          "dp_ms": round(float(stages[longest][0]) * 1e3, 1),
                          "backtrack_ms": round(float(stages[longest][1]) * 1e3, 1),
                          "removal_ms": round(float(stages[longest][2]) * 1e3, 1)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(jobs, imgs_np, fb.results(), args.cpu_seconds, forward=True)
    print(json.dumps(out), flush=True)


def forward_single(args, dev):
    """Forward-energy carve of one 1920x1080 RGB image to 1440 columns (480 seams)."""
    import torch

    import synth
    from paper_2410_21207_amd import api

    H, W, tw = 1080, 1920, 1440
    src = torch.from_numpy(synth.blob_image(H, W, 3, seed=1)).to(dev)
    dst = torch.empty_like(src)
    ws = api.workspace(api._lib.load().sc_forward_workspace_bytes(H, W, 3), dev)
    ps = H * sum(range(tw + 1, W + 1))
    for _ in range(args.warmup):
        api.carve_forward(dst, tw, src=src, record=False, ws=ws)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        api.carve_forward(dst, tw, src=src, record=False, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"metric": METRIC, "value": round(ps / wall, 1), "unit": "pixel-seams/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1000.0, 3),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                      "data": "synthetic",
                      "config": {"workload": "forward-energy carve: one 1920x1080 RGB uint8 blob+noise image "
                                             "(seed 1) to 1440 columns", "pixel_seams": ps},
                      "gpu_ms_per_step": round(e0.elapsed_time(e1) / args.steps, 3),
                      "stages_ms_last_call": _stage_ms(api, ws, ["dp", "backtrack_removal"])}), flush=True)


def _stage_ms(api, ws, names):
    """Per-stage device clocks of the last carve in a single-image workspace, in ms."""
    st = api.read_stages(ws, 1)[0]  # seconds
    return {n: round(float(st[i]) * 1000.0, 3) for i, n in enumerate(names)}


def object_byte_model(h: int, w0: int, C: int, seams: np.ndarray) -> int:
    """Algorithmic HBM bytes of the masked carve of an h-row frame from its recorded seams.

    Per seam on a frame of current width w: the DP reads the pixels and the mask byte of every
    cell and writes a 2-bit direction ((C + 1.25) bytes per cell; the energy is computed from the
    pixels it reads); the removal moves the pixels and mask bytes right of the seam one column
    left (read and write, 2 * (C + 1) bytes each)."""
    total = 0
    for j in range(seams.shape[0]):
        w = w0 - j
        total += int(h * w * (C + 1.25)) + 2 * (C + 1) * int(np.sum(w - 1 - seams[j].astype(np.int64)))
    return total


def object_removal(args, dev):
    """Object removal with a mask: one 1920x1080 RGB blob+noise image (seed 1) with a filled
    elliptical object of semi-axes 100 x 200 px at the centre, removed by masked vertical seams
    and the size restored by seam insertion."""
    import torch

    import synth
    from paper_2410_21207_amd import api

    H, W, C = 1080, 1920, 3
    img_np = synth.blob_image(H, W, C, seed=1)
    mask_np = synth.ellipse_mask(H, W, 540, 960, 200, 100)
    img = torch.from_numpy(img_np).to(dev)
    mask = torch.from_numpy(mask_np).to(dev)
    lib = api._lib.load()
    ws = api.workspace(lib.sc_object_workspace_bytes(H, W, C, 1), dev)
    for _ in range(args.warmup):
        api.remove_object(img, mask, restore=True, record=False, ws=ws)
    torch.cuda.synchronize()
    walls, carve_ms, stages = [], [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        out, info, _, _ = api.remove_object(img, mask, restore=True, record=False, ws=ws)  # synchronous
        walls.append(time.perf_counter() - t0)
        carve_ms.append(info["carve_ms"])
        stages.append(info["stage_ms"])
    out, info, seams, costs = api.remove_object(img, mask, restore=True, ws=ws)
    seams = seams.cpu().numpy()
    k = info["k"]
    h, w0 = (H, W) if info["direction"] == 0 else (W, H)
    ps = h * sum(w0 - j for j in range(k))  # pixel-seams of the masked carve
    model = object_byte_model(h, w0, C, seams)
    cms = float(np.median(carve_ms))
    wall = float(np.median(walls))
    res = {"metric": METRIC, "value": round(ps / wall, 1), "unit": "pixel-seams/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1000.0, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": "object removal: one 1920x1080 RGB uint8 blob+noise image (seed 1), filled "
                                  "ellipse mask of semi-axes 100x200 px at the centre, masked seams until the "
                                  "object is gone, then the size restored by seam insertion",
                      "direction": info["direction"], "seams": k, "pixel_seams": ps},
           "roofline": {"bound": "hbm", "achieved": round(model / (cms / 1000.0) / 1e9, 1), "peak": 8000.0,
                        "unit": "GB/s", "frac": round(model / (cms / 1000.0) / 8e12, 4), "traffic": None,
                        "kernel": "obj_carve_kernel", "model_bytes_per_launch": model,
                        "kernel_ms": round(cms, 3)},
           "stages_ms": {"dp": round(float(np.median([s[0] for s in stages])), 3),
                         "argmin_backtrack": round(float(np.median([s[1] for s in stages])), 3),
                         "removal": round(float(np.median([s[2] for s in stages])), 3)},
           "carve_pixel_seams_per_s": round(ps / (cms / 1000.0), 1),
           "restore_and_rest_ms": round(wall * 1000.0 - cms, 3)}
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        o_out, o_info, o_seams, o_costs = oracle.remove_object(img_np, mask_np, -1, True)
        ct = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(ps / ct, 1), "unit": "pixel-seams/s (whole call incl. restore)",
                               "cores": 1, "kind": "oracle", "sample": "the whole workload, one host thread",
                               "seconds": round(ct, 2),
                               "matches_gpu": bool(np.array_equal(o_seams, seams) and
                                                   np.array_equal(o_costs, costs.cpu().numpy()) and
                                                   np.array_equal(o_out, out.cpu().numpy()))}
    print(json.dumps(res), flush=True)


def cpu_baseline(jobs, imgs_np, gpu_results, seconds, forward=False, must=()):
    """The oracle, as it stands, on a bounded sample of the same workload on the host cores.

    The sample is the images in `must` (the batch's critical images), then images in job order up
    to about `seconds` of work per core; every sampled image's seams, costs and output pixels are
    compared with the GPU's."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    budget = seconds * (3e7 if forward else 1e8) * cores  # the forward oracle does three pair sums per cell
    idx = list(dict.fromkeys(int(i) for i in must))
    acc = sum(jobs[i].pixel_seams for i in idx)
    for i, j in enumerate(jobs):
        if i in idx:
            continue
        if acc + j.pixel_seams > budget:
            continue
        idx.append(i)
        acc += j.pixel_seams
        if acc >= budget * 0.9:
            break
    oracle.default()

    def run(i):
        if forward:
            return oracle.carve_forward(imgs_np[i], jobs[i].target_w)
        return oracle.carve(imgs_np[i], jobs[i].target_w)

    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        outs = list(ex.map(run, idx))  # the critical images start first
    dt = time.perf_counter() - t
    agree = {"seams": True, "costs": True, "pixels": True}
    for o, i in zip(outs, idx):
        g_out, g_seams, g_costs = gpu_results[i]
        if g_seams is None:
            agree["seams"] &= o[1].size == 0
            agree["costs"] &= o[2].size == 0
        else:
            agree["seams"] &= bool(np.array_equal(o[1], g_seams.cpu().numpy()))
            agree["costs"] &= bool(np.array_equal(o[2], g_costs.cpu().numpy()))
        agree["pixels"] &= bool(np.array_equal(o[0], g_out.cpu().numpy()))
    crit = ", ".join(f"{jobs[i].w}x{jobs[i].h}" for i in dict.fromkeys(int(i) for i in must))
    order = f"the critical image(s) {crit}, then job order" if must else "job order"
    return {"value": round(acc / dt, 1), "unit": "pixel-seams/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} of the {len(jobs)} batch images ({order} up to ~{seconds:.0f}s per core), "
                      f"full carves, one image per thread, {dt:.1f}s wall",
            "seams_match_gpu": agree["seams"], "costs_match_gpu": agree["costs"],
            "pixels_match_gpu": agree["pixels"]}


def copy_bandwidth(dev, nbytes=1 << 30, reps=5):
    """Achievable HBM bandwidth: a plain device-to-device copy of nbytes, timed with HIP events on
    its stream; read plus write bytes per second."""
    import torch

    a = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    gbps = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbps, 1)


if __name__ == "__main__":
    main()
