"""Autotuner for the carve launch shape: kernel variant (columns per lane, rows per DP phase,
threads per workgroup) and the largest team of workgroups per image.

Every candidate computes the same seams, costs and pixels (the parity tests check each variant
and team size against the oracle); only the time differs.  ``autotune_batch`` and
``autotune_single`` time the candidates on the caller's own workload and record the fastest in a
JSON cache keyed by GPU architecture and a size bucket; ``api.carve`` and ``api.BatchCarver``
consult the cache whenever the caller does not fix the launch shape.

    python -m paper_2410_21207_amd.tune [--out PATH]   # tune the standard workloads on this GPU
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")

# (variant id, largest team) pairs tried by default; variant ids index sc_variant_name().  A batch
# carves most of its images with one workgroup each, which the 2-columns-per-lane variant (9)
# slows down, so only single images try it.
BATCH_CANDIDATES = [(v, g) for v in (1, 5, 7) for g in (8, 16, 32)]
SINGLE_CANDIDATES = [(v, g) for v in (1, 5, 7, 9) for g in (4, 8, 16, 32)]

_cache: dict | None = None
_cache_path: str | None = None


def cache_path() -> str:
    return os.environ.get("SC_TUNE_CACHE", DEFAULT_CACHE)


def _bucket(x: int) -> int:
    """Smallest power of two >= x (size buckets of the cache keys)."""
    return 1 << max(0, math.ceil(math.log2(max(1, int(x)))))


def key_single(arch: str, H: int, W: int) -> str:
    return f"{arch}/single/{_bucket(H)}x{_bucket(W)}"


def key_batch(arch: str, shapes) -> str:
    """shapes: iterable of (H, W); bucketed by the tallest and widest image and the batch size."""
    shapes = list(shapes)
    hmax = max(h for h, _ in shapes)
    wmax = max(w for _, w in shapes)
    return f"{arch}/batch/{_bucket(hmax)}x{_bucket(wmax)}/n{_bucket(len(shapes))}"


def load(path: str | None = None) -> dict:
    """The cache as a dict {key: {"variant": v, "team": g, ...}} (empty if the file is absent)."""
    global _cache, _cache_path
    path = path or cache_path()
    if _cache is not None and _cache_path == path:
        return _cache
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
        if not isinstance(data, dict):
            raise ValueError(f"{path}: not a tuning cache")
    _cache, _cache_path = data, path
    return data


def save(entries: dict, path: str | None = None) -> str:
    """Merge `entries` into the cache file and return its path."""
    global _cache, _cache_path
    path = path or cache_path()
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.update(entries)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    _cache, _cache_path = data, path
    return path


def lookup(key: str, path: str | None = None):
    """(variant, team) recorded for `key`, or None."""
    e = load(path).get(key)
    if not e:
        return None
    return int(e["variant"]), int(e["team"])


def device_arch(device=None) -> str:
    import torch
    name = torch.cuda.get_device_properties(device or 0).gcnArchName
    return name.split(":")[0]


def pick(timings: dict):
    """The fastest candidate of {(variant, team): seconds}; ties go to the earlier candidate."""
    return min(timings, key=lambda c: (timings[c], list(timings).index(c)))


def autotune_batch(imgs, targets, srcs=None, candidates=None, reps: int = 2, path: str | None = None,
                   record: bool = True, log=None):
    """Time every candidate launch shape on this batch; record and return the fastest.

    imgs/targets/srcs as for api.BatchCarver.  Returns (best, {candidate: seconds}).
    """
    import torch

    from . import api
    candidates = list(candidates or BATCH_CANDIDATES)
    timings = {}
    for v, g in candidates:
        bc = api.BatchCarver(imgs, targets, srcs=srcs, record=False, team=g, variant=v)
        bc.launch()
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            t = time.perf_counter()
            bc.launch()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        if any(s != 0 for s in bc.status()):
            continue  # a shape whose team could not be placed is not a candidate
        timings[(v, g)] = best
        if log:
            log(f"batch v{v} team {g}: {best * 1e3:.1f} ms")
    best = pick(timings)
    if record:
        key = key_batch(device_arch(imgs[0].device), [(t.shape[0], t.shape[1]) for t in imgs])
        save({key: {"variant": best[0], "team": best[1], "ms": round(timings[best] * 1e3, 3),
                    "candidates": {f"v{v}/g{g}": round(s * 1e3, 3) for (v, g), s in timings.items()}}}, path)
    return best, timings


def autotune_single(img, target_w: int, src=None, candidates=None, reps: int = 2, path: str | None = None,
                    record: bool = True, log=None):
    """Time every candidate on one image carve; record and return the fastest."""
    import torch

    from . import _lib, api
    candidates = list(candidates or SINGLE_CANDIDATES)
    H, W, C = img.shape
    ws = api.workspace(_lib.load().sc_workspace_bytes(H, W, C), img.device)
    src = img.clone() if src is None else src
    timings = {}
    for v, g in candidates:
        api.carve(img, target_w, src=src, record=False, team=g, variant=v, ws=ws)
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            t = time.perf_counter()
            api.carve(img, target_w, src=src, record=False, team=g, variant=v, ws=ws)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        if api.read_status(ws, 1) != [0]:
            continue
        timings[(v, g)] = best
        if log:
            log(f"single {H}x{W} v{v} team {g}: {best * 1e3:.1f} ms")
    best = pick(timings)
    if record:
        save({key_single(device_arch(img.device), H, W): {
            "variant": best[0], "team": best[1], "ms": round(timings[best] * 1e3, 3),
            "candidates": {f"v{v}/g{g}": round(s * 1e3, 3) for (v, g), s in timings.items()}}}, path)
    return best, timings


def main():
    ap = argparse.ArgumentParser(description="autotune the carve launch shape on this GPU")
    ap.add_argument("--out", default=None, help="cache file (default: the package's tune_cache.json)")
    args = ap.parse_args()
    import sys

    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import synth

    def log(m):
        print(m, flush=True)

    dev = torch.device("cuda")
    # batched workload: 256 blob images, H, W ~ U[240, 2160], 10-40 % of the width removed (seed 3)
    jobs = synth.batch_jobs(n=256)
    srcs = [torch.from_numpy(j.image()).to(dev) for j in jobs]
    imgs = [torch.empty_like(s) for s in srcs]
    best, _ = autotune_batch(imgs, [j.target_w for j in jobs], srcs=srcs, path=args.out, log=log)
    log(f"batch best: variant {best[0]}, team {best[1]}")
    del srcs, imgs
    # single images: 1920x1080 (480 seams) and 3840x2160 (960 seams), blob seeds 1 and 2
    for (h, w, tw, seed) in [(1080, 1920, 1440, 1), (2160, 3840, 2880, 2)]:
        img = torch.from_numpy(synth.blob_image(h, w, 3, seed=seed)).to(dev)
        best, _ = autotune_single(torch.empty_like(img), tw, src=img, path=args.out, log=log)
        log(f"single {h}x{w} best: variant {best[0]}, team {best[1]}")
    print(json.dumps(load(args.out or cache_path()), indent=1), flush=True)


if __name__ == "__main__":
    main()
