"""Torch-facing helpers over the C ABI (PyTorch is used only for device memory and streams).

Images are CUDA/HIP uint8 tensors [H, W, C] whose rows may be padded (stride(0) = pitch
bytes, stride(1) = C, stride(2) = 1).  Every function here only marshals arguments into the
C entry points of libseamcarve.so; all computation happens in its HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib

__all__ = ["energy", "dp_seam", "remove_seam", "transpose", "carve", "carve_hv", "insert_seams", "workspace",
           "BatchCarver", "variants", "read_status", "read_times", "read_stages", "remove_object"]


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _image(t: torch.Tensor, name="img"):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.dim() != 3 or not t.is_cuda:
        raise ValueError(f"{name} must be a uint8 [H, W, C] tensor on the GPU")
    H, W, C = t.shape
    if t.stride(2) != 1 or t.stride(1) != C:
        raise ValueError(f"{name} pixels must be packed (stride(1) == C, stride(2) == 1)")
    return H, W, C, t.stride(0)


def _check_status(ws: torch.Tensor, n: int, what: str):
    """Raise ScError when any image of the workspace reports a device-side failure (a team barrier
    that timed out, a team not placed on one XCD): its results are then invalid."""
    flags = read_status(ws, n)
    bad = [(i, f) for i, f in enumerate(flags) if f]
    if bad:
        raise _lib.ScError(_lib.SC_EHIP, what, f"device status of images {bad[:8]} (1 = team barrier timed out, "
                                              "2 = team not on one XCD): results invalid")


def workspace(nbytes: int, device) -> torch.Tensor:
    """A fresh byte buffer for a workspace (the caching allocator aligns blocks to >= 512 B)."""
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def variants():
    lib = _lib.load()
    return [lib.sc_variant_name(v).decode() for v in range(lib.sc_variant_count())]


def energy(img: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """e1 energy map, int32 [H, W]."""
    H, W, C, pitch = _image(img)
    if out is None:
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _lib.call("sc_energy", _ptr(img), H, W, C, pitch, _ptr(out), _stream(stream))
    return out


def dp_seam(e: torch.Tensor, dirs: bool = False, ws: torch.Tensor | None = None, stream=None, check: bool = True):
    """Minimum vertical seam of an int32 [H, W] energy map -> (seam int32 [H], cost int64 [1][, dirs uint8 [H, W]]).

    check: read the device status afterwards (synchronises) and raise ScError on a device failure."""
    if e.dtype != torch.int32 or e.dim() != 2 or not e.is_cuda:
        raise ValueError("energy must be an int32 [H, W] GPU tensor")
    e = e.contiguous()
    H, W = e.shape
    lib = _lib.load()
    need = lib.sc_workspace_bytes(H, W, 1)
    if ws is None or ws.numel() < need:
        ws = workspace(need, e.device)
    seam = torch.empty(H, dtype=torch.int32, device=e.device)
    cost = torch.empty(1, dtype=torch.int64, device=e.device)
    d = torch.empty((H, W), dtype=torch.uint8, device=e.device) if dirs else None
    _lib.call("sc_dp_seam", _ptr(e), H, W, _ptr(seam), _ptr(cost), _ptr(ws), ws.numel(), _stream(stream), _ptr(d))
    if check:
        _check_status(ws, 1, "sc_dp_seam")
    return (seam, cost, d) if dirs else (seam, cost)


def remove_seam(img: torch.Tensor, seam: torch.Tensor, stream=None) -> torch.Tensor:
    """Remove one vertical seam in place; returns the view img[:, :W-1]."""
    H, W, C, pitch = _image(img)
    if seam.dtype != torch.int32 or seam.numel() != H or not seam.is_cuda:
        raise ValueError("seam must be an int32 [H] GPU tensor")
    _lib.call("sc_remove_seam", _ptr(img), H, W, C, pitch, _ptr(seam.contiguous()), _stream(stream))
    return img[:, : W - 1]


def transpose(img: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """J(x, y, c) = I(y, x, c) -> uint8 [W, H, C]."""
    H, W, C, pitch = _image(img)
    if out is None:
        out = torch.empty((W, H, C), dtype=torch.uint8, device=img.device)
    _, _, _, opitch = _image(out, "out")
    _lib.call("sc_transpose_u8", _ptr(img), H, W, C, pitch, _ptr(out), opitch, _stream(stream))
    return out


_arch: dict = {}


def _tuned(device, key_fn):
    """(variant, team) the autotuner recorded for this device and size bucket, else (None, None)."""
    from . import tune
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _arch:
        _arch[idx] = tune.device_arch(idx)
    hit = tune.lookup(key_fn(_arch[idx]))
    return hit if hit else (None, None)


def _tune(team=None, variant=None, minside=True, xcd=0):
    if team is None and variant is None and minside and not xcd:
        return None
    return ctypes.byref(_lib.sc_tune(team or 0, -1 if variant is None else variant,
                                     (0 if minside else _lib.SC_TUNE_NO_MINSIDE) | ((xcd & 7) << _lib.SC_TUNE_XCD_SHIFT)))


def carve(img: torch.Tensor, target_w: int, src: torch.Tensor | None = None, record: bool = True,
          team: int | None = None, variant: int | None = None, ws: torch.Tensor | None = None, stream=None,
          minside: bool = True, check: bool = True):
    """Carve `img` to target_w columns (in place; from `src` when given).

    Returns (img[:, :target_w], seams int32 [k, H] or None, costs int64 [k] or None).
    check: read the device status afterwards (synchronises the device) and raise ScError when the
    carve failed on the device; with check=False the caller reads it (read_status on `ws`).
    """
    H, W, C, pitch = _image(img)
    if src is not None:
        sH, sW, sC, spitch = _image(src, "src")
        if (sH, sW, sC, spitch) != (H, W, C, pitch):
            raise ValueError("src must have the shape and pitch of img")
    if team is None and variant is None:  # the autotuner's choice for this size, if any
        from . import tune
        variant, team = _tuned(img.device, lambda a: tune.key_single(a, H, W))
    k = W - int(target_w)
    lib = _lib.load()
    need = lib.sc_workspace_bytes(H, W, C)
    if ws is None or ws.numel() < need:
        ws = workspace(need, img.device)
    seams = costs = None
    if record and k > 0:
        seams = torch.empty((k, H), dtype=torch.int32, device=img.device)
        costs = torch.empty(k, dtype=torch.int64, device=img.device)
    _lib.call("sc_carve", _ptr(img), H, W, C, int(target_w), pitch, _ptr(seams), _ptr(costs), _ptr(ws), ws.numel(),
              _stream(stream), _ptr(src), _tune(team, variant, minside))
    if check:
        _check_status(ws, 1, "sc_carve")
    return img[:, : int(target_w)], seams, costs


def carve_forward(img: torch.Tensor, target_w: int, src: torch.Tensor | None = None, record: bool = True,
                  ws: torch.Tensor | None = None, stream=None):
    """Carve `img` to target_w columns with forward-energy seams (in place; from `src` when given).

    Returns (img[:, :target_w], seams int32 [k, H] or None, costs int64 [k] or None).
    """
    H, W, C, pitch = _image(img)
    if src is not None and _image(src, "src") != (H, W, C, pitch):
        raise ValueError("src must have the shape and pitch of img")
    k = W - int(target_w)
    need = _lib.load().sc_forward_workspace_bytes(H, W, C)
    if ws is None or ws.numel() < need:
        ws = workspace(need, img.device)
    seams = costs = None
    if record and k > 0:
        seams = torch.empty((k, H), dtype=torch.int32, device=img.device)
        costs = torch.empty(k, dtype=torch.int64, device=img.device)
    _lib.call("sc_carve_forward", _ptr(img), H, W, C, int(target_w), pitch, _ptr(seams), _ptr(costs), _ptr(ws),
              ws.numel(), _stream(stream), _ptr(src))
    return img[:, : int(target_w)], seams, costs


def insert_seams(img: torch.Tensor, k: int, out: torch.Tensor | None = None, record: bool = True,
                 team: int | None = None, variant: int | None = None, ws: torch.Tensor | None = None, stream=None,
                 check: bool = True):
    """Widen `img` by k seams (img is not modified).

    Returns (out [H, W + k, C], original seam columns int32 [k, H] or None).
    check: as in carve (the seam search is a carve whose workspace starts the insertion workspace).
    """
    H, W, C, pitch = _image(img)
    k = int(k)
    if out is None:
        out = torch.empty((H, W + k, C), dtype=torch.uint8, device=img.device)
    oH, oW, oC, opitch = _image(out, "out")
    if (oH, oW, oC) != (H, W + k, C):
        raise ValueError(f"out must be [{H}, {W + k}, {C}]")
    if team is None and variant is None:  # the seams come from a carve: use its tuned shape
        from . import tune
        variant, team = _tuned(img.device, lambda a: tune.key_single(a, H, W))
    lib = _lib.load()
    need = lib.sc_insert_workspace_bytes(H, W, C, pitch, k)
    if need == 0:
        raise ValueError(f"bad insertion: H={H}, W={W}, C={C}, k={k}")
    if ws is None or ws.numel() < need:
        ws = workspace(need, img.device)
    seams = torch.empty((k, H), dtype=torch.int32, device=img.device) if record and k > 0 else None
    _lib.call("sc_insert_seams", _ptr(img), H, W, C, pitch, k, _ptr(out), opitch, _ptr(seams),
              _tune(team, variant), _ptr(ws), ws.numel(), _stream(stream))
    if check and k > 0:
        _check_status(ws, 1, "sc_insert_seams")
    return out, seams


def carve_hv(img: torch.Tensor, target_w: int, target_h: int, record: bool = True, team=None, variant=None,
             stream=None):
    """Vertical seams to target_w (in place), then horizontal seams via a transpose to target_h.

    Returns (out [target_h, target_w, C] new tensor, vseams, vcosts, hseams, hcosts).
    """
    H, W, C, _ = _image(img)
    a, vs, vc = carve(img, target_w, record=record, team=team, variant=variant, stream=stream)
    t = transpose(a, stream=stream)                       # [target_w, H, C]
    b, hs, hc = carve(t, target_h, record=record, team=team, variant=variant, stream=stream)
    out = transpose(b, stream=stream)                     # [target_h, target_w, C]
    return out, vs, vc, hs, hc


def remove_object(img: torch.Tensor, mask: torch.Tensor, direction: int = _lib.SC_OBJ_AUTO, restore: bool = False,
                  record: bool = True, ws: torch.Tensor | None = None, stream=None):
    """Remove the object under `mask` (uint8 [H, W] on the GPU, nonzero = object) from `img`
    (sc_remove_object; synchronous).  direction: -1 = from the mask's extent, 0 = vertical seams,
    1 = horizontal seams.  restore: insert as many seams afterwards to get the size back.

    Returns (out [rows, cols, C] view of a new tensor, info dict, seams int32 [k, h] or None,
    costs int64 [k] or None); h = H for vertical seams, W for horizontal ones.
    """
    H, W, C, pitch = _image(img)
    if (not isinstance(mask, torch.Tensor) or mask.dtype != torch.uint8 or mask.dim() != 2 or not mask.is_cuda
            or tuple(mask.shape) != (H, W) or mask.stride(1) != 1):
        raise ValueError("mask must be a uint8 [H, W] GPU tensor with unit column stride")
    lib = _lib.load()
    need = lib.sc_object_workspace_bytes(H, W, C, int(bool(restore)))
    if ws is None or ws.numel() < need:
        ws = workspace(need, img.device)
    out = torch.empty((H, W, C), dtype=torch.uint8, device=img.device)
    seams = costs = None
    if record:
        seams = torch.empty(H * W, dtype=torch.int32, device=img.device)
        costs = torch.empty(max(H, W), dtype=torch.int64, device=img.device)
    info = _lib.sc_object_info()
    _lib.call("sc_remove_object", _ptr(img), _ptr(mask), H, W, C, pitch, mask.stride(0), int(direction),
              int(bool(restore)), _ptr(out), W * C, ctypes.byref(info), _ptr(seams), _ptr(costs), _ptr(ws),
              ws.numel(), _stream(stream))
    d = {"direction": info.direction, "k": info.k, "rows": info.rows, "cols": info.cols, "left": info.left,
         "carve_ms": info.carve_ms, "stage_ms": list(info.stage_ms)}
    h = H if info.direction == _lib.SC_OBJ_VERTICAL else W
    if record:
        seams = seams[: info.k * h].view(info.k, h)
        costs = costs[: info.k]
    return out[: info.rows, : info.cols], d, seams, costs


def read_status(ws: torch.Tensor, n: int = 1):
    """Device status flags of the images of a workspace (synchronises the device)."""
    flags = (ctypes.c_uint32 * n)()
    got = _lib.load().sc_read_status(_ptr(ws), flags, n)
    if got < 0:
        raise _lib.ScError(got, "sc_read_status", _lib.load().sc_last_error().decode())
    return list(flags)[:got]


def read_times(ws: torch.Tensor, n: int = 1):
    """[(t_begin_s, t_end_s)] per image of the last carve in this workspace (synchronises)."""
    tb = (ctypes.c_uint64 * n)()
    te = (ctypes.c_uint64 * n)()
    hz = ctypes.c_double(0)
    got = _lib.load().sc_read_times(_ptr(ws), tb, te, n, ctypes.byref(hz))
    if got < 0:
        raise _lib.ScError(got, "sc_read_times", _lib.load().sc_last_error().decode())
    return [(tb[i] / hz.value, te[i] / hz.value) for i in range(got)]


def read_stages(ws: torch.Tensor, n: int = 1):
    """Seconds each image spent in (DP sweep, backtrack + removal, band update), summed over seams."""
    out = (ctypes.c_uint64 * (3 * n))()
    got = _lib.load().sc_read_stages(_ptr(ws), out, n)
    if got < 0:
        raise _lib.ScError(got, "sc_read_stages", _lib.load().sc_last_error().decode())
    hz = read_times_hz(ws)
    return [tuple(out[3 * i + j] / hz for j in range(3)) for i in range(got)]


def read_times_hz(ws: torch.Tensor) -> float:
    tb = (ctypes.c_uint64 * 1)()
    te = (ctypes.c_uint64 * 1)()
    hz = ctypes.c_double(0)
    _lib.load().sc_read_times(_ptr(ws), tb, te, 1, ctypes.byref(hz))
    return hz.value or 100e6


@dataclass
class _Job:
    src: torch.Tensor | None
    img: torch.Tensor
    target_w: int
    seams: torch.Tensor | None
    costs: torch.Tensor | None


class BatchCarver:
    """Carve many images of uneven sizes in one persistent launch.

    ``prepare()`` plans the launch (synchronous upload of the plan into the workspace);
    ``launch()`` enqueues it (no host-to-device copy, no allocation), so it can be captured
    in a HIP graph with ``capture()`` and replayed with ``replay()``.
    """

    def __init__(self, imgs, targets, srcs=None, record: bool = True, team: int | None = None,
                 variant: int | None = None, minside: bool = True):
        self.jobs = []
        for i, (img, tw) in enumerate(zip(imgs, targets)):
            H, W, C, pitch = _image(img)
            src = None if srcs is None else srcs[i]
            if src is not None and _image(src, "src") != (H, W, C, pitch):
                raise ValueError("src must have the shape and pitch of img")
            k = W - int(tw)
            seams = torch.empty((k, H), dtype=torch.int32, device=img.device) if record and k > 0 else None
            costs = torch.empty(k, dtype=torch.int64, device=img.device) if record and k > 0 else None
            self.jobs.append(_Job(src, img, int(tw), seams, costs))
        n = len(self.jobs)
        if team is None and variant is None:  # the autotuner's choice for this batch shape, if any
            from . import tune
            shapes = [(j.img.shape[0], j.img.shape[1]) for j in self.jobs]
            variant, team = _tuned(self.jobs[0].img.device, lambda a: tune.key_batch(a, shapes))
        self.tuned = (variant, team)
        self._cjobs = (_lib.sc_job * n)()
        for i, j in enumerate(self.jobs):
            H, W, C, pitch = _image(j.img)
            self._cjobs[i] = _lib.sc_job(j.img.data_ptr(), H, W, C, pitch, j.target_w,
                                         None if j.seams is None else j.seams.data_ptr(),
                                         None if j.costs is None else j.costs.data_ptr(),
                                         None if j.src is None else j.src.data_ptr())
        self._tune = _lib.sc_tune(team or 0, -1 if variant is None else variant,
                                  0 if minside else _lib.SC_TUNE_NO_MINSIDE)
        need = _lib.load().sc_batch_workspace_bytes(self._cjobs, n)
        if need == 0:
            raise ValueError("bad batch")
        self.ws = workspace(need, self.jobs[0].img.device)
        self.info = _lib.sc_batch_info()
        self.graph = None
        self.prepare()

    def prepare(self):
        _lib.call("sc_batch_prepare", self._cjobs, len(self.jobs), ctypes.byref(self._tune), _ptr(self.ws),
                  self.ws.numel(), ctypes.byref(self.info))

    def launch(self, stream=None):
        _lib.call("sc_batch_launch", ctypes.byref(self.info), _ptr(self.ws), _stream(stream))

    def launch_energy(self, stream=None):
        _lib.call("sc_batch_launch_energy", ctypes.byref(self.info), _ptr(self.ws), _stream(stream))

    def launch_carve(self, stream=None):
        _lib.call("sc_batch_launch_carve", ctypes.byref(self.info), _ptr(self.ws), _stream(stream))

    def times(self):
        """Per-image (begin, end) of the last carve in seconds of the device clock."""
        return read_times(self.ws, len(self.jobs))

    def stages(self):
        """Per-image seconds in (DP sweep, backtrack + removal, band update) of the last carve."""
        return read_stages(self.ws, len(self.jobs))

    def capture(self):
        """Capture launch() in a CUDA/HIP graph (requires every job to have a src)."""
        if any(j.src is None for j in self.jobs):
            raise ValueError("graph replay needs src images (in-place jobs would be carved twice)")
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.graph.capture_begin()
            self.launch(stream=s)
            self.graph.capture_end()
        torch.cuda.current_stream().wait_stream(s)
        return self.graph

    def replay(self):
        self.graph.replay()

    def results(self, check: bool = True):
        """[(img[:, :target_w], seams, costs)] per job.  check: read the device status first
        (synchronises) and raise ScError if any image failed on the device."""
        if check:
            _check_status(self.ws, len(self.jobs), "sc_batch_launch")
        return [(j.img[:, : j.target_w], j.seams, j.costs) for j in self.jobs]

    def status(self):
        return read_status(self.ws, len(self.jobs))


class ForwardBatch:
    """Forward-energy carve of many images of uneven sizes, each by a team of workgroups on one XCD.

    ``prepare()`` uploads the image descriptors (synchronous); ``launch()`` enqueues the copy-in
    pass and the carve with no host-to-device copy and no allocation.
    """

    def __init__(self, imgs, targets, srcs=None, record: bool = True):
        self.jobs = []
        for i, (img, tw) in enumerate(zip(imgs, targets)):
            H, W, C, pitch = _image(img)
            src = None if srcs is None else srcs[i]
            if src is not None and _image(src, "src") != (H, W, C, pitch):
                raise ValueError("src must have the shape and pitch of img")
            k = W - int(tw)
            seams = torch.empty((k, H), dtype=torch.int32, device=img.device) if record and k > 0 else None
            costs = torch.empty(k, dtype=torch.int64, device=img.device) if record and k > 0 else None
            self.jobs.append(_Job(src, img, int(tw), seams, costs))
        n = len(self.jobs)
        self._cjobs = (_lib.sc_job * n)()
        for i, j in enumerate(self.jobs):
            H, W, C, pitch = _image(j.img)
            self._cjobs[i] = _lib.sc_job(j.img.data_ptr(), H, W, C, pitch, j.target_w,
                                         None if j.seams is None else j.seams.data_ptr(),
                                         None if j.costs is None else j.costs.data_ptr(),
                                         None if j.src is None else j.src.data_ptr())
        need = _lib.load().sc_forward_batch_workspace_bytes(self._cjobs, n)
        if need == 0:
            raise ValueError("bad batch")
        self.ws = workspace(need, self.jobs[0].img.device)
        self.info = _lib.sc_batch_info()
        self.prepare()

    def prepare(self):
        _lib.call("sc_forward_batch_prepare", self._cjobs, len(self.jobs), _ptr(self.ws), self.ws.numel(),
                  ctypes.byref(self.info))

    def launch(self, stream=None):
        _lib.call("sc_forward_batch_launch", ctypes.byref(self.info), _ptr(self.ws), _stream(stream))

    def launch_copy(self, stream=None):
        _lib.call("sc_forward_batch_launch_copy", ctypes.byref(self.info), _ptr(self.ws), _stream(stream))

    def launch_carve(self, stream=None):
        _lib.call("sc_forward_batch_launch_carve", ctypes.byref(self.info), _ptr(self.ws), _stream(stream))

    def times(self):
        """Per-image (begin, end) of the last carve in seconds of the device clock."""
        return read_times(self.ws, len(self.jobs))

    def stages(self):
        """Per-image seconds in (DP sweep, argmin + backtrack, removal) of the last carve."""
        return read_stages(self.ws, len(self.jobs))

    def results(self, check: bool = True):
        if check:
            _check_status(self.ws, len(self.jobs), "sc_forward_batch_launch")
        return [(j.img[:, : j.target_w], j.seams, j.costs) for j in self.jobs]
