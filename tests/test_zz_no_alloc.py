"""The allocation-free carve (sc_carve_noalloc: scratch in the library's fixed per-GPU array)
against sc_carve with a caller workspace, through the C ABI: two calls in a row on one GPU, the
second on a smaller image, each bit-exact (seams, costs, pixels) and with a clean device status."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import dev, host, log

pytestmark = pytest.mark.gpu

from paper_2410_21207_amd import _lib, api  # noqa: E402  (a missing library fails these tests)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _noalloc(img_np, target_w):
    H, W, C = img_np.shape
    k = W - target_w
    src = dev(img_np)
    out = torch.full_like(src, 0x5A)  # stale bytes: only the carved columns are compared
    seams = torch.full((k, H), -7, dtype=torch.int32, device="cuda")
    costs = torch.full((k,), -7, dtype=torch.int64, device="cuda")
    status = torch.full((1,), 0xFFFF, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib = _lib.load()
    _lib.check(lib.sc_carve_noalloc(_p(out), H, W, C, target_w, W * C, _p(seams), _p(costs), _p(status), stream,
                                    _p(src), None), "sc_carve_noalloc")
    return host(out[:, :target_w]), host(seams), host(costs), int(host(status)[0])


def _with_workspace(img_np, target_w):
    src = dev(img_np)
    out, seams, costs = api.carve(torch.empty_like(src), target_w, src=src)  # checks the device status
    return host(out), host(seams), host(costs)


@pytest.mark.parametrize("shapes", [[(720, 1280, 3, 960, 11), (200, 300, 3, 230, 12)]])
def test_noalloc_matches_carve_twice(shapes):
    for H, W, C, tw, seed in shapes:  # the second call is smaller and reuses the same scratch
        img = synth.blob_image(H, W, C, seed=seed)
        log("noalloc carve", W, "x", H, "->", tw)
        n_out, n_seams, n_costs, st = _noalloc(img, tw)
        r_out, r_seams, r_costs = _with_workspace(img, tw)
        assert st == 0, f"device status {st:#x}"
        assert np.array_equal(n_seams, r_seams), "seams differ"
        assert np.array_equal(n_costs, r_costs), "costs differ"
        assert np.array_equal(n_out, r_out), "pixels differ"


def test_noalloc_rejects_oversize():
    lib = _lib.load()
    H, W, C = 4096, 4096, 3
    assert lib.sc_workspace_bytes(H, W, C) > _lib.SC_NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)
    rc = lib.sc_carve_noalloc(fake, H, W, C, W - 1, W * C, None, None, None, None, None, None)
    assert rc == _lib.SC_ENOMEM and b"fixed scratch" in lib.sc_last_error()
