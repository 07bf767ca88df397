"""CPU checks of the C ABI: the library loads, exports every symbol include/sc.h declares, and
rejects bad arguments before touching a device (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2410_21207_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "sc.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} declared in sc.h but not exported"
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_struct_sizes_match_header(lib):
    assert ctypes.sizeof(_lib.sc_job) == 8 + 5 * 4 + 4 + 8 + 8 + 8  # padding after target_w
    assert [f[0] for f in _lib.sc_job._fields_][:8] == ["img", "H", "W", "C", "pitch", "target_w", "seams_out",
                                                       "costs_out"]
    assert [f[0] for f in _lib.sc_batch_info._fields_][4:6] == ["team", "teams_used"]
    assert ctypes.sizeof(_lib.sc_tune) == 12
    assert ctypes.sizeof(_lib.sc_batch_info) == 6 * 4 + 4 * 8


def test_workspace_sizes(lib):
    assert lib.sc_workspace_bytes(0, 10, 3) == 0
    assert lib.sc_workspace_bytes(10, 10, 5) == 0
    a = lib.sc_workspace_bytes(1080, 1920, 3)
    b = lib.sc_workspace_bytes(2160, 3840, 3)
    assert a > 1080 * 1920 * 2 and b > 4 * a * 0.9 and a % 256 == 0


def test_variants(lib):
    n = lib.sc_variant_count()
    assert n >= 1
    assert all(lib.sc_variant_name(v) for v in range(n))
    assert lib.sc_variant_name(n) == b""


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("args,code", [
    ((FAKE, 0, 5, 3, 15, FAKE, None), _lib.SC_EINVAL),          # H < 1
    ((FAKE, 5, 5, 5, 25, FAKE, None), _lib.SC_EINVAL),          # C > 4
    ((FAKE, 5, 5, 3, 14, FAKE, None), _lib.SC_EINVAL),          # pitch < W*C
    ((None, 5, 5, 3, 15, FAKE, None), _lib.SC_EINVAL),          # null image
    ((FAKE, 5483, 5, 3, 15, FAKE, None), _lib.SC_EUNSUPPORTED),  # column cost > 23 bits
])
def test_energy_validation(lib, args, code):
    assert lib.sc_energy(*args) == code
    assert lib.sc_last_error()


def carve(lib, img, H, W, C, tw, pitch, ws, ws_bytes, tune=None, src=None):
    # the problem's arguments first (img, H, W, C, target_w, pitch, outputs, workspace, stream),
    # then the trailing plumbing (src, tune)
    return lib.sc_carve(img, H, W, C, tw, pitch, None, None, ws, ws_bytes, None, src, tune)


def test_carve_signature_order():
    """sc_carve's leading arguments are the problem statement's, in its order (img, H, W, C,
    target_w, pitch, seams_out, costs_out, ws, ws_bytes, stream); src and tune trail."""
    with open(os.path.join(ROOT, "include", "sc.h")) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    decl = re.search(r"sc_status\s+sc_carve\s*\(([^)]*)\)", text).group(1)
    names = [re.findall(r"(\w+)\s*$", a.strip())[0] for a in decl.split(",")]
    assert names == ["img", "H", "W", "C", "target_w", "pitch", "seams_out", "costs_out", "ws", "ws_bytes",
                     "stream", "src", "tune"]
    decl = re.search(r"sc_status\s+sc_dp_seam\s*\(([^)]*)\)", text).group(1)
    names = [re.findall(r"(\w+)\s*$", a.strip())[0] for a in decl.split(",")]
    assert names == ["energy", "H", "W", "seam", "cost", "ws", "ws_bytes", "stream", "dirs_out"]


def test_carve_validation(lib):
    ws = FAKE
    assert carve(lib, FAKE, 10, 10, 3, 0, 30, ws, 1 << 30) == _lib.SC_EINVAL
    assert carve(lib, FAKE, 10, 10, 3, 11, 30, ws, 1 << 30) == _lib.SC_EINVAL
    assert carve(lib, FAKE, 10, 10, 3, 5, 30, ws, 10) == _lib.SC_ENOMEM
    assert b"workspace" in lib.sc_last_error()
    assert carve(lib, FAKE, 10, 10, 3, 5, 30, ctypes.c_void_p(0x1001), 1 << 30) == _lib.SC_EINVAL  # misaligned ws
    assert carve(lib, FAKE, 10, 10, 3, 5, 29, ws, 1 << 30) == _lib.SC_EINVAL  # pitch < W * C
    assert carve(lib, None, 10, 10, 3, 5, 30, ws, 1 << 30) == _lib.SC_EINVAL  # null image
    bad = _lib.sc_tune(1, 99)
    assert carve(lib, FAKE, 10, 10, 3, 5, 30, ws, 1 << 30, ctypes.byref(bad)) == _lib.SC_EINVAL
    big = _lib.sc_tune(33, -1)
    assert carve(lib, FAKE, 10, 10, 3, 5, 30, ws, 1 << 30, ctypes.byref(big)) == _lib.SC_EUNSUPPORTED


def test_noalloc_validation(lib):
    """sc_carve_noalloc rejects bad shapes and images larger than its fixed scratch before any
    device call."""
    big = (4096, 4096, 3)
    assert lib.sc_workspace_bytes(*big) > _lib.SC_NOALLOC_SCRATCH_BYTES
    assert lib.sc_carve_noalloc(FAKE, *big, 4000, 4096 * 3, None, None, None, None, None, None) == _lib.SC_ENOMEM
    assert b"fixed scratch" in lib.sc_last_error()
    assert lib.sc_carve_noalloc(FAKE, 0, 10, 3, 5, 30, None, None, None, None, None, None) == _lib.SC_EINVAL
    assert lib.sc_carve_noalloc(FAKE, 10, 10, 3, 11, 30, None, None, None, None, None, None) == _lib.SC_EINVAL
    assert lib.sc_carve_noalloc(None, 10, 10, 3, 5, 30, None, None, None, None, None, None) == _lib.SC_EINVAL
    assert lib.sc_workspace_bytes(2160, 3840, 3) <= _lib.SC_NOALLOC_SCRATCH_BYTES  # 3840x2160 RGB fits


def test_dp_and_remove_and_transpose_validation(lib):
    assert lib.sc_dp_seam(FAKE, 4, 4, FAKE, FAKE, FAKE, 8, None, None) == _lib.SC_ENOMEM
    assert lib.sc_dp_seam(None, 4, 4, FAKE, FAKE, FAKE, 1 << 20, None, None) == _lib.SC_EINVAL
    assert lib.sc_remove_seam(FAKE, 4, 0, 3, 12, FAKE, None) == _lib.SC_EINVAL
    # overlapping transpose buffers
    assert lib.sc_transpose_u8(FAKE, 4, 4, 3, 12, ctypes.c_void_p(0x1008), 12, None) == _lib.SC_EINVAL


def test_batch_validation(lib):
    jobs = (_lib.sc_job * 2)()
    jobs[0] = _lib.sc_job(0x1000, 10, 10, 3, 30, 5, None, None, None)
    jobs[1] = _lib.sc_job(0x2000, 10, 10, 3, 30, 0, None, None, None)  # bad target
    info = _lib.sc_batch_info()
    assert lib.sc_batch_prepare(jobs, 2, None, FAKE, 1 << 30, ctypes.byref(info)) == _lib.SC_EINVAL
    assert b"job 1" in lib.sc_last_error()
    assert lib.sc_batch_workspace_bytes(jobs, 2) > 0
    assert lib.sc_batch_launch(ctypes.byref(info), FAKE, None) == _lib.SC_EINVAL  # nothing prepared


def test_insert_validation(lib):
    assert lib.sc_insert_workspace_bytes(10, 10, 3, 30, 10) == 0  # k must be < W
    assert lib.sc_insert_workspace_bytes(10, 10, 3, 20, 2) == 0   # pitch < W * C
    assert lib.sc_insert_workspace_bytes(10, 10, 3, 30, -1) == 0
    a = lib.sc_insert_workspace_bytes(1080, 1920, 3, 5760, 480)
    assert a > lib.sc_workspace_bytes(1080, 1920, 3) + 1080 * 5760 and a % 256 == 0
    big = ctypes.c_void_p(1 << 40)
    # k out of range, short output pitch, overlapping buffers, small workspace: all rejected up front
    assert lib.sc_insert_seams(FAKE, 4, 8, 3, 24, 8, big, 48, None, None, FAKE, 1 << 20, None) == _lib.SC_EINVAL
    assert lib.sc_insert_seams(FAKE, 4, 8, 3, 24, 2, big, 29, None, None, FAKE, 1 << 20, None) == _lib.SC_EINVAL
    assert lib.sc_insert_seams(FAKE, 4, 8, 3, 24, 2, ctypes.c_void_p(0x1010), 30, None, None, big, 1 << 20,
                               None) == _lib.SC_EINVAL
    assert lib.sc_insert_seams(FAKE, 4, 8, 3, 24, 2, big, 30, None, None, ctypes.c_void_p(1 << 41), 64,
                               None) == _lib.SC_ENOMEM


def test_slot_step_validation(lib):
    job = _lib.sc_job(0x1000, 10, 10, 3, 30, 5, None, None, None)
    ws = ctypes.c_void_p(1 << 40)
    for n_slots, slot in [(4, 4), (4, -1), (0, 0), (1, 7)]:  # slot outside the table
        assert lib.sc_slot_start(ctypes.byref(job), ws, 1 << 30, FAKE, n_slots, slot, None) == _lib.SC_EINVAL
        assert b"slot" in lib.sc_last_error()
        assert lib.sc_slot_clear(FAKE, n_slots, slot, None) == _lib.SC_EINVAL
    assert lib.sc_slots_step(None, 4, 16, None, None) == _lib.SC_EINVAL
    assert lib.sc_slots_step_timed(FAKE, 4, 16, -1, None, None) == _lib.SC_EINVAL
    assert lib.sc_slots_step_timed(FAKE, 0, 16, 100, None, None) == _lib.SC_EINVAL


def test_tune_flag_bits_do_not_overlap():
    flags = [_lib.SC_TUNE_NO_MINSIDE] + [x << _lib.SC_TUNE_XCD_SHIFT for x in (1, 2, 4)]
    acc = 0
    for f in flags:
        assert acc & f == 0
        acc |= f


def test_forward_validation(lib):
    assert lib.sc_forward_workspace_bytes(0, 10, 3) == 0 and lib.sc_forward_workspace_bytes(10, 10, 5) == 0
    a = lib.sc_forward_workspace_bytes(2076, 2113, 4)
    assert a % 256 == 0 and a > 2076 * 2113 * 4  # the working copy alone
    ws = ctypes.c_void_p(1 << 40)
    # width beyond the forward path, cost bound, bad target, small or misaligned workspace
    def fwd(H, W, C, tw, pitch, ws_, nbytes):
        return lib.sc_carve_forward(FAKE, H, W, C, tw, pitch, None, None, ws_, nbytes, None, None)
    assert fwd(4, 8193, 1, 8000, 8193, ws, 1 << 30) == _lib.SC_EUNSUPPORTED
    assert fwd(5483, 5, 3, 4, 15, ws, 1 << 30) == _lib.SC_EUNSUPPORTED
    assert fwd(4, 8, 3, 0, 24, ws, 1 << 20) == _lib.SC_EINVAL
    assert fwd(4, 8, 3, 9, 24, ws, 1 << 20) == _lib.SC_EINVAL
    assert fwd(4, 8, 3, 4, 24, ws, 64) == _lib.SC_ENOMEM
    assert fwd(4, 8, 3, 4, 24, ctypes.c_void_p((1 << 40) + 8), 1 << 20) == _lib.SC_EINVAL
    jobs = (_lib.sc_job * 2)()
    jobs[0] = _lib.sc_job(0x1000, 4, 8, 3, 24, 4, None, None, None)
    jobs[1] = _lib.sc_job(0x2000, 5, 9000, 1, 9000, 10, None, None, None)
    info = _lib.sc_batch_info()
    assert lib.sc_forward_batch_prepare(jobs, 2, ws, 1 << 40, ctypes.byref(info)) == _lib.SC_EUNSUPPORTED
    assert lib.sc_forward_batch_prepare(jobs, 1, ws, 64, ctypes.byref(info)) == _lib.SC_ENOMEM
    # an e1 batch plan is not a forward plan and the other way round
    info.n, info.nblocks, info.team, info.variant = 1, 1, 4, 7
    assert lib.sc_forward_batch_launch(ctypes.byref(info), ws, None) == _lib.SC_EINVAL
    info.team, info.variant = 0, 100
    assert lib.sc_batch_launch(ctypes.byref(info), ws, None) == _lib.SC_EINVAL
