"""ctypes binding of libseamcarve.so: the C ABI of include/sc.h, same names, argument marshalling only.

Every step of the seam-carving path runs in the library's HIP kernels.  There is no
fallback: if the library is missing or cannot be loaded this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseamcarve.so")

SC_OK, SC_EINVAL, SC_ENOMEM, SC_EHIP, SC_EBUSY, SC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
_NAMES = {0: "SC_OK", -1: "SC_EINVAL", -2: "SC_ENOMEM", -3: "SC_EHIP", -4: "SC_EBUSY", -5: "SC_EUNSUPPORTED"}

P, I, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t


class sc_tune(ctypes.Structure):
    _fields_ = [("team", ctypes.c_int), ("variant", ctypes.c_int), ("flags", ctypes.c_int)]


SC_TUNE_NO_MINSIDE = 1
SC_TUNE_XCD_SHIFT = 8
SC_NOALLOC_SCRATCH_BYTES = 64 << 20


class sc_job(ctypes.Structure):
    _fields_ = [("img", P), ("H", I), ("W", I), ("C", I), ("pitch", I), ("target_w", I),
                ("seams_out", P), ("costs_out", P), ("src", P)]


class sc_batch_info(ctypes.Structure):
    _fields_ = [("n", I), ("nblocks", I), ("variant", I), ("max_rows", I), ("team", I), ("teams_used", I),
                ("off_imgs", Z), ("off_blk", Z), ("off_teams", Z), ("off_team_imgs", Z)]


class sc_object_info(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("k", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("left", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("carve_ms", ctypes.c_double), ("stage_ms", ctypes.c_double * 3)]


SC_OBJ_AUTO, SC_OBJ_VERTICAL, SC_OBJ_HORIZONTAL = -1, 0, 1

# name -> (restype, argtypes); exactly the functions declared in include/sc.h
SIGNATURES = {
    "sc_last_error": (ctypes.c_char_p, []),
    "sc_version": (ctypes.c_char_p, []),
    "sc_workspace_bytes": (Z, [I, I, I]),
    "sc_energy": (I, [P, I, I, I, I, P, P]),
    "sc_dp_seam": (I, [P, I, I, P, P, P, Z, P, P]),
    "sc_remove_seam": (I, [P, I, I, I, I, P, P]),
    "sc_transpose_u8": (I, [P, I, I, I, I, P, I, P]),
    "sc_variant_count": (I, []),
    "sc_variant_name": (ctypes.c_char_p, [I]),
    "sc_carve": (I, [P, I, I, I, I, I, P, P, P, Z, P, P, ctypes.POINTER(sc_tune)]),
    "sc_carve_noalloc": (I, [P, I, I, I, I, I, P, P, P, P, P, ctypes.POINTER(sc_tune)]),
    "sc_insert_workspace_bytes": (Z, [I, I, I, I, I]),
    "sc_insert_seams": (I, [P, I, I, I, I, I, P, I, P, ctypes.POINTER(sc_tune), P, Z, P]),
    "sc_batch_workspace_bytes": (Z, [ctypes.POINTER(sc_job), I]),
    "sc_batch_prepare": (I, [ctypes.POINTER(sc_job), I, ctypes.POINTER(sc_tune), P, Z,
                             ctypes.POINTER(sc_batch_info)]),
    "sc_batch_launch": (I, [ctypes.POINTER(sc_batch_info), P, P]),
    "sc_batch_launch_energy": (I, [ctypes.POINTER(sc_batch_info), P, P]),
    "sc_batch_launch_carve": (I, [ctypes.POINTER(sc_batch_info), P, P]),
    "sc_carve_batch": (I, [ctypes.POINTER(sc_job), I, ctypes.POINTER(sc_tune), P, Z, P]),
    "sc_forward_workspace_bytes": (Z, [I, I, I]),
    "sc_carve_forward": (I, [P, I, I, I, I, I, P, P, P, Z, P, P]),
    "sc_forward_batch_workspace_bytes": (Z, [ctypes.POINTER(sc_job), I]),
    "sc_forward_batch_prepare": (I, [ctypes.POINTER(sc_job), I, P, Z, ctypes.POINTER(sc_batch_info)]),
    "sc_forward_batch_launch": (I, [ctypes.POINTER(sc_batch_info), P, P]),
    "sc_forward_batch_launch_copy": (I, [ctypes.POINTER(sc_batch_info), P, P]),
    "sc_forward_batch_launch_carve": (I, [ctypes.POINTER(sc_batch_info), P, P]),
    "sc_read_status": (I, [P, ctypes.POINTER(ctypes.c_uint32), I]),
    "sc_read_times": (I, [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), I,
                          ctypes.POINTER(ctypes.c_double)]),
    "sc_read_stages": (I, [P, ctypes.POINTER(ctypes.c_uint64), I]),
    "sc_object_workspace_bytes": (Z, [I, I, I, I]),
    "sc_remove_object": (I, [P, P, I, I, I, I, I, I, I, P, I, ctypes.POINTER(sc_object_info), P, P, P, Z, P]),
    "sc_slot_table_bytes": (Z, [I]),
    "sc_slot_start": (I, [ctypes.POINTER(sc_job), P, Z, P, I, I, P]),
    "sc_slot_clear": (I, [P, I, I, P]),
    "sc_slots_step": (I, [P, I, I, P, P]),
    "sc_slots_step_timed": (I, [P, I, I, ctypes.c_longlong, P, P]),
    "sc_slots_step_teams": (I, [P, I, I, ctypes.POINTER(ctypes.c_int32), I, ctypes.c_longlong, P, P]),
}

_lib = None


class ScError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} failed: {_NAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libseamcarve.so (built in-tree by paper_2410_21207_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first with `python -m paper_2410_21207_amd.build` "
                          "(the seam-carving path has no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int, fn: str):
    if rc != SC_OK:
        raise ScError(rc, fn, load().sc_last_error().decode())
    return rc


def call(name: str, *args, checked: bool = True):
    """Call C function `name`; raise ScError on a negative status when `checked`."""
    rc = getattr(load(), name)(*args)
    if checked and SIGNATURES[name][0] is I:
        check(rc, name)
    return rc
