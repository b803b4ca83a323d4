"""ctypes binding of ``libtsr.so`` (the C ABI declared in ``include/tsr.h``).

Argument marshalling only: every step of the rasterizer runs in the HIP kernels behind the
C ABI.  The library must have been built (``paper_2605_31419_amd.build``); loading fails
loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# $TSR_LIB selects another build of the same ABI (e.g. a compile-time variant being timed)
LIB_PATH = os.environ.get("TSR_LIB") or os.path.join(HERE, "libtsr.so")

TSR_OK = 0
TSR_EINVAL = -1
TSR_EWORKSPACE = -2
TSR_ECAPACITY = -3
TSR_EHIP = -4
TSR_EINTERNAL = -5
TSR_MAX_VIEWS = 32
TSR_EQUI_NOALLOC_MAX_FACES = 4194304
TSR_TILE = 16

EXPORTED = ["tsr_workspace_size", "tsr_workspace_init", "tsr_bin_and_sort", "tsr_count", "tsr_binning_view", "tsr_render_forward",
            "tsr_render_backward", "tsr_render_train_l1", "tsr_pose_step", "tsr_pose_compose", "tsr_pose_tau_grad", "tsr_dssim_scratch_size", "tsr_dssim", "tsr_render_train_photometric", "tsr_equilateral_scratch_size", "tsr_equilateral", "tsr_equilateral_noalloc", "tsr_face_stats", "tsr_sensor_normals", "tsr_normal_scratch_size", "tsr_render_train_normal", "tsr_mapping_scratch_size", "tsr_render_train_mapping", "tsr_check", "tsr_last_error",
            "tsr_profile_enable", "tsr_profile_reset", "tsr_profile_read"]


class TsrIntrinsics(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class TsrParams(C.Structure):
    _fields_ = [("sigma", C.c_float), ("t_min", C.c_float), ("z_near", C.c_float), ("r_min", C.c_float),
                ("w_color", C.c_float), ("w_depth", C.c_float), ("opacity_min", C.c_int32),
                ("tight_tiles", C.c_int32), ("perspective", C.c_int32)]


class TsrScene(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("col", C.c_void_p), ("opa", C.c_void_p), ("faces", C.c_void_p),
                ("n_vertices", C.c_int64), ("n_faces", C.c_int64), ("face_sigma", C.c_void_p),
                ("grad_face_sigma", C.c_void_p)]


class TsrSchedule(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("order", C.c_int32), ("grid", C.c_int32)]


class TsrBinning(C.Structure):
    _fields_ = [("pairs", C.c_void_p), ("ranges", C.c_void_p), ("n_pairs", C.c_void_p), ("overflow", C.c_void_p),
                ("tile_counts", C.c_void_p), ("records", C.c_void_p), ("capacity", C.c_int64),
                ("n_tiles", C.c_int64), ("n_pixels", C.c_int64), ("last_face", C.c_void_p)]


class TsrError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load libtsr.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    P, I64, I = C.c_void_p, C.c_int64, C.c_int
    lib.tsr_workspace_size.argtypes = [P, P, I, I64, P]
    lib.tsr_workspace_init.argtypes = [P, C.c_size_t, P]
    lib.tsr_bin_and_sort.argtypes = [P, P, P, I, P, P, C.c_size_t, P]
    lib.tsr_count.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P]
    lib.tsr_binning_view.argtypes = [P, P, I, P, C.c_size_t, P]
    lib.tsr_render_forward.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P, P, P]
    lib.tsr_render_backward.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P, P, P, P, P, P, P]
    lib.tsr_render_train_l1.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.tsr_pose_step.argtypes = [P, P, I, C.c_float, C.c_float, P]
    lib.tsr_pose_compose.argtypes = [P, P, I, P, P]
    lib.tsr_pose_tau_grad.argtypes = [P, P, I, P, P]
    lib.tsr_dssim_scratch_size.argtypes = [P, I, P]
    lib.tsr_dssim.argtypes = [P, I, P, P, C.c_float, I, P, P, P, C.c_size_t, P]
    lib.tsr_render_train_photometric.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P, C.c_float, P, P, P, P, P, P, P, P,
                                                 P, C.c_size_t, P]
    lib.tsr_equilateral_scratch_size.argtypes = [I64, P]
    lib.tsr_equilateral.argtypes = [P, C.c_float, I, P, P, P, C.c_size_t, P]
    lib.tsr_equilateral_noalloc.argtypes = [P, C.c_float, I, P, P, P]
    lib.tsr_face_stats.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P, P, P]
    lib.tsr_sensor_normals.argtypes = [P, P, I, P, P]
    lib.tsr_normal_scratch_size.argtypes = [P, P, I, P]
    lib.tsr_render_train_normal.argtypes = [P, P, P, I, P, P, C.c_size_t, P, C.c_float, P, P, P, P, P, I, P,
                                            C.c_size_t, P]
    lib.tsr_mapping_scratch_size.argtypes = [P, P, I, P]
    lib.tsr_render_train_mapping.argtypes = [P, P, P, I, P, P, C.c_size_t, P, P, P, C.c_float, C.c_float, P, P, P, P,
                                             P, P, P, P, P, P, P, C.c_size_t, P]
    lib.tsr_check.argtypes = [P, P, P]
    lib.tsr_last_error.restype = C.c_char_p
    lib.tsr_profile_enable.argtypes = [I]
    lib.tsr_profile_reset.argtypes = []
    lib.tsr_profile_read.argtypes = [C.c_char_p, C.c_size_t]
    for fn in EXPORTED:
        getattr(lib, fn).restype = C.c_char_p if fn == "tsr_last_error" else C.c_int
    _lib = lib
    return lib


def check(rc: int, where: str) -> None:
    if rc != TSR_OK:
        raise TsrError(rc, where, load().tsr_last_error().decode())


def profile_enable(on: bool = True) -> None:
    check(load().tsr_profile_enable(1 if on else 0), "tsr_profile_enable")


def profile_reset() -> None:
    check(load().tsr_profile_reset(), "tsr_profile_reset")


def profile_read() -> dict:
    """{kernel: (launches, total_ms)} since the last reset (synchronises the recorded events)."""
    import json

    buf = C.create_string_buffer(1 << 16)
    check(load().tsr_profile_read(buf, len(buf)), "tsr_profile_read")
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}
