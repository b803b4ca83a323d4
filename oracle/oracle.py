"""ctypes wrapper of the FP64 oracle (``liboracle.so`` built from ``tsr_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the CPU-baseline
leg of the benchmark.  It never imports the HIP package; the only thing the two sides share
is the seeded input arrays.

Inputs are normally the float32 arrays the GPU path also receives; they are promoted to FP64
exactly.  Float64 inputs pass unchanged, which lets finite differences perturb them freely.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE = os.path.join(_HERE, "tsr_oracle.c")
# Compiler line used by the build step (kept here so the build and a stale-check agree).
CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11"]


class _Scene(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("col", C.c_void_p), ("opa", C.c_void_p),
                ("faces", C.c_void_p), ("n_vertices", C.c_int64), ("n_faces", C.c_int64),
                ("face_sigma", C.c_void_p)]


class _Cam(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class _Par(C.Structure):
    _fields_ = [("sigma", C.c_double), ("z_near", C.c_double), ("r_min", C.c_double), ("opa_min", C.c_double),
                ("tight_tiles", C.c_double), ("persp", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library not built: {LIB_PATH} (run __graft_entry__.build())")
        _lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        _lib.orc_render.argtypes = [P, P, P, P, P, C.c_int64, P, P, P]
        _lib.orc_backward.argtypes = [P, P, P, P, P, C.c_int64, P, P, P, P, P, P, P]
        _lib.orc_backward_abs.argtypes = [P, P, P, P, P, C.c_int64, P, P, P, P, P, P, P, P, P, P]
        _lib.orc_backward_sigma.argtypes = [P, P, P, P, P, C.c_int64, P, P, P, P, P, P, P, P, P, P, P, P]
        _lib.orc_project.argtypes = [P, P, P, P, P, P, P, P]
        _lib.orc_bin.argtypes = [P, P, P, C.c_int, P, C.c_int64, P, P, P, P, P]
        _lib.orc_l1_seeds.argtypes = [P, P, P, P, C.c_int64, C.c_int64, C.c_double, C.c_double, P, P]
        _lib.orc_l1_seeds.restype = C.c_double
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_max_threads.restype = C.c_int
        _lib.orc_state.argtypes = [P, P, P, P, P, C.c_int64, C.c_double, P]
        _lib.orc_face_stats.argtypes = [P, P, P, P, C.c_double, P, P, P, P, P]
        _lib.orc_min_rho.argtypes = [P, P, P, P, P, C.c_int64, P]
        _lib.orc_ridge_gap.argtypes = [P, P, P, P, P, C.c_int64, P]
    return _lib


class use_library:
    """Context manager that points this wrapper at another build of the oracle (used by the
    mutation tests, which compile deliberately broken copies and check the pins reject them)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, LIB_PATH
        self.saved = (_lib, LIB_PATH)
        _lib, LIB_PATH = None, self.path
        return self

    def __exit__(self, *exc):
        global _lib, LIB_PATH
        _lib, LIB_PATH = self.saved
        return False


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Args:
    """Keeps the contiguous arrays alive for the duration of a call."""

    def __init__(self, scene, pose, intr, sigma, z_near, r_min, opacity_min=False, tight_tiles=False,
                 perspective=False):
        # float32 inputs are promoted exactly; float64 inputs (finite differences) pass as is
        self.pos = np.ascontiguousarray(scene.pos, dtype=np.float64)
        self.col = np.ascontiguousarray(scene.col, dtype=np.float64)
        self.opa = np.ascontiguousarray(scene.opa, dtype=np.float64)
        self.faces = None if scene.faces is None else np.ascontiguousarray(scene.faces, dtype=np.int32)
        fs = getattr(scene, "face_sigma", None)
        self.face_sigma = None if fs is None else np.ascontiguousarray(fs, dtype=np.float64)
        self.sc = _Scene(_ptr(self.pos), _ptr(self.col), _ptr(self.opa), _ptr(self.faces),
                         self.pos.shape[1], scene.n_faces, _ptr(self.face_sigma))
        self.pose = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(-1))
        self.cam = _cam(intr)
        self.par = _Par(sigma, z_near, r_min, 1.0 if opacity_min else 0.0, 1.0 if tight_tiles else 0.0,
                        1.0 if perspective else 0.0)


def _cam(intr) -> _Cam:
    w, h, fx, fy, cx, cy = intr.as_tuple() if hasattr(intr, "as_tuple") else intr
    return _Cam(int(w), int(h), fx, fy, cx, cy)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def render(scene, pose, intr, sigma=1.0, z_near=0.1, r_min=1e-3,
           pixels: Optional[np.ndarray] = None, opacity_min: bool = False,
           perspective: bool = False) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Colour [3, P], depth [P], final transmittance [P] of the listed pixel indices
    (y*W + x), or of the whole frame when `pixels` is None (P = H*W).  `opacity_min` selects
    the face opacity min(o_i) instead of the mean; `perspective` the perspective-correct
    colour interpolation and plane depth."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min, opacity_min, perspective=perspective)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    n = a.cam.width * a.cam.height if pix is None else pix.shape[0]
    col = np.zeros((3, n)); dep = np.zeros(n); tr = np.zeros(n)
    rc = lib().orc_render(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix),
                          n, _ptr(col), _ptr(dep), _ptr(tr))
    if rc:
        raise ValueError(f"orc_render failed ({rc})")
    return col, dep, tr


def backward(scene, pose, intr, g_color: np.ndarray, g_depth: np.ndarray,
             g_trans: Optional[np.ndarray] = None, sigma=1.0, z_near=0.1, r_min=1e-3,
             pixels: Optional[np.ndarray] = None, with_abs: bool = False, opacity_min: bool = False,
             want_sigma: bool = False, perspective: bool = False):
    """Gradients (pos [3,N], col [3,N], opa [N], pose [6]) from the listed pixels' upstream
    gradients g_color [3,P], g_depth [P], g_trans [P].  With `with_abs`, also returns the
    per-element sums of absolute per-pixel contributions (pos, col, opa) -- the conditioning
    that bounds the rounding error of a lower-precision implementation.  With `want_sigma`
    (scenes with per-face exponents), also returns dL/dsigma per face [M].  `perspective` as
    for render."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min, opacity_min, perspective=perspective)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    n = a.cam.width * a.cam.height if pix is None else pix.shape[0]
    gc = np.ascontiguousarray(np.asarray(g_color, np.float64).reshape(3, n))
    gd = np.ascontiguousarray(np.asarray(g_depth, np.float64).reshape(n))
    gt = None if g_trans is None else np.ascontiguousarray(np.asarray(g_trans, np.float64).reshape(n))
    N = a.pos.shape[1]
    gpos = np.zeros((3, N)); gcol = np.zeros((3, N)); gopa = np.zeros(N); gpose = np.zeros(6)
    if want_sigma:
        M = int(a.sc.n_faces)
        gsig = np.zeros(max(M, 1))
        absv = [np.zeros((3, N)), np.zeros((3, N)), np.zeros(N), np.zeros(max(M, 1))] if with_abs else [None] * 4
        rc = lib().orc_backward_sigma(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix), n,
                                      _ptr(gc), _ptr(gd), _ptr(gt), _ptr(gpos), _ptr(gcol), _ptr(gopa), _ptr(gpose),
                                      _ptr(gsig), *[_ptr(x) for x in absv])
        if rc:
            raise ValueError(f"orc_backward_sigma failed ({rc})")
        if with_abs:
            return gpos, gcol, gopa, gpose, gsig[:M], (absv[0], absv[1], absv[2], absv[3][:M])
        return gpos, gcol, gopa, gpose, gsig[:M]
    if with_abs:
        apos = np.zeros((3, N)); acol = np.zeros((3, N)); aopa = np.zeros(N)
        rc = lib().orc_backward_abs(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix), n,
                                    _ptr(gc), _ptr(gd), _ptr(gt), _ptr(gpos), _ptr(gcol), _ptr(gopa), _ptr(gpose),
                                    _ptr(apos), _ptr(acol), _ptr(aopa))
        if rc:
            raise ValueError(f"orc_backward_abs failed ({rc})")
        return gpos, gcol, gopa, gpose, (apos, acol, aopa)
    rc = lib().orc_backward(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix), n,
                            _ptr(gc), _ptr(gd), _ptr(gt), _ptr(gpos), _ptr(gcol), _ptr(gopa), _ptr(gpose))
    if rc:
        raise ValueError(f"orc_backward failed ({rc})")
    return gpos, gcol, gopa, gpose


def project(scene, pose, intr, sigma=1.0, z_near=0.1, r_min=1e-3):
    """Per-face q [6, M], (r, o_F, z_F, zkey) [4, M], pixel rect [4, M], tile count [M]."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min)
    M = scene.n_faces
    q = np.zeros((6, M)); f = np.zeros((4, M)); rect = np.zeros((4, M), np.int32)
    tiles = np.zeros(M, np.int64)
    rc = lib().orc_project(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(q),
                           _ptr(f), _ptr(rect), _ptr(tiles))
    if rc:
        raise ValueError(f"orc_project failed ({rc})")
    return q, f, rect, tiles


def bin_pairs(scene, poses: Sequence[np.ndarray], intrs: Sequence, sigma=1.0, z_near=0.1, r_min=1e-3,
              tight_tiles=False):
    """Reference tile lists: (tile[K], zbits[K], face[K], ranges[T_total, 2]); `tight_tiles`
    keeps only the tiles of a face's rectangle that can hold a pixel the face covers."""
    a = _Args(scene, poses[0], intrs[0], sigma, z_near, r_min, tight_tiles=tight_tiles)
    V = len(poses)
    ps = np.ascontiguousarray(np.stack([np.asarray(p, np.float64).reshape(12) for p in poses]))
    cams = (_Cam * V)(*[_cam(i) for i in intrs])
    t_total = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    K = C.c_int64(0)
    rc = lib().orc_bin(C.byref(a.sc), _ptr(ps), cams, V, C.byref(a.par), 0, C.byref(K),
                       None, None, None, None)
    if rc not in (0, -2):
        raise ValueError(f"orc_bin failed ({rc})")
    k = K.value
    tile = np.zeros(max(k, 1), np.int64); zb = np.zeros(max(k, 1), np.uint32)
    face = np.zeros(max(k, 1), np.int64); ranges = np.zeros((max(t_total, 1), 2), np.int64)
    rc = lib().orc_bin(C.byref(a.sc), _ptr(ps), cams, V, C.byref(a.par), k, C.byref(K),
                       _ptr(tile), _ptr(zb), _ptr(face), _ptr(ranges))
    if rc:
        raise ValueError(f"orc_bin failed ({rc})")
    return tile[:k], zb[:k], face[:k], ranges[:t_total]


def l1_seeds(color, depth, target_color, target_depth, norm_pix: int, w_c=0.8, w_d=0.05):
    """L1 loss (means, weights w_c, w_d; depth masked where the target is <= 0) and its
    per-pixel derivatives.  Arrays are [3, P] / [P]."""
    color = np.ascontiguousarray(color, np.float64); depth = np.ascontiguousarray(depth, np.float64)
    tc = np.ascontiguousarray(target_color, np.float32).reshape(color.shape)
    td = np.ascontiguousarray(target_depth, np.float32).reshape(depth.shape)
    n = depth.shape[0]
    gc = np.zeros_like(color); gd = np.zeros_like(depth)
    L = lib().orc_l1_seeds(_ptr(color), _ptr(depth), _ptr(tc), _ptr(td), n, int(norm_pix), w_c, w_d,
                           _ptr(gc), _ptr(gd))
    return float(L), gc, gd


def state(scene, pose, intr, sigma=1.0, z_near=0.1, r_min=1e-3, pixels=None, rho_eps=1e-3):
    """Per-pixel hash of the piecewise-constant rendering state (covering set and order,
    maximising edge, clamp and steep-edge flags); equal hashes at both ends of a finite
    difference mean no discontinuity was crossed."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    n = a.cam.width * a.cam.height if pix is None else pix.shape[0]
    out = np.zeros(n, np.uint64)
    rc = lib().orc_state(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix), n,
                         rho_eps, _ptr(out))
    if rc:
        raise ValueError(f"orc_state failed ({rc})")
    return out


def min_rho(scene, pose, intr, sigma=1.0, z_near=0.1, r_min=1e-3, pixels=None, opacity_min=False):
    """Per pixel, the smallest |rho| = |phi/phi(s)| over the faces whose bounding box contains
    it (+inf where none); |rho| < 1e-3 marks the steep-edge band of sigma < 1 windows."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min, opacity_min)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    n = a.cam.width * a.cam.height if pix is None else pix.shape[0]
    out = np.zeros(n)
    rc = lib().orc_min_rho(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix), n, _ptr(out))
    if rc:
        raise ValueError(f"orc_min_rho failed ({rc})")
    return out


def ridge_gap(scene, pose, intr, sigma=1.0, z_near=0.1, r_min=1e-3, pixels=None, opacity_min=False):
    """Per pixel, the smallest gap (in rho units) between the two smallest normalised edge
    distances of the faces blended there (+inf where none): near 0 on a ridge of phi, where
    the edge that attains the minimum flips under rounding."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min, opacity_min)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)
    n = a.cam.width * a.cam.height if pix is None else pix.shape[0]
    out = np.zeros(n)
    rc = lib().orc_ridge_gap(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), _ptr(pix), n, _ptr(out))
    if rc:
        raise ValueError(f"orc_ridge_gap failed ({rc})")
    return out


def face_stats(scene, pose, intr, t_min=1e-6, sigma=1.0, z_near=0.1, r_min=1e-3, opacity_min=False):
    """Per-face projected area [M], coverage interval (cov_lo, cov_hi) [M] and visibility
    (certain, possible) [M] of one view; see orc_face_stats for the definitions."""
    a = _Args(scene, pose, intr, sigma, z_near, r_min, opacity_min)
    M = int(a.sc.n_faces)
    area = np.zeros(max(M, 1))
    lo, hi, vc, vp = (np.zeros(max(M, 1), np.int32) for _ in range(4))
    rc = lib().orc_face_stats(C.byref(a.sc), _ptr(a.pose), C.byref(a.cam), C.byref(a.par), float(t_min),
                              _ptr(area), _ptr(lo), _ptr(hi), _ptr(vc), _ptr(vp))
    if rc:
        raise ValueError(f"orc_face_stats failed ({rc})")
    return area[:M], lo[:M], hi[:M], vc[:M].astype(bool), vp[:M].astype(bool)
