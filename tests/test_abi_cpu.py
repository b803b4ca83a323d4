"""CPU checks of the C ABI: the library loads, exports every symbol the header declares, and
its host-side argument validation and workspace sizing behave as documented (no kernel is
launched by any of these calls)."""
import ctypes as C
import os
import re

import pytest

from paper_2605_31419_amd import _lib
from paper_2605_31419_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tsr.h")).read()
    return sorted(set(re.findall(r"TSR_API\s+(?:const\s+)?\w+\s*\*?\s*(tsr_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["tsr_bin_and_sort", "tsr_render_forward", "tsr_render_backward"]:
        assert name in syms
    assert sorted(syms) == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def _scene(n_faces=10):
    return _lib.TsrScene(1, 1, 1, None, 3 * n_faces, n_faces)      # dummy non-null pointers


def _intr(*sizes):
    arr = (_lib.TsrIntrinsics * len(sizes))()
    for i, (w, h) in enumerate(sizes):
        arr[i] = _lib.TsrIntrinsics(w, h, 100.0, 100.0, (w - 1) / 2, (h - 1) / 2)
    return arr


def test_workspace_size_grows_with_capacity_and_views():
    lib = _lib.load()
    sc = _scene(1000)
    b0, b1, b2 = C.c_size_t(), C.c_size_t(), C.c_size_t()
    assert lib.tsr_workspace_size(C.byref(sc), _intr((64, 48)), 1, 0, C.byref(b0)) == 0
    assert lib.tsr_workspace_size(C.byref(sc), _intr((64, 48)), 1, 1000, C.byref(b1)) == 0
    assert lib.tsr_workspace_size(C.byref(sc), _intr((64, 48), (64, 48)), 2, 0, C.byref(b2)) == 0
    assert b1.value - b0.value >= 16 * 1000
    assert b2.value > b0.value
    # per face: record 96 B + gradient accumulator 80 B + count 4 B
    assert b0.value >= 1000 * (96 + 80 + 4)


@pytest.mark.parametrize("case", ["null_scene", "bad_views", "bad_size", "bad_sigma", "bad_tmin",
                                  "small_ws", "null_ws", "soup_size"])
def test_invalid_arguments_are_rejected(case):
    lib = _lib.load()
    sc = _scene(10)
    intr = _intr((64, 48))
    par = _lib.TsrParams(1.0, 1e-6, 0.1, 1e-3, 0.8, 0.05)
    nviews, ws, nbytes, poses = 1, C.c_void_p(1), C.c_size_t(1 << 30), C.c_void_p(1)
    expect = _lib.TSR_EINVAL
    if case == "null_scene":
        sc_arg = None
    else:
        sc_arg = C.byref(sc)
    if case == "bad_views":
        nviews = 0
    if case == "bad_size":
        intr = _intr((0, 48))
    if case == "bad_sigma":
        par.sigma = 0.0
    if case == "bad_tmin":
        par.t_min = 1.0
    if case == "small_ws":
        nbytes = C.c_size_t(100)
        expect = _lib.TSR_EWORKSPACE
    if case == "null_ws":
        ws = None
    if case == "soup_size":
        sc = _lib.TsrScene(1, 1, 1, None, 5, 10)
        sc_arg = C.byref(sc)
    rc = lib.tsr_bin_and_sort(sc_arg, poses, intr, nviews, C.byref(par), ws, nbytes, None)
    assert rc == expect, (rc, lib.tsr_last_error())
    assert len(lib.tsr_last_error()) > 0


def test_too_many_views_rejected():
    lib = _lib.load()
    sizes = [(32, 32)] * (_lib.TSR_MAX_VIEWS + 1)
    out = C.c_size_t()
    assert lib.tsr_workspace_size(C.byref(_scene(4)), _intr(*sizes), len(sizes), 0, C.byref(out)) == _lib.TSR_EINVAL


def test_generators_are_seeded_and_shaped():
    a = S.workload("single_64x48")
    b = S.workload("single_64x48")
    assert (a.scene.pos == b.scene.pos).all() and a.scene.pos.shape == (3, 6000)
    assert a.scene.pos.dtype.name == "float32" and a.scene.opa.min() >= 0.3 and a.scene.opa.max() <= 1.0
    z = a.scene.pos[2].reshape(-1, 3).mean(axis=1)
    assert 0.45 < z.min() and z.max() < 4.1
    r = S.room_soup(5, 20000, size_range=(0.005, 0.03))
    e = r.pos.reshape(3, -1, 3)
    edge = (((e[:, :, 1] - e[:, :, 0]) ** 2).sum(axis=0)) ** 0.5
    assert 0.002 < edge.min() and edge.max() < 0.06
    assert (r.pos[0] > -0.03).all() and (r.pos[0] < 4.03).all()      # faces straddle the walls by < one radius


# ---------------------------------------------------------------------------- training-energy entry points

def _params(**kw):
    par = _lib.TsrParams(1.0, 1e-6, 0.1, 1e-3, 0.8, 0.05, 0)
    for k, v in kw.items():
        setattr(par, k, v)
    return par


def test_dssim_scratch_size_and_validation():
    lib = _lib.load()
    b1, b2 = C.c_size_t(), C.c_size_t()
    assert lib.tsr_dssim_scratch_size(_intr((64, 48)), 1, C.byref(b1)) == 0
    assert lib.tsr_dssim_scratch_size(_intr((64, 48), (33, 17)), 2, C.byref(b2)) == 0
    assert b1.value >= 52 * 64 * 48 and b2.value >= b1.value + 52 * 33 * 17
    assert lib.tsr_dssim_scratch_size(_intr((0, 48)), 1, C.byref(b1)) == _lib.TSR_EINVAL
    assert lib.tsr_dssim_scratch_size(_intr((64, 48)), 0, C.byref(b1)) == _lib.TSR_EINVAL
    p = C.c_void_p(256)
    need = C.c_size_t()
    lib.tsr_dssim_scratch_size(_intr((64, 48)), 1, C.byref(need))
    args = lambda color, loss, grad, scratch, nbytes: lib.tsr_dssim(_intr((64, 48)), 1, color, p, 1.0, 0, loss, grad,
                                                                  scratch, nbytes, None)
    assert args(None, p, p, p, need) == _lib.TSR_EINVAL                      # no colour
    assert args(p, None, None, p, need) == _lib.TSR_EINVAL                   # no output
    assert args(p, p, p, p, C.c_size_t(need.value - 1)) == _lib.TSR_EWORKSPACE
    assert args(p, p, p, C.c_void_p(257), need) == _lib.TSR_EINVAL          # misaligned scratch


def test_equilateral_scratch_size_and_validation():
    lib = _lib.load()
    b = C.c_size_t()
    assert lib.tsr_equilateral_scratch_size(1000, C.byref(b)) == 0 and b.value >= 8 * 4
    assert lib.tsr_equilateral_scratch_size(-1, C.byref(b)) == _lib.TSR_EINVAL
    sc = _scene(1000)
    p = C.c_void_p(256)
    assert lib.tsr_equilateral(C.byref(sc), 1.0, 0, None, None, p, b, None) == _lib.TSR_EINVAL
    assert lib.tsr_equilateral(C.byref(sc), 1.0, 0, p, p, p, C.c_size_t(8), None) == _lib.TSR_EWORKSPACE
    pos_only = _lib.TsrScene(1, None, None, None, 3000, 1000)      # colours and opacities unused
    assert lib.tsr_equilateral(C.byref(pos_only), 1.0, 0, p, p, p, C.c_size_t(8), None) == _lib.TSR_EWORKSPACE
    no_pos = _lib.TsrScene(None, 1, 1, None, 3000, 1000)
    assert lib.tsr_equilateral(C.byref(no_pos), 1.0, 0, p, p, p, b, None) == _lib.TSR_EINVAL


def test_face_stats_and_photometric_validation():
    lib = _lib.load()
    sc, intr, p = _scene(10), _intr((64, 48)), C.c_void_p(256)
    big = C.c_size_t(1 << 30)
    assert lib.tsr_face_stats(C.byref(sc), p, intr, 1, C.byref(_params()), p, big, None, None, None,
                              None) == _lib.TSR_EINVAL
    assert lib.tsr_render_train_photometric(C.byref(sc), p, intr, 1, C.byref(_params()), p, big, p, p, 0.2,
                                            None, p, None, None, None, None, None, None, p, big,
                                            None) == _lib.TSR_EINVAL        # the D-SSIM term reads colour
    assert lib.tsr_render_train_photometric(C.byref(sc), p, intr, 1, C.byref(_params()), p, big, p, p, 0.2,
                                            p, p, None, None, None, None, None, None, p, C.c_size_t(16),
                                            None) == _lib.TSR_EWORKSPACE
    assert lib.tsr_bin_and_sort(C.byref(sc), p, intr, 1, C.byref(_params(opacity_min=2)), p, big,
                                None) == _lib.TSR_EINVAL


def test_normal_entry_points_validation():
    lib = _lib.load()
    p = C.c_void_p(256)
    assert lib.tsr_sensor_normals(None, _intr((64, 48)), 1, p, None) == _lib.TSR_EINVAL
    assert lib.tsr_sensor_normals(p, _intr((64, 0)), 1, p, None) == _lib.TSR_EINVAL
    zero_f = _intr((64, 48))
    zero_f[0].fx = 0.0
    assert lib.tsr_sensor_normals(p, zero_f, 1, p, None) == _lib.TSR_EINVAL
    mesh = _lib.TsrScene(1, 1, 1, 1, 30, 10)                        # indexed faces
    big = C.c_size_t(1 << 30)
    assert lib.tsr_render_train_normal(C.byref(mesh), p, _intr((64, 48)), 1, C.byref(_params()), p, big, p, 0.05,
                                       None, None, None, None, None, 0, p, big, None) == _lib.TSR_EINVAL
    sc = _scene(10)
    need = C.c_size_t()
    assert lib.tsr_normal_scratch_size(C.byref(sc), _intr((64, 48)), 1, C.byref(need)) == 0
    assert need.value >= 40 * 30 + 32 * 64 * 48
    assert lib.tsr_render_train_normal(C.byref(sc), p, _intr((64, 48)), 1, C.byref(_params()), p, big, None, 0.05,
                                       None, None, None, None, None, 0, p, need, None) == _lib.TSR_EINVAL
    assert lib.tsr_render_train_normal(C.byref(sc), p, _intr((64, 48)), 1, C.byref(_params()), p, big, p, 0.05,
                                       None, None, None, None, None, 1, p, C.c_size_t(need.value - 1),
                                       None) == _lib.TSR_EWORKSPACE


def test_mapping_step_validation():
    """The one-binning mapping step: soups only, all three targets, colour and depth outputs,
    and a scratch of at least the D-SSIM scratch + 32 bytes per face + 128 per 16x16 tile."""
    lib = _lib.load()
    p = C.c_void_p(256)
    big = C.c_size_t(1 << 30)
    sc, intr = _scene(10), _intr((64, 48))
    need, ssim = C.c_size_t(), C.c_size_t()
    assert lib.tsr_mapping_scratch_size(C.byref(sc), intr, 1, C.byref(need)) == 0
    assert lib.tsr_dssim_scratch_size(intr, 1, C.byref(ssim)) == 0
    assert need.value >= ssim.value + 32 * 10 + 128 * 4 * 3
    assert lib.tsr_mapping_scratch_size(C.byref(sc), intr, 0, C.byref(need)) == _lib.TSR_EINVAL

    def call(scene=sc, tn=p, color=p, scratch_bytes=need):
        return lib.tsr_render_train_mapping(C.byref(scene), p, intr, 1, C.byref(_params()), p, big, p, p, tn, 0.2,
                                            0.05, color, p, None, None, None, None, None, None, None, None, p,
                                            scratch_bytes, None)
    mesh = _lib.TsrScene(1, 1, 1, 1, 30, 10)
    assert call(scene=mesh) == _lib.TSR_EINVAL
    assert call(tn=None) == _lib.TSR_EINVAL
    assert call(color=None) == _lib.TSR_EINVAL
    assert call(scratch_bytes=C.c_size_t(need.value - 1)) == _lib.TSR_EWORKSPACE


def test_equilateral_noalloc_validation():
    """The allocation-free E_equi variant validates like tsr_equilateral and refuses more than
    TSR_EQUI_NOALLOC_MAX_FACES faces before any device call."""
    lib = _lib.load()
    p = C.c_void_p(256)
    M = _lib.TSR_EQUI_NOALLOC_MAX_FACES
    too_big = _lib.TsrScene(1, None, None, None, 3 * (M + 1), M + 1)
    assert lib.tsr_equilateral_noalloc(C.byref(too_big), 1.0, 0, p, p, None) == _lib.TSR_EINVAL
    assert b"at most" in lib.tsr_last_error()
    sc = _scene(10)
    assert lib.tsr_equilateral_noalloc(C.byref(sc), 1.0, 0, None, None, None) == _lib.TSR_EINVAL
    assert lib.tsr_equilateral_noalloc(None, 1.0, 0, p, p, None) == _lib.TSR_EINVAL
    short_soup = _lib.TsrScene(1, None, None, None, 20, 10)
    assert lib.tsr_equilateral_noalloc(C.byref(short_soup), 1.0, 0, p, p, None) == _lib.TSR_EINVAL


def test_packaged_schedule_table_covers_the_standard_workloads():
    """The committed tile-schedule table (written on an MI355X by tune_table.py) has an entry
    for each standard workload's key and ``lookup`` returns it (nearest pair-count bucket for
    a nearby count)."""
    from paper_2605_31419_amd import autotune
    from paper_2605_31419_amd import scenes as S

    tab = autotune.load_table(autotune.DEFAULT_TABLE)
    assert len(tab) >= 5
    i1200 = S.intrinsics_for(1200, 680)
    for intrs, k in (([S.intrinsics_for(64, 48)], 512), ([S.intrinsics_for(640, 480)], 18000),
                     ([i1200] * 8, 280000), ([i1200], 392216), ([i1200] * 8, 1930600)):
        key = autotune.key_for(intrs, k)
        assert key in tab, key
        sched = autotune.lookup(intrs, k, autotune.DEFAULT_TABLE)
        assert sched == tuple(tab[key]["schedule"]) and sched in autotune.CANDIDATES
    assert autotune.lookup([i1200], 300000, autotune.DEFAULT_TABLE) is not None     # nearest bucket
