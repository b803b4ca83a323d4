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
