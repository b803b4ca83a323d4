"""The allocation-free E_equi entry point (tsr_equilateral_noalloc, static per-device partials)
against tsr_equilateral with a caller-provided scratch buffer, through the C ABI: two calls in a
row, the second on a smaller input, each equal to the scratch-buffer call (soups: bit for bit,
the same kernels in the same order; an indexed mesh adds its gradients with float atomics, so
its gradients agree to FP32 rounding), and the size limit rejected before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2605_31419_amd import _lib, raster
from tests.helpers import grad_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _soup(M, seed):
    pos = np.random.default_rng(seed).normal(size=(3, 3 * M)).astype(np.float32)
    N = pos.shape[1]
    return raster.DeviceScene(torch.as_tensor(pos, device="cuda"), torch.zeros(3, N, device="cuda"),
                              torch.zeros(N, device="cuda"))


def _mesh(M, N, seed):
    g = np.random.default_rng(seed)
    pos = g.normal(size=(3, N)).astype(np.float32)
    faces = np.stack([g.choice(N, size=3, replace=False) for _ in range(M)]).astype(np.int32)
    return raster.DeviceScene(torch.as_tensor(pos, device="cuda"), torch.zeros(3, N, device="cuda"),
                              torch.zeros(N, device="cuda"), torch.as_tensor(faces, device="cuda").contiguous())


def _both(sc, weight, accumulate_into=None):
    init = accumulate_into
    g_ref = None if init is None else init.clone()
    g_new = None if init is None else init.clone()
    l_ref, g_ref = raster.equilateral(sc, weight=weight, grad=g_ref, accumulate=init is not None)
    l_new, g_new = raster.equilateral(sc, weight=weight, grad=g_new, accumulate=init is not None, noalloc=True)
    torch.cuda.synchronize()
    return (l_ref.cpu().numpy(), g_ref.cpu().numpy()), (l_new.cpu().numpy(), g_new.cpu().numpy())


def test_noalloc_matches_scratch_call_two_calls_second_smaller():
    for M, seed in [(1_000_000, 1), (1007, 2)]:
        _say(f"[noalloc] soup M={M}")
        sc = _soup(M, seed)
        (lr, gr), (ln, gn) = _both(sc, 1.2)
        assert np.array_equal(lr, ln), (lr, ln)
        assert np.array_equal(gr, gn)


def test_noalloc_limits_and_other_modes():
    # largest size it takes, then a smaller indexed mesh, then accumulate mode
    M = _lib.TSR_EQUI_NOALLOC_MAX_FACES
    _say(f"[noalloc] soup M={M} (the limit)")
    sc = _soup(M, 3)
    (lr, gr), (ln, gn) = _both(sc, 0.7)
    assert np.array_equal(lr, ln) and np.array_equal(gr, gn)
    del sc, gr, gn
    _say("[noalloc] indexed mesh M=5000")
    sc = _mesh(5000, 3000, 4)
    (lr, gr), (ln, gn) = _both(sc, 1.0)
    assert np.array_equal(lr, ln)
    ok, msg, _ = grad_close(gn, gr, rel=1e-6, abs_frac=1e-7, name="mesh grad")
    _say("  " + msg)
    assert ok, msg
    _say("[noalloc] accumulate, M=300")
    sc = _soup(300, 5)
    base = torch.as_tensor(np.random.default_rng(6).normal(size=3 * 900).astype(np.float32), device="cuda")
    (lr, gr), (ln, gn) = _both(sc, 1.0, accumulate_into=base)
    assert np.array_equal(lr, ln) and np.array_equal(gr, gn)
    # one face beyond the limit is refused before any device work
    big = _lib.TsrScene(1, 1, 1, None, 3 * (M + 1), M + 1)
    loss = torch.empty(1, device="cuda")
    rc = _lib.load().tsr_equilateral_noalloc(C.byref(big), 1.0, 0, raster._ptr(loss), None, raster._stream())
    assert rc == _lib.TSR_EINVAL
