"""Shared test utilities: SE(3) exponential (library matrix exponential), tiny scenes,
and the gradient comparison rule.  No rasterizer arithmetic lives here."""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from paper_2605_31419_amd import scenes as S


def hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]], dtype=np.float64)


def se3_exp(tau):
    """Exp of tau = (rho, theta) in se(3) as a 4x4 matrix (scipy's matrix exponential)."""
    X = np.zeros((4, 4))
    X[:3, :3] = hat(tau[3:])
    X[:3, 3] = tau[:3]
    return scipy.linalg.expm(X)


def left_perturb(pose12, tau):
    """Pose (float64 [12]) of Exp(tau) o T_CW."""
    p = np.asarray(pose12, np.float64)
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:12]
    T2 = se3_exp(np.asarray(tau, np.float64)) @ T
    return np.concatenate([T2[:3, :3].reshape(9), T2[:3, 3]])


def plain_scene(verts, col=None, opa=None):
    """Soup from explicit vertex triplets [M, 3, 3] (float32 arrays)."""
    verts = np.asarray(verts, np.float64)
    m = verts.shape[0]
    pos = verts.reshape(m * 3, 3).T.astype(np.float32)
    colv = (np.ones((3, 3 * m)) if col is None else np.asarray(col, np.float64).reshape(m * 3, 3).T).astype(np.float32)
    opav = (np.ones(3 * m) if opa is None else np.asarray(opa, np.float64).reshape(-1)).astype(np.float32)
    return S.Scene(np.ascontiguousarray(pos), np.ascontiguousarray(colv), np.ascontiguousarray(opav), None)


IDENTITY = np.concatenate([np.eye(3).reshape(9), np.zeros(3)]).astype(np.float32)


def unit_cam(w=32, h=32):
    """q = (x/z, y/z): focal 1, principal point 0 -- so z=1 vertices land on their (x, y)."""
    return S.Intrinsics(w, h, 1.0, 1.0, 0.0, 0.0)


def tiny_scene(seed, n_faces=8, w=32, h=24, f=30.0, z=(1.0, 3.0), size=(0.15, 0.6)):
    intr = S.Intrinsics(w, h, f, f, (w - 1) / 2.0, (h - 1) / 2.0)
    sc = S.frustum_soup(seed, n_faces, intr, z_range=z, size_range=size)
    return sc, intr


# Element-wise rounding allowance for an FP32 implementation: a few FP32 ulps (2e-6 relative)
# of the sum of absolute per-pixel contributions to the element.  When an element is a large
# cancellation over many pixels (e.g. random-sign upstream gradients on a face covering 1e5+
# pixels), correlated FP32 rounding of the per-pixel terms is bounded by this, not by |g*|.
COND_ULPS = 2e-6


def grad_close(g, ref, rel=1e-3, abs_frac=1e-5, name="", cond=None):
    """Norm-wise and element-wise agreement; returns (ok, message, bad_indices).
    `cond` (optional) holds each element's sum of absolute per-pixel contributions."""
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nr = np.linalg.norm(ref)
    inf = np.max(np.abs(ref)) if ref.size else 0.0
    norm_ok = np.linalg.norm(g - ref) <= rel * nr + 1e-30
    floor = abs_frac * inf + 1e-30
    err = np.abs(g - ref)
    base_bar = rel * np.abs(ref) + floor
    n_cond = 0
    if cond is not None:
        floor = floor + COND_ULPS * np.asarray(cond, np.float64).reshape(-1)
        # elements inside the bar only thanks to the rounding allowance of their conditioning
        n_cond = int(np.count_nonzero((err > base_bar) & (err <= rel * np.abs(ref) + floor)))
    bad = np.nonzero(err > rel * np.abs(ref) + floor)[0]
    msg = (f"{name}: |d|/|ref| = {np.linalg.norm(g - ref) / max(nr, 1e-300):.3e}, "
           f"{bad.size} elementwise outliers of {g.size}")
    if cond is not None:
        msg += f", {n_cond} within the bar only through the conditioning allowance"
    if bad.size:
        worst = bad[np.argsort(-np.abs(g[bad] - ref[bad]))[:5]]
        msg += " [" + "; ".join(f"i={i} got={g[i]:.6e} ref={ref[i]:.6e}" for i in worst) + f"] max|ref|={inf:.3e}"
    return norm_ok and bad.size == 0, msg, bad
