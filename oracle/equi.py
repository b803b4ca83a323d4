"""FP64 reference of the equilateral regulariser E_equi (Sec. 3.4, eq. 14).

TEST INFRASTRUCTURE ONLY: imported by the test-suite; it never imports the HIP package.

For each face with corners a, b, c and each corner, the cosine of the internal angle is the
dot product of the two unit edge vectors leaving that corner; the loss is the mean over faces
of the mean over the three corners of (cos - 1/2)^2.  The paper gives no rule for a face with
a zero-length edge (its angles are undefined); the reading taken here: such a face contributes
0 to the sum and receives no gradient, and still counts in the mean's 1/|F|.

Positions are SoA [3, N]; faces [M, 3] vertex indices (None for a soup, face m = vertices
3m, 3m+1, 3m+2).
"""
from __future__ import annotations

import numpy as np


def _corners(pos: np.ndarray, faces):
    pos = np.asarray(pos, np.float64)
    if faces is None:
        M = pos.shape[1] // 3
        idx = np.arange(3 * M).reshape(M, 3)
    else:
        idx = np.asarray(faces, np.int64).reshape(-1, 3)
    return idx, [pos[:, idx[:, k]].T for k in range(3)]       # three [M, 3] corner arrays


def corner_cosines(pos: np.ndarray, faces=None) -> np.ndarray:
    """[M, 3]: cosine of the internal angle at corner k of each face (NaN-free: faces with a
    zero-length edge get 0.5, which contributes nothing)."""
    _, P = _corners(pos, faces)
    out = np.full((P[0].shape[0], 3), 0.5)
    for k in range(3):
        u = P[(k + 1) % 3] - P[k]
        v = P[(k + 2) % 3] - P[k]
        nu = np.linalg.norm(u, axis=1)
        nv = np.linalg.norm(v, axis=1)
        ok = (nu > 0) & (nv > 0)
        out[ok, k] = np.sum(u[ok] * v[ok], axis=1) / (nu[ok] * nv[ok])
    return out


def _degenerate(pos, faces) -> np.ndarray:
    _, P = _corners(pos, faces)
    bad = np.zeros(P[0].shape[0], bool)
    for k in range(3):
        bad |= np.linalg.norm(P[(k + 1) % 3] - P[k], axis=1) == 0
    return bad


def e_equi(pos: np.ndarray, faces=None) -> float:
    c = corner_cosines(pos, faces)
    c[_degenerate(pos, faces)] = 0.5
    M = c.shape[0]
    return float(np.sum((c - 0.5) ** 2) / (3.0 * M)) if M else 0.0


def e_equi_grad(pos: np.ndarray, faces=None) -> np.ndarray:
    """dE_equi/dpos, [3, N].  With unit edges u^ = u/|u|, v^ = v/|v| leaving corner a towards
    b and c, cos = u^.v^ has d cos/db = (v^ - cos u^)/|u|, d cos/dc = (u^ - cos v^)/|v| and
    d cos/da = -(d cos/db + d cos/dc); each corner adds (2/3M)(cos - 1/2) times these."""
    pos = np.asarray(pos, np.float64)
    idx, P = _corners(pos, faces)
    M = idx.shape[0]
    g = np.zeros_like(pos)
    if M == 0:
        return g
    bad = _degenerate(pos, faces)
    for k in range(3):
        ia, ib, ic = idx[:, k], idx[:, (k + 1) % 3], idx[:, (k + 2) % 3]
        u = P[(k + 1) % 3] - P[k]
        v = P[(k + 2) % 3] - P[k]
        nu = np.linalg.norm(u, axis=1, keepdims=True)
        nv = np.linalg.norm(v, axis=1, keepdims=True)
        ok = ~bad
        uh = np.where(ok[:, None], u / np.where(nu > 0, nu, 1), 0)
        vh = np.where(ok[:, None], v / np.where(nv > 0, nv, 1), 0)
        cos = np.sum(uh * vh, axis=1, keepdims=True)
        s = np.where(ok[:, None], 2.0 / (3.0 * M) * (cos - 0.5), 0)
        db = s * (vh - cos * uh) / np.where(nu > 0, nu, 1)
        dc = s * (uh - cos * vh) / np.where(nv > 0, nv, 1)
        for ax in range(3):
            np.add.at(g[ax], ib, db[:, ax])
            np.add.at(g[ax], ic, dc[:, ax])
            np.add.at(g[ax], ia, -(db[:, ax] + dc[:, ax]))
    return g
