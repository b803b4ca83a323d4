"""FP64 reference of the normal supervision of mapping (Sec. 3.4): sensor normals from depth
and the normal loss E_norm, with its gradient.

TEST INFRASTRUCTURE ONLY: imported by the test-suite; it never imports the HIP package.

Readings (the paper gives the formulas, not these details):
  * sensor normals: back-project every pixel, p_d(u, v) = D(u, v) ((u - cx)/fx, (v - cy)/fy, 1);
    the image-space differences are central, dx = (p(u+1, v) - p(u-1, v))/2 and likewise dy;
    N_bar = (dx x dy) / |dx x dy|.  A pixel is valid when it is not on the image border, its
    depth and its four neighbours' depths are > 0 and the cross product is not zero.  With x
    right, y down and z forward, a surface facing the camera gets N_bar pointing away from it
    (+z for a frontal plane).
  * face normal: n_F = (v1 - v0) x (v2 - v0) / |...| in vertex order, no flip.
  * rendered normal map: N(p) = R_CW sum_F n_F alpha_F T_F -- the faces' world normals
    composited like a colour that is constant over the face, then rotated into the camera
    frame; it is not renormalised.
  * E_norm = mean over valid pixels of (1 - N(p) . N_bar(p)) (0 when no pixel is valid): the
    mean, like the other terms of the energy.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def backproject(depth: np.ndarray, intr) -> np.ndarray:
    """[3, H, W] camera-space points of a depth map [H, W]."""
    H, W = depth.shape
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    d = np.asarray(depth, np.float64)
    return np.stack([d * (u - intr.cx) / intr.fx, d * (v - intr.cy) / intr.fy, d])


def sensor_normals(depth: np.ndarray, intr):
    """(N_bar [3, H, W], valid [H, W] bool); invalid pixels hold 0."""
    H, W = depth.shape
    p = backproject(depth, intr)
    out = np.zeros((3, H, W))
    valid = np.zeros((H, W), bool)
    if H < 3 or W < 3:
        return out, valid
    dx = (p[:, 1:-1, 2:] - p[:, 1:-1, :-2]) / 2.0
    dy = (p[:, 2:, 1:-1] - p[:, :-2, 1:-1]) / 2.0
    c = np.cross(dx, dy, axis=0)
    n = np.linalg.norm(c, axis=0)
    d = np.asarray(depth, np.float64)
    ok = (d[1:-1, 1:-1] > 0) & (d[1:-1, 2:] > 0) & (d[1:-1, :-2] > 0) & (d[2:, 1:-1] > 0) & (d[:-2, 1:-1] > 0) & (n > 0)
    inner = np.where(ok, c / np.where(n > 0, n, 1.0), 0.0)
    out[:, 1:-1, 1:-1] = inner
    valid[1:-1, 1:-1] = ok
    return out, valid


def face_normals(pos: np.ndarray) -> np.ndarray:
    """[3, M] unit normals of a soup (vertex order)."""
    pos = np.asarray(pos, np.float64)
    a, b, c = pos[:, 0::3], pos[:, 1::3], pos[:, 2::3]
    cr = np.cross(b - a, c - a, axis=0)
    return cr / np.linalg.norm(cr, axis=0)


class _Soup:
    """A soup with the attributes the renderer reads."""

    def __init__(self, pos, col, opa, face_sigma=None):
        self.pos, self.col, self.opa, self.faces = pos, col, opa, None
        self.n_faces = pos.shape[1] // 3
        self.face_sigma = face_sigma


def normal_scene(scene):
    """The soup with every vertex colour replaced by its face's world normal; per-face window
    exponents (when the scene has them) are kept, since the normal map is rendered with the
    same blending weights as the colours."""
    n = face_normals(scene.pos)
    col = np.repeat(n, 3, axis=1)
    fs = getattr(scene, "face_sigma", None)
    return _Soup(np.asarray(scene.pos, np.float64), col, np.asarray(scene.opa, np.float64),
                 None if fs is None else np.asarray(fs, np.float64))


def _rot(pose):
    return np.asarray(pose, np.float64).reshape(12)[:9].reshape(3, 3)


def render_normals(scene, pose, intr, sigma=1.0) -> np.ndarray:
    """Rendered normal map N [3, P] in the camera frame."""
    Nw = O.render(normal_scene(scene), pose, intr, sigma=sigma)[0]
    return _rot(pose) @ Nw


def e_norm(scene, pose, intr, nbar, valid, sigma=1.0) -> float:
    N = render_normals(scene, pose, intr, sigma)
    m = np.asarray(valid, bool).reshape(-1)
    if not m.any():
        return 0.0
    nb = np.asarray(nbar, np.float64).reshape(3, -1)
    return float(np.sum(1.0 - np.sum(N[:, m] * nb[:, m], axis=0)) / m.sum())


def e_norm_grad(scene, pose, intr, nbar, valid, sigma=1.0):
    """(dE/dpos [3, N], dE/dopa [N], dE/dtau [6]) of a soup; tau = (rho, theta) is the left
    perturbation of T_CW.  The loss sees the geometry through alpha (the rasteriser's
    backward with the world normals as colours and dE/dN_w = R^T dE/dN as the colour seed),
    through the face normals (chain rule of the normalised cross product), and sees the
    rotation once more through N = R N_w (dE/dtheta += sum_p N x dE/dN)."""
    R = _rot(pose)
    m = np.asarray(valid, bool).reshape(-1)
    nb = np.asarray(nbar, np.float64).reshape(3, -1)
    P = nb.shape[1]
    gN = np.zeros((3, P))
    if m.any():
        gN[:, m] = -nb[:, m] / m.sum()
    gNw = R.T @ gN
    sn = normal_scene(scene)
    gpos, gcol, gopa, gpose = O.backward(sn, pose, intr, gNw, np.zeros(P), None, sigma=sigma)
    gpos = np.array(gpos, np.float64)
    # through the face normals: dE/dn_F = sum of the three vertex-colour gradients
    pos = np.asarray(scene.pos, np.float64)
    a, b, c = pos[:, 0::3], pos[:, 1::3], pos[:, 2::3]
    e1, e2 = b - a, c - a
    cr = np.cross(e1, e2, axis=0)
    L = np.linalg.norm(cr, axis=0)
    n = cr / L
    gn = gcol[:, 0::3] + gcol[:, 1::3] + gcol[:, 2::3]
    gc = (gn - n * np.sum(n * gn, axis=0)) / L
    ge1 = np.cross(e2, gc, axis=0)
    ge2 = np.cross(gc, e1, axis=0)
    gpos[:, 1::3] += ge1
    gpos[:, 2::3] += ge2
    gpos[:, 0::3] -= ge1 + ge2
    # the rotation of the rendered map into the camera frame
    N = R @ O.render(sn, pose, intr, sigma=sigma)[0]
    gpose = np.array(gpose, np.float64).reshape(6)
    gpose[3:] += np.sum(np.cross(N, gN, axis=0), axis=1)
    return gpos, np.asarray(gopa, np.float64), gpose
