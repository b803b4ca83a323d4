"""Seeded synthetic workloads for the triangle-soup rasterizer.

This module only draws random numbers and lays them out; it holds none of the
rasterizer's arithmetic (no projection, windowing, blending or gradients), so
both the HIP path and the FP64 oracle may consume what it produces.

Workloads (all seeded through ``numpy.random.Generator(PCG64(seed))``):

* ``frustum_soup``  -- faces scattered through a camera frustum (small parity case:
  64x48, 2,000 faces, depths 0.5-4 m with volume-uniform density, edge lengths
  log-uniform 1-10 cm, per-vertex RGB U[0,1], opacity U[0.3,1]).
* ``room_soup``     -- faces sampled area-weighted on the surfaces of a synthetic room
  (a 4.0 x 3.0 x 2.6 m box plus random interior rectangles), lying in the surface
  plane, with a smooth procedural colour texture.  Stands in for the indoor RGB-D
  sequences (Replica, TUM RGB-D) the paper evaluates on (Sec. 4.2), which are not
  available here.
* camera helpers -- pinhole intrinsics per resolution, random poses inside the room,
  small pose perturbations (1 cm / 0.5 deg) and smooth keyframe trajectories.

Conventions: world frame z-up; camera frame x right, y down, z forward (OpenCV);
a pose is T_CW (world -> camera) stored as 12 float32 values: R row-major then t.
Vertex arrays are SoA float32: ``pos[3, N]``, ``col[3, N]``, ``opa[N]``.  A soup has
N = 3M and face m uses vertices 3m, 3m+1, 3m+2 (``faces`` is None).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Focal lengths used for the synthetic cameras (the paper gives no intrinsics).
FOCAL_BY_RES = {(64, 48): 52.5, (320, 240): 262.5, (640, 480): 525.0, (1200, 680): 600.0}

ROOM_SIZE = (4.0, 3.0, 2.6)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def as_tuple(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy)


def intrinsics_for(width: int, height: int, focal: Optional[float] = None) -> Intrinsics:
    """Pinhole intrinsics with the principal point at the image centre of integer
    pixel centres, c = ((W-1)/2, (H-1)/2)."""
    f = focal if focal is not None else FOCAL_BY_RES.get((width, height), 0.9375 * width)
    return Intrinsics(width, height, float(np.float32(f)), float(np.float32(f)),
                      float(np.float32((width - 1) / 2.0)), float(np.float32((height - 1) / 2.0)))


@dataclasses.dataclass
class Scene:
    pos: np.ndarray            # [3, N] float32
    col: np.ndarray            # [3, N] float32
    opa: np.ndarray            # [N] float32
    faces: Optional[np.ndarray] = None   # [M, 3] int32, None = soup
    face_sigma: Optional[np.ndarray] = None   # [M] float32 per-face window exponents, None = global

    @property
    def n_vertices(self) -> int:
        return int(self.pos.shape[1])

    @property
    def n_faces(self) -> int:
        return int(self.faces.shape[0]) if self.faces is not None else self.n_vertices // 3

    def subset(self, face_ids: np.ndarray) -> "Scene":
        """Soup made of the given faces (vertex attributes copied)."""
        face_ids = np.asarray(face_ids, dtype=np.int64)
        if self.faces is None:
            vid = (3 * face_ids[:, None] + np.arange(3)[None, :]).reshape(-1)
        else:
            vid = self.faces[face_ids].reshape(-1).astype(np.int64)
        fs = None if self.face_sigma is None else np.ascontiguousarray(self.face_sigma[face_ids])
        return Scene(np.ascontiguousarray(self.pos[:, vid]), np.ascontiguousarray(self.col[:, vid]),
                     np.ascontiguousarray(self.opa[vid]), None, fs)


# ----------------------------------------------------------------------------- poses

def _rodrigues(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * k + (1 - math.cos(angle)) * (k @ k)


def look_pose(position: Sequence[float], yaw: float, pitch: float) -> np.ndarray:
    """T_CW (as [12] float32) for a camera at `position` looking along yaw/pitch (z-up world)."""
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    r_wc = np.stack([right, down, fwd], axis=1)       # columns: camera axes in world
    r_cw = r_wc.T
    t_cw = -r_cw @ np.asarray(position, dtype=np.float64)
    return pose_pack(r_cw, t_cw)


def pose_pack(r: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.concatenate([np.asarray(r, np.float64).reshape(9), np.asarray(t, np.float64).reshape(3)]).astype(np.float32)


def pose_unpack(p: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    p = np.asarray(p, dtype=np.float64)
    return p[:9].reshape(3, 3), p[9:12].copy()


def perturb_pose(pose: np.ndarray, g: np.random.Generator, trans_m: float = 0.01,
                 rot_deg: float = 0.5) -> np.ndarray:
    """Left-compose a rigid motion of exactly `trans_m` metres (random direction) and
    `rot_deg` degrees (random axis) onto T_CW."""
    r, t = pose_unpack(pose)
    d = g.normal(size=3)
    d /= np.linalg.norm(d)
    ax = g.normal(size=3)
    dr = _rodrigues(ax, math.radians(rot_deg))
    return pose_pack(dr @ r, dr @ t + trans_m * d)


def random_room_pose(g: np.random.Generator) -> np.ndarray:
    pos = np.array([g.uniform(0.6, 3.4), g.uniform(0.6, 2.4), g.uniform(1.0, 1.8)])
    yaw = g.uniform(-math.pi, math.pi)
    pitch = math.radians(g.uniform(-15.0, 15.0))
    return look_pose(pos, yaw, pitch)


def room_trajectory(g: np.random.Generator, n_views: int) -> List[np.ndarray]:
    """Keyframe poses along a smooth path: consecutive views 10-30 cm and 5-15 deg apart."""
    pos = np.array([g.uniform(1.2, 2.8), g.uniform(1.0, 2.0), g.uniform(1.2, 1.6)])
    yaw = g.uniform(-math.pi, math.pi)
    pitch = math.radians(g.uniform(-10.0, 10.0))
    heading = g.uniform(-math.pi, math.pi)
    out = [look_pose(pos, yaw, pitch)]
    lo = np.array([0.6, 0.6, 1.0])
    hi = np.array([3.4, 2.4, 1.8])
    for _ in range(n_views - 1):
        step = g.uniform(0.10, 0.30)
        heading += g.uniform(-0.6, 0.6)
        d = np.array([math.cos(heading), math.sin(heading), g.uniform(-0.2, 0.2)])
        d /= np.linalg.norm(d)
        nxt = pos + step * d
        if np.any(nxt < lo) or np.any(nxt > hi):       # bounce off the walls
            heading += math.pi
            nxt = np.clip(pos - step * d, lo, hi)
        pos = nxt
        turn = math.radians(g.uniform(5.0, 15.0)) * (1 if g.uniform() < 0.5 else -1)
        yaw += turn
        pitch = float(np.clip(pitch + math.radians(g.uniform(-3, 3)), -math.radians(15), math.radians(15)))
        out.append(look_pose(pos, yaw, pitch))
    return out


# ----------------------------------------------------------------------------- face shapes

def _triangles_around(g: np.random.Generator, centres: np.ndarray, sizes: np.ndarray,
                      t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """Vertices [M, 3, 3] at angles 2*pi*k/3 + U(-0.3, 0.3) on a circle of radius s/sqrt(3)
    spanned by the unit tangents t1, t2 (so an undisturbed triangle has edge length s)."""
    m = centres.shape[0]
    ang = (2.0 * math.pi / 3.0) * np.arange(3)[None, :] + g.uniform(-0.3, 0.3, size=(m, 3))
    ang += g.uniform(0, 2 * math.pi, size=(m, 1))
    rad = (sizes / math.sqrt(3.0))[:, None]
    return (centres[:, None, :] + (rad * np.cos(ang))[:, :, None] * t1[:, None, :]
            + (rad * np.sin(ang))[:, :, None] * t2[:, None, :])


def _random_unit(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _tangents(normals: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    helper = np.where(np.abs(normals[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(normals, helper)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(normals, t1)
    return t1, t2


def _pack_soup(verts: np.ndarray, col: np.ndarray, opa: np.ndarray) -> Scene:
    m = verts.shape[0]
    pos = np.ascontiguousarray(verts.reshape(m * 3, 3).T.astype(np.float32))
    colv = np.ascontiguousarray(col.reshape(m * 3, 3).T.astype(np.float32))
    return Scene(pos, colv, np.ascontiguousarray(opa.reshape(-1).astype(np.float32)), None)


def frustum_soup(seed: int, n_faces: int = 2000, intr: Optional[Intrinsics] = None,
                 z_range=(0.5, 4.0), size_range=(0.01, 0.10)) -> Scene:
    """Faces scattered in the camera frustum of an identity pose (camera frame == world)."""
    g = rng(seed)
    intr = intr or intrinsics_for(64, 48)
    z0, z1 = z_range
    z = np.cbrt(z0 ** 3 + g.uniform(size=n_faces) * (z1 ** 3 - z0 ** 3))    # pdf ~ z^2
    u = g.uniform(-0.5, intr.width - 0.5, size=n_faces)
    v = g.uniform(-0.5, intr.height - 0.5, size=n_faces)
    centres = np.stack([(u - intr.cx) * z / intr.fx, (v - intr.cy) * z / intr.fy, z], axis=1)
    sizes = np.exp(g.uniform(math.log(size_range[0]), math.log(size_range[1]), size=n_faces))
    t1, t2 = _tangents(_random_unit(g, n_faces))
    verts = _triangles_around(g, centres, sizes, t1, t2)
    col = g.uniform(0.0, 1.0, size=(n_faces, 3, 3))
    opa = g.uniform(0.3, 1.0, size=(n_faces, 3))
    return _pack_soup(verts, col, opa)


@dataclasses.dataclass
class _Surface:
    origin: np.ndarray   # corner
    a: np.ndarray        # first side vector
    b: np.ndarray        # second side vector
    tex_k: np.ndarray    # [3, n_waves, 3] wave vectors per channel
    tex_phase: np.ndarray
    tex_amp: np.ndarray
    base: np.ndarray     # [3] base colour

    @property
    def area(self) -> float:
        return float(np.linalg.norm(np.cross(self.a, self.b)))


def _room_surfaces(g: np.random.Generator, n_rects: int = 6) -> List[_Surface]:
    lx, ly, lz = ROOM_SIZE
    o = np.zeros(3)
    ex, ey, ez = np.eye(3)
    quads = [
        (o, lx * ex, ly * ey),                        # floor
        (lz * ez, lx * ex, ly * ey),                  # ceiling
        (o, lx * ex, lz * ez),                        # wall y = 0
        (ly * ey, lx * ex, lz * ez),                  # wall y = ly
        (o, ly * ey, lz * ez),                        # wall x = 0
        (lx * ex, ly * ey, lz * ez),                  # wall x = lx
    ]
    for _ in range(n_rects):                          # random interior rectangles
        n = _random_unit(g, 1)
        t1, t2 = _tangents(n)
        sa, sb = g.uniform(0.4, 1.5, size=2)
        centre = np.array([g.uniform(0.8, lx - 0.8), g.uniform(0.8, ly - 0.8), g.uniform(0.5, lz - 0.5)])
        quads.append((centre - 0.5 * sa * t1[0] - 0.5 * sb * t2[0], sa * t1[0], sb * t2[0]))
    out = []
    for origin, a, b in quads:
        out.append(_Surface(np.asarray(origin, float), np.asarray(a, float), np.asarray(b, float),
                            tex_k=g.normal(scale=6.0, size=(3, 3, 3)),
                            tex_phase=g.uniform(0, 2 * math.pi, size=(3, 3)),
                            tex_amp=g.uniform(0.05, 0.2, size=(3, 3)),
                            base=g.uniform(0.2, 0.8, size=3)))
    return out


def room_soup(seed: int, n_faces: int, size_range=(0.005, 0.03),
              size_mixture: Optional[Sequence[Tuple[float, float, float]]] = None,
              n_rects: int = 6) -> Scene:
    """Faces sampled area-weighted on the room surfaces, in the surface plane.

    `size_mixture` is a list of (weight, s_min, s_max) log-uniform size components,
    e.g. [(0.9, 0.005, 0.02), (0.1, 0.05, 0.20)]; otherwise `size_range` is used."""
    g = rng(seed)
    surfs = _room_surfaces(g, n_rects)
    areas = np.array([s.area for s in surfs])
    which = g.choice(len(surfs), size=n_faces, p=areas / areas.sum())
    su = g.uniform(size=n_faces)
    sv = g.uniform(size=n_faces)
    if size_mixture is None:
        size_mixture = [(1.0, size_range[0], size_range[1])]
    w = np.array([c[0] for c in size_mixture], dtype=np.float64)
    comp = g.choice(len(size_mixture), size=n_faces, p=w / w.sum())
    lo = np.array([c[1] for c in size_mixture])[comp]
    hi = np.array([c[2] for c in size_mixture])[comp]
    sizes = np.exp(np.log(lo) + g.uniform(size=n_faces) * (np.log(hi) - np.log(lo)))

    origin = np.stack([s.origin for s in surfs])[which]
    a = np.stack([s.a for s in surfs])[which]
    b = np.stack([s.b for s in surfs])[which]
    centres = origin + su[:, None] * a + sv[:, None] * b
    t1 = a / np.linalg.norm(a, axis=1, keepdims=True)
    nrm = np.cross(a, b)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    verts = _triangles_around(g, centres, sizes, t1, t2)

    # smooth per-surface texture (a few sinusoids per channel) plus vertex noise
    col = np.empty((n_faces, 3, 3))
    for si, s in enumerate(surfs):
        idx = np.nonzero(which == si)[0]
        if idx.size == 0:
            continue
        p = verts[idx]                                       # [m, 3, 3]
        for ch in range(3):
            val = np.full(p.shape[:2], s.base[ch])
            for wv in range(3):
                val += s.tex_amp[ch, wv] * np.sin(p @ s.tex_k[ch, wv] + s.tex_phase[ch, wv])
            col[idx, :, ch] = val
    col += g.normal(scale=0.03, size=col.shape)
    col = np.clip(col, 0.0, 1.0)
    opa = g.uniform(0.3, 1.0, size=(n_faces, 3))
    return _pack_soup(verts, col, opa)


def random_targets(seed: int, intr: Intrinsics, z_range=(0.5, 4.0)) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform random colour [3, H, W] in [0,1] and depth [H, W] targets."""
    g = rng(seed)
    c = g.uniform(0, 1, size=(3, intr.height, intr.width)).astype(np.float32)
    d = g.uniform(z_range[0], z_range[1], size=(intr.height, intr.width)).astype(np.float32)
    return c, d


def image_pair(seed: int, width: int, height: int, noise: float = 0.05) -> Tuple[np.ndarray, np.ndarray]:
    """A (rendered, target) pair of colour images [3, H, W] in [0, 1], float32: the target is
    a smooth texture (three random plane waves per channel) with pixel noise, the rendered
    image that texture shifted by up to a pixel with its own noise -- the kind of pair the
    photometric term compares while tracking and mapping."""
    g = rng(seed)
    y, x = np.mgrid[0:height, 0:width].astype(np.float64)
    dx, dy = g.uniform(-1, 1, size=2)
    out = [np.empty((3, height, width)) for _ in range(2)]
    k = g.uniform(0.02, 0.3, size=(3, 3, 2)) * g.choice([-1, 1], size=(3, 3, 2))
    amp = g.uniform(0.05, 0.2, size=(3, 3))
    ph = g.uniform(0, 2 * np.pi, size=(3, 3))
    base = g.uniform(0.3, 0.7, size=3)
    for img, (sx, sy) in zip(out, ((0.0, 0.0), (dx, dy))):
        for ch in range(3):
            v = np.full((height, width), base[ch])
            for w in range(3):
                v += amp[ch, w] * np.sin(k[ch, w, 0] * (x + sx) + k[ch, w, 1] * (y + sy) + ph[ch, w])
            img[ch] = v + g.normal(scale=noise, size=v.shape)
    return np.clip(out[1], 0, 1).astype(np.float32), np.clip(out[0], 0, 1).astype(np.float32)


def random_pixel_grads(seed: int, n_pix: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Seeded upstream gradients (colour [3, P], depth [P], transmittance [P])."""
    g = rng(seed)
    return (g.normal(size=(3, n_pix)).astype(np.float32), g.normal(size=n_pix).astype(np.float32),
            g.normal(size=n_pix).astype(np.float32))


# ----------------------------------------------------------------------------- named workloads

@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    poses: List[np.ndarray]            # per view T_CW [12] float32
    intr: List[Intrinsics]
    target_poses: List[np.ndarray]     # per view pose the targets are rendered from
    sigma: float = 1.0


def workload(name: str, instance: int = 0, n_faces: Optional[int] = None) -> Workload:
    """The named synthetic workloads; seed = 1000 * config + instance."""
    if name == "single_64x48":
        seed = 1000 * 1 + instance
        intr = intrinsics_for(64, 48)
        sc = frustum_soup(seed, n_faces or 2000, intr)
        ident = pose_pack(np.eye(3), np.zeros(3))
        return Workload(name, sc, [ident], [intr], [ident], 1.0)
    if name == "track_640x480":
        seed = 1000 * 2 + instance
        g = rng(seed + 500)
        sc = room_soup(seed, n_faces or 200_000, size_range=(0.005, 0.03))
        pose = random_room_pose(g)
        return Workload(name, sc, [pose], [intrinsics_for(640, 480)], [perturb_pose(pose, g)], 1.0)
    if name == "window_8x1200x680":
        seed = 1000 * 3 + instance
        g = rng(seed + 500)
        sc = room_soup(seed, n_faces or 500_000, size_range=(0.005, 0.03))
        poses = room_trajectory(g, 8)
        return Workload(name, sc, poses, [intrinsics_for(1200, 680)] * 8,
                        [perturb_pose(p, g) for p in poses], 1.0)
    if name == "serve_1M":
        seed = 1000 * 4 + instance
        g = rng(seed + 500)
        sc = room_soup(seed, n_faces or 1_000_000, size_mixture=[(0.9, 0.005, 0.02), (0.1, 0.05, 0.20)])
        pose = random_room_pose(g)
        return Workload(name, sc, [pose], [intrinsics_for(640, 480)], [pose], 1.0)
    if name == "track_1200x680_1M":
        seed = 1000 * 5 + instance
        g = rng(seed + 500)
        sc = room_soup(seed, n_faces or 1_000_000, size_mixture=[(0.9, 0.005, 0.02), (0.1, 0.05, 0.20)])
        pose = random_room_pose(g)
        return Workload(name, sc, [pose], [intrinsics_for(1200, 680)], [perturb_pose(pose, g)], 1.0)
    raise KeyError(name)


SERVE_RESOLUTIONS = [(320, 240), (640, 480), (1200, 680)]


def serving_queries(seed: int, n: int, qps: float) -> List[Tuple[float, Intrinsics, np.ndarray]]:
    """Poisson arrivals at `qps`: (arrival_time_s, intrinsics, pose) per query."""
    g = rng(seed)
    t = np.cumsum(g.exponential(1.0 / qps, size=n))
    out = []
    for i in range(n):
        w, h = SERVE_RESOLUTIONS[int(g.integers(0, len(SERVE_RESOLUTIONS)))]
        out.append((float(t[i]), intrinsics_for(w, h), random_room_pose(g)))
    return out
