"""Seeded synthetic scenes for the light-stage face renderer.

The paper fits a morphable face model lit by a virtual light stage to real
photographs (Face Modeling and Results paragraphs).  Neither the photographs
nor the morphable model are available, so this module builds a stand-in
scene of the same structure, from seeds:

* a mean face shape: a regular vertex grid lifted onto an ellipsoid cap,
  two counter-clockwise triangles per cell;
* identity (80), expression (90) and albedo (80) bases, each a smooth
  Gaussian random field over the vertices (random Fourier features),
  matching the coefficient counts of the Face Modeling paragraph;
* N = 20 square area lights on vertices of an icosphere hemisphere, each
  facing the origin (the virtual light stage of the Face Modeling
  paragraph), with RGB intensities, five of them switched off;
* a 32x32 gray specular texture, a pinhole camera facing the face, a pose.

This module only produces input arrays.  It holds none of the renderer's
arithmetic: both the CPU oracle and the GPU library consume what it returns.
All arrays are float32 (int32 for indices) in the layouts the library takes:
per-vertex data is structure-of-arrays ``[3][V]`` and a basis is ``[K][3][V]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_ID, N_EXP, N_ALB = 80, 90, 80
N_LIGHTS = 20
SPEC_RES = 32

# Workload configurations: grid size, image size, samples per pixel.
CONFIGS = {
    # tiny: 1,024 vertices / 1,922 triangles, 64x64, 4 spp
    "tiny": dict(nx=32, ny=32, width=64, height=64, spp=4),
    # paper scale: 20,000 vertices / 39,432 triangles, 256x256, 16 spp
    "paper": dict(nx=125, ny=160, width=256, height=256, spp=16),
    # sequence fitting at full size: 60,000 vertices / 119,022 triangles, 512x512
    "sequence512": dict(nx=240, ny=250, width=512, height=512, spp=4),
}

GEN_SEED = 0        # mesh and bases
TARGET_SCENE_SEED = 1
EVAL_SCENE_SEED = 2
TARGET_RENDER_SEED = 7
TARGET_SPP = 256


@dataclass
class Model:
    """Morphable face model: topology, mean shape, bases, albedo, uv."""
    nx: int
    ny: int
    faces: np.ndarray        # int32 [F][3]
    mean: np.ndarray         # float32 [3][V]
    b_id: np.ndarray         # float32 [N_ID][3][V]
    b_exp: np.ndarray        # float32 [N_EXP][3][V]
    alb_mean: np.ndarray     # float32 [3][V]
    b_alb: np.ndarray        # float32 [N_ALB][3][V]
    uv: np.ndarray           # float32 [2][V]

    @property
    def n_vertices(self) -> int:
        return self.mean.shape[1]

    @property
    def n_faces(self) -> int:
        return self.faces.shape[0]


@dataclass
class Scene:
    """Camera, light stage geometry and image size."""
    width: int
    height: int
    cam: np.ndarray          # float32 [3]
    pix_scale: float         # image-plane size of one pixel at unit depth
    light_geom: np.ndarray   # float32 [N][12]: centre, e1, e2, unit normal
    spec_res: int = SPEC_RES


@dataclass
class Params:
    """Differentiable parameters of one evaluation."""
    alpha: np.ndarray        # float32 [N_ID]
    beta: np.ndarray         # float32 [N_EXP]
    delta: np.ndarray        # float32 [N_ALB]
    pose: np.ndarray         # float32 [6]: rx, ry, rz (radians), tx, ty, tz
    lights: np.ndarray       # float32 [N][3] RGB intensities
    spec: np.ndarray         # float32 [SPEC_RES*SPEC_RES]

    def copy(self) -> "Params":
        return Params(*(np.array(getattr(self, k)) for k in
                        ("alpha", "beta", "delta", "pose", "lights", "spec")))


# ---------------------------------------------------------------- mesh ----

def grid_faces(nx: int, ny: int) -> np.ndarray:
    """Two triangles per grid cell, split along (i,j)-(i+1,j+1), CCW from +z."""
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    v00 = (j * nx + i).ravel()
    v10 = v00 + 1
    v01 = v00 + nx
    v11 = v01 + 1
    a = np.stack([v00, v10, v11], axis=1)
    b = np.stack([v00, v11, v01], axis=1)
    f = np.empty((2 * a.shape[0], 3), dtype=np.int32)
    f[0::2] = a
    f[1::2] = b
    return f


def _rff_fields(x: np.ndarray, n_fields: int, ell: float,
                rng: np.random.Generator, m: int = 64) -> np.ndarray:
    """n_fields smooth Gaussian random fields at points x [V][3] (float64).

    g(x) = sqrt(2/m) sum_k w_k cos(omega_k . x + phi_k), omega ~ N(0, I/ell^2),
    phi ~ U[0, 2 pi), w ~ N(0, 1): a unit-variance field with a Gaussian
    covariance of length scale ell.  (Evaluated in float32 with torch CPU
    ops for multithreading; the random draws come from ``rng``.)
    """
    import torch
    omega = rng.normal(0.0, 1.0 / ell, size=(n_fields, m, 3))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n_fields, m))
    w = rng.normal(0.0, 1.0, size=(n_fields, m))
    X = torch.from_numpy(np.ascontiguousarray(x, np.float32))
    Om, Ph, Wt = (torch.from_numpy(a.astype(np.float32)) for a in (omega, phi, w))
    out = torch.empty((n_fields, x.shape[0]), dtype=torch.float32)
    chunk = max(1, 16_000_000 // max(1, x.shape[0] * m))
    for s in range(0, n_fields, chunk):
        e = min(n_fields, s + chunk)
        ph = torch.einsum("vc,fmc->fvm", X, Om[s:e]) + Ph[s:e, None, :]
        out[s:e] = math.sqrt(2.0 / m) * torch.einsum("fvm,fm->fv", torch.cos(ph), Wt[s:e])
    return out.numpy().astype(np.float64)


def make_model(nx: int, ny: int, seed: int = GEN_SEED,
               n_id: int = N_ID, n_exp: int = N_EXP, n_alb: int = N_ALB) -> Model:
    rng = np.random.default_rng(seed)
    xs = np.linspace(-0.6, 0.6, nx)
    ys = np.linspace(-0.75, 0.75, ny)
    gx, gy = np.meshgrid(xs, ys, indexing="xy")
    gx, gy = gx.ravel(), gy.ravel()
    gz = np.sqrt(1.0 - gx * gx - gy * gy)
    ax, ay, az = np.array([0.08, 0.10, 0.12]) * (1.0 + 0.1 * rng.uniform(-1, 1, 3))
    mean = np.stack([ax * gx, ay * gy, az * (gz - 0.6)])            # [3][V]
    uv = np.stack([(gx / 0.6 + 1) / 2, (gy / 0.75 + 1) / 2])
    V = nx * ny
    pts = mean.T
    b_id = 0.003 * _rff_fields(pts, n_id * 3, 0.03, rng).reshape(n_id, 3, V)
    b_exp = 0.002 * _rff_fields(pts, n_exp * 3, 0.03, rng).reshape(n_exp, 3, V)
    b_alb = 0.01 * _rff_fields(pts, n_alb * 3, 0.03, rng).reshape(n_alb, 3, V)
    alb_mean = np.tile(np.array([0.55, 0.38, 0.30])[:, None], (1, V))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Model(nx, ny, grid_faces(nx, ny), f32(mean), f32(b_id), f32(b_exp),
                 f32(alb_mean), f32(b_alb), f32(uv))


# --------------------------------------------------------- light stage ----

def icosphere1() -> np.ndarray:
    """Vertices (float64 [42][3], unit length) of a once-subdivided icosahedron."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
         (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, float) / np.linalg.norm(x) for x in v]
    mid = {}
    for a, b, c in f:
        for e in ((a, b), (b, c), (c, a)):
            k = tuple(sorted(e))
            if k not in mid:
                m = verts[k[0]] + verts[k[1]]
                mid[k] = len(verts)
                verts.append(m / np.linalg.norm(m))
    base = np.mean([verts[i] for i in f[1]], axis=0)   # face (0, 5, 1)
    return np.array(verts), base / np.linalg.norm(base)


def _rot_to_z(u: np.ndarray) -> np.ndarray:
    """Smallest rotation taking unit vector u to +z (Rodrigues)."""
    z = np.array([0.0, 0.0, 1.0])
    ax = np.cross(u, z)
    s, c = np.linalg.norm(ax), float(u @ z)
    if s < 1e-15:
        return np.eye(3)
    k = ax / s
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + s * K + (1 - c) * K @ K


def light_stage(n: int = N_LIGHTS, radius: float = 1.0, side: float = 0.2) -> np.ndarray:
    """Light quads [n][12] (centre, e1, e2, unit emitting normal), float32.

    The icosphere is turned so a face centroid points along +z (toward the
    camera); the n highest vertices by (z, y, x) are kept.  Each light is a
    side x side square facing the origin; e1 x e2 points along the normal.
    """
    verts, base = icosphere1()
    R = _rot_to_z(base)
    pts = verts @ R.T
    key = np.round(pts, 9)
    order = sorted(range(len(pts)), key=lambda i: (-key[i, 2], -key[i, 1], -key[i, 0]))
    out = np.zeros((n, 12), dtype=np.float64)
    yhat = np.array([0.0, 1.0, 0.0])
    for slot, i in enumerate(order[:n]):
        c = radius * pts[i]
        nrm = -pts[i] / np.linalg.norm(pts[i])
        a = np.cross(yhat, nrm)
        if np.linalg.norm(a) < 1e-9:
            a = np.array([1.0, 0.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(nrm, a)
        out[slot] = np.concatenate([c, side * a, side * b, nrm])
    return out.astype(np.float32)


def make_scene(width: int, height: int, fov_y_deg: float = 28.0) -> Scene:
    pix = math.tan(math.radians(fov_y_deg) / 2.0) / (height / 2.0)
    return Scene(width, height, np.array([0.0, 0.0, 0.5], np.float32),
                 float(np.float32(pix)), light_stage())


def make_params(seed: int, n_id: int = N_ID, n_exp: int = N_EXP,
                n_alb: int = N_ALB, n_lights: int = N_LIGHTS, n_off: int = 5) -> Params:
    rng = np.random.default_rng(1000003 * seed + 17)
    d2r = math.pi / 180.0
    pose = np.array([rng.uniform(-15, 15) * d2r, rng.uniform(-15, 15) * d2r,
                     rng.uniform(-5, 5) * d2r, *rng.uniform(-0.01, 0.01, 3)])
    lights = rng.uniform(0.0, 1.0, (n_lights, 3))
    lights[rng.choice(n_lights, n_off, replace=False)] = 0.0
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Params(f32(rng.normal(size=n_id)), f32(rng.normal(size=n_exp)),
                  f32(rng.normal(size=n_alb)), f32(pose), f32(lights),
                  f32(rng.uniform(0.1, 0.5, SPEC_RES * SPEC_RES)))


def perturb(p: Params, seed: int) -> Params:
    """Fitting start: coefficients += N(0, 0.3^2), lights x U[0.7, 1.3] (off
    lights start at 0.05), a fresh specular map, pose +-2 deg and +-5 mm."""
    rng = np.random.default_rng(7919 * seed + 5)
    q = p.copy()
    q.alpha += rng.normal(0, 0.3, q.alpha.shape).astype(np.float32)
    q.beta += rng.normal(0, 0.3, q.beta.shape).astype(np.float32)
    q.delta += rng.normal(0, 0.3, q.delta.shape).astype(np.float32)
    lit = q.lights * rng.uniform(0.7, 1.3, q.lights.shape)
    lit[q.lights == 0] = 0.05
    q.lights = lit.astype(np.float32)
    q.spec = rng.uniform(0.1, 0.5, q.spec.shape).astype(np.float32)
    d2r = math.pi / 180.0
    q.pose = (q.pose + np.concatenate([rng.uniform(-2, 2, 3) * d2r,
                                       rng.uniform(-0.005, 0.005, 3)])).astype(np.float32)
    return q


_MODEL_CACHE: dict = {}


def workload(name: str):
    """(model, scene, params at the evaluation seed, spp) for a named config."""
    cfg = CONFIGS[name]
    key = (cfg["nx"], cfg["ny"])
    if key not in _MODEL_CACHE:
        _MODEL_CACHE[key] = make_model(cfg["nx"], cfg["ny"])
    model = _MODEL_CACHE[key]
    scene = make_scene(cfg["width"], cfg["height"])
    return model, scene, make_params(EVAL_SCENE_SEED), cfg["spp"]


# ------------------------------------------------------ batched faces ----
# Many faces per launch: each instance draws its mesh size, its (square)
# image size and its sample count, and has its own parameters and light
# colours (make_params at its own seed) in the common light stage.
BATCH_GRIDS = ((62, 80), (88, 114), (125, 160), (153, 196), (177, 226))   # 5k, 10k, 20k, 30k, 40k vertices
BATCH_RES = (128, 192, 256, 384, 512)
BATCH_SPP = (4, 8, 16)
BATCH_N = 32


def model_cached(nx: int, ny: int) -> Model:
    key = (nx, ny)
    if key not in _MODEL_CACHE:
        _MODEL_CACHE[key] = make_model(nx, ny)
    return _MODEL_CACHE[key]


def batch_workload(n: int = BATCH_N, seed: int = 0, grids=BATCH_GRIDS, res=BATCH_RES, spps=BATCH_SPP):
    """n instances (model, scene, params, spp), drawn from a seeded generator."""
    rng = np.random.default_rng(4711 + seed)
    out = []
    for i in range(n):
        g = grids[int(rng.integers(len(grids)))]
        r = res[int(rng.integers(len(res)))]
        if isinstance(r, int):
            r = (r, r)
        spp = int(spps[int(rng.integers(len(spps)))])
        out.append((model_cached(*g), make_scene(r[0], r[1]), make_params(100 + 7 * seed + i), spp))
    return out


# ------------------------------------------------------ simple scenes ----
# Small hand-built scenes for closed-form checks (flat receivers, single
# occluders, a closed box of emitters).  They bypass the morphable model.

@dataclass
class Mesh:
    """Explicit mesh with per-vertex attributes (positions already posed)."""
    pos: np.ndarray          # float32 [3][V]
    faces: np.ndarray        # int32 [F][3]
    albedo: np.ndarray       # float32 [3][V]
    uv: np.ndarray           # float32 [2][V]
    extra: dict = field(default_factory=dict)


def flat_grid(n: int, half: float, z: float = 0.0, albedo=(1.0, 1.0, 1.0)) -> Mesh:
    """(n x n)-vertex square grid at height z spanning [-half, half]^2, facing +z."""
    xs = np.linspace(-half, half, n)
    gx, gy = np.meshgrid(xs, xs, indexing="xy")
    pos = np.stack([gx.ravel(), gy.ravel(), np.full(n * n, z)]).astype(np.float32)
    uv = np.stack([(gx.ravel() / half + 1) / 2, (gy.ravel() / half + 1) / 2]).astype(np.float32)
    alb = np.tile(np.asarray(albedo, np.float32)[:, None], (1, n * n))
    return Mesh(pos, grid_faces(n, n), alb, uv)


def quad_light(centre, e1, e2) -> np.ndarray:
    """One light record (centre, e1, e2, unit normal along e1 x e2)."""
    c, a, b = (np.asarray(x, np.float64) for x in (centre, e1, e2))
    nrm = np.cross(a, b)
    nrm /= np.linalg.norm(nrm)
    return np.concatenate([c, a, b, nrm]).astype(np.float32)
