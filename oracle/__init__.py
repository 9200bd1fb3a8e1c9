"""CPU oracle for the light-stage face renderer (test infrastructure only).

This package is the plain, slow reference the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import it; the product path never does, and it shares no code with
the GPU library.  ``oracle.c`` holds the estimator (see its header for the
paper passages each part follows); this module is ctypes marshalling plus the
closing linear steps of the gradient chain, done with float64 numpy:

* d alpha = B_id^T (R^T dL/dv), d beta = B_exp^T (R^T dL/dv) and
  d delta = B_alb^T dL/dA, the transposes of the blend (Face Modeling
  paragraph: identity, expression and albedo coefficients);
* d pose from dL/dR = sum_i dL/dv_i (x) v_model_i and dL/dt = sum_i dL/dv_i,
  with R = Rz(rz) Ry(ry) Rx(rx) (the [R t] geometry transform).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
# FACERT_ORACLE_SANITIZE=1 selects the AddressSanitizer + UBSan build of the
# same source (oracle/sanitize.py runs the oracle's pins under it)
SANITIZE = os.environ.get("FACERT_ORACLE_SANITIZE") == "1"
LIB_PATH = os.path.join(HERE, "liboracle_asan.so" if SANITIZE else "liboracle.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

FLAG_INTERIOR, FLAG_PRIMARY, FLAG_SECONDARY = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        extra = SAN_FLAGS if SANITIZE else []
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", *extra,
                               "-fPIC", "-shared", "-pthread", "-o", LIB_PATH, SRC, "-lm"])
    return LIB_PATH


class _Scene(C.Structure):
    _fields_ = [("V", C.c_int32), ("F", C.c_int32),
                ("faces", C.c_void_p), ("pos", C.c_void_p), ("pos_d", C.c_void_p),
                ("alb", C.c_void_p), ("uv", C.c_void_p),
                ("W", C.c_int32), ("H", C.c_int32),
                ("cam", C.c_float * 3), ("pix_scale", C.c_float),
                ("n_lights", C.c_int32), ("light_geom", C.c_void_p), ("light_rgb", C.c_void_p),
                ("spec_res", C.c_int32), ("spec", C.c_void_p)]


class _Grads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("d_light", "d_spec", "d_pos", "d_alb",
                                          "d_pos_interior", "d_pos_primary", "d_pos_secondary")]


class Counts(C.Structure):
    _fields_ = [("camera", C.c_int64), ("shadow", C.c_int64),
                ("edge_primary", C.c_int64), ("edge_secondary", C.c_int64)]

    def total(self) -> int:
        return self.camera + self.shadow + self.edge_primary + self.edge_secondary


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        L.orc_philox.argtypes = [C.c_uint32] * 6 + [vp]
        L.orc_rotation.argtypes = [vp, vp]
        L.orc_blend_geometry.argtypes = [i32, i32, i32] + [vp] * 8
        L.orc_blend_albedo.argtypes = [i32, i32, vp, vp, vp, vp]
        L.orc_vertex_normals.argtypes = [i32, i32, vp, vp, vp]
        L.orc_build_edges.argtypes = [i32, i32, vp, vp]
        L.orc_build_edges.restype = i32
        L.orc_ray_tri.argtypes = [vp] * 5 + [C.c_float, C.c_float] + [vp] * 4
        L.orc_closest_hit.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_closest_hit.restype = i32
        L.orc_any_hit.argtypes = [vp, C.c_int, vp, vp, i32]
        L.orc_render.argtypes = [vp, u64, i32, i32, vp, vp]
        L.orc_render_pixels.argtypes = [vp, u64, i32, i32, vp, i32, vp]
        L.orc_aov_pixels.argtypes = [vp, u64, i32, i32, vp, i32, vp]
        L.orc_record_decisions.argtypes = [vp, u64, i32, i32, vp]
        L.orc_render_frozen.argtypes = [vp, u64, i32, vp, i32, vp]
        L.orc_backward.argtypes = [vp, u64, i32, vp, i32, i32, vp, vp]
        L.orc_backward_frozen.argtypes = [vp, u64, i32, vp, vp, i32, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------- pieces ----

def philox(key: int, ctr) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox(key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF, *[int(c) for c in ctr], _p(out))
    return out


def rotation(pose) -> np.ndarray:
    pose = np.ascontiguousarray(pose, np.float32)
    R = np.zeros(9)
    lib().orc_rotation(_p(pose), _p(R))
    return R.reshape(3, 3)


def blend(model, params):
    """(v_model, v, A, R) in float64; v, v_model, A are [3][V]."""
    V = model.n_vertices
    vm = np.zeros((3, V)); v = np.zeros((3, V)); A = np.zeros((3, V))
    a = np.ascontiguousarray(params.alpha, np.float32)
    b = np.ascontiguousarray(params.beta, np.float32)
    d = np.ascontiguousarray(params.delta, np.float32)
    pose = np.ascontiguousarray(params.pose, np.float32)
    lib().orc_blend_geometry(V, model.b_id.shape[0], model.b_exp.shape[0], _p(model.mean),
                             _p(model.b_id), _p(model.b_exp), _p(a), _p(b), _p(pose), _p(vm), _p(v))
    lib().orc_blend_albedo(V, model.b_alb.shape[0], _p(model.alb_mean), _p(model.b_alb), _p(d), _p(A))
    return vm, v, A, rotation(pose)


def vertex_normals(faces: np.ndarray, pos: np.ndarray) -> np.ndarray:
    pos = np.ascontiguousarray(pos, np.float64)
    faces = np.ascontiguousarray(faces, np.int32)
    out = np.zeros_like(pos)
    lib().orc_vertex_normals(pos.shape[1], faces.shape[0], _p(faces), _p(pos), _p(out))
    return out


def build_edges(faces: np.ndarray, V: int) -> np.ndarray:
    faces = np.ascontiguousarray(faces, np.int32)
    out = np.zeros((3 * faces.shape[0], 4), np.int32)
    E = lib().orc_build_edges(V, faces.shape[0], _p(faces), _p(out))
    if E < 0:
        raise ValueError("non-manifold mesh")
    return out[:E].copy()


# ------------------------------------------------------------- scenes ----

@dataclass
class OScene:
    """Arrays kept alive for an orc_scene."""
    faces: np.ndarray
    pos: np.ndarray        # float32 [3][V]
    pos_d: np.ndarray      # float64 [3][V]
    alb: np.ndarray        # float64 [3][V]
    uv: np.ndarray         # float32 [2][V]
    width: int
    height: int
    cam: np.ndarray
    pix_scale: float
    light_geom: np.ndarray  # float32 [n][12]
    light_rgb: np.ndarray   # float64 [n][3]
    spec: np.ndarray        # float64 [res*res]
    spec_res: int = 32

    def struct(self) -> _Scene:
        for k in ("faces", "pos", "pos_d", "alb", "uv", "light_geom", "light_rgb", "spec"):
            a = getattr(self, k)
            assert a.flags.c_contiguous, k
        s = _Scene()
        s.V, s.F = self.pos.shape[1], self.faces.shape[0]
        s.faces, s.pos, s.pos_d = _p(self.faces), _p(self.pos), _p(self.pos_d)
        s.alb, s.uv = _p(self.alb), _p(self.uv)
        s.W, s.H = self.width, self.height
        for i in range(3):
            s.cam[i] = float(self.cam[i])
        s.pix_scale = float(self.pix_scale)
        s.n_lights = self.light_geom.shape[0]
        s.light_geom, s.light_rgb = _p(self.light_geom), _p(self.light_rgb)
        s.spec_res, s.spec = self.spec_res, _p(self.spec)
        return s

    @property
    def V(self) -> int:
        return self.pos.shape[1]


def scene_from_model(model, scene, params):
    """Blend + pose in float64, positions rounded once to float32."""
    vm, v, A, R = blend(model, params)
    # the rendered mesh is the float32 rounding of the posed blend; the
    # estimator evaluates it in double
    v32 = v.astype(np.float32)
    osc = OScene(np.ascontiguousarray(model.faces, np.int32), v32, v32.astype(np.float64),
                 A, np.ascontiguousarray(model.uv, np.float32), scene.width, scene.height,
                 np.asarray(scene.cam, np.float32), float(scene.pix_scale),
                 np.ascontiguousarray(scene.light_geom, np.float32),
                 np.ascontiguousarray(params.lights, np.float64).reshape(-1, 3).copy(),
                 np.ascontiguousarray(params.spec, np.float64).copy(), scene.spec_res)
    return osc, vm, R


def scene_from_mesh(mesh, width, height, cam, pix_scale, light_geom, light_rgb, spec, spec_res=32):
    pos = np.ascontiguousarray(mesh.pos, np.float32)
    return OScene(np.ascontiguousarray(mesh.faces, np.int32), pos, pos.astype(np.float64),
                  np.ascontiguousarray(mesh.albedo, np.float64),
                  np.ascontiguousarray(mesh.uv, np.float32), width, height,
                  np.asarray(cam, np.float32), float(np.float32(pix_scale)),
                  np.ascontiguousarray(light_geom, np.float32).reshape(-1, 12),
                  np.ascontiguousarray(light_rgb, np.float64).reshape(-1, 3),
                  np.ascontiguousarray(spec, np.float64).ravel(), spec_res)


# ------------------------------------------------------------ estimator --

def render(osc: OScene, seed: int, spp: int, threads: int | None = None, counts: bool = False):
    st = osc.struct()
    img = np.zeros((osc.height, osc.width, 3))
    cnt = Counts()
    r = lib().orc_render(C.byref(st), seed, spp, threads or default_threads(), _p(img), C.byref(cnt))
    if r:
        raise ValueError("orc_render failed")
    return (img, cnt) if counts else img


def render_pixels(osc: OScene, seed: int, spp: int, pixels, threads: int | None = None):
    st = osc.struct()
    pix = np.ascontiguousarray(pixels, np.int32)
    out = np.zeros((pix.size, 3))
    lib().orc_render_pixels(C.byref(st), seed, spp, pix.size, _p(pix), threads or default_threads(), _p(out))
    return out


def aov(osc: OScene, seed: int, spp: int, pixels=None, threads: int | None = None):
    """Auxiliary buffers [n][7] (albedo RGB, normal xyz, depth) of the given
    flat pixel indices (all pixels, as [H][W][7], when pixels is None)."""
    st = osc.struct()
    full = pixels is None
    pix = np.arange(osc.height * osc.width, dtype=np.int32) if full else np.ascontiguousarray(pixels, np.int32)
    out = np.zeros((pix.size, 7))
    if lib().orc_aov_pixels(C.byref(st), seed, spp, pix.size, _p(pix), threads or default_threads(), _p(out)):
        raise ValueError("orc_aov_pixels failed")
    return out.reshape(osc.height, osc.width, 7) if full else out


def record(osc: OScene, seed: int, spp: int, threads: int | None = None):
    st = osc.struct()
    rec = np.zeros((osc.height * osc.width * spp, 9), np.int32)
    if lib().orc_record_decisions(C.byref(st), seed, spp, threads or default_threads(), _p(rec)):
        raise ValueError("record failed")
    return rec


def render_frozen(osc: OScene, seed: int, spp: int, rec, threads: int | None = None):
    st = osc.struct()
    img = np.zeros((osc.height, osc.width, 3))
    lib().orc_render_frozen(C.byref(st), seed, spp, _p(rec), threads or default_threads(), _p(img))
    return img


def _grad_bufs(osc: OScene):
    V, n = osc.V, osc.light_geom.shape[0]
    return {"d_light": np.zeros((n, 3)), "d_spec": np.zeros(osc.spec_res ** 2),
            "d_pos": np.zeros((3, V)), "d_alb": np.zeros((3, V)),
            "d_pos_interior": np.zeros((3, V)), "d_pos_primary": np.zeros((3, V)),
            "d_pos_secondary": np.zeros((3, V))}


def backward(osc: OScene, seed: int, spp: int, dLdI, flags: int = 7,
             threads: int | None = None, counts: bool = False):
    st = osc.struct()
    dL = np.ascontiguousarray(dLdI, np.float64).reshape(osc.height, osc.width, 3)
    g = _grad_bufs(osc)
    gs = _Grads(*[_p(g[k]) for k, _ in _Grads._fields_])
    cnt = Counts()
    if lib().orc_backward(C.byref(st), seed, spp, _p(dL), flags, threads or default_threads(),
                          C.byref(gs), C.byref(cnt)):
        raise ValueError("orc_backward failed")
    return (g, cnt) if counts else g


def backward_frozen(osc: OScene, seed: int, spp: int, rec, dLdI, threads: int | None = None):
    st = osc.struct()
    dL = np.ascontiguousarray(dLdI, np.float64).reshape(osc.height, osc.width, 3)
    g = _grad_bufs(osc)
    gs = _Grads(*[_p(g[k]) for k, _ in _Grads._fields_])
    lib().orc_backward_frozen(C.byref(st), seed, spp, _p(rec), _p(dL), threads or default_threads(), C.byref(gs))
    return g


# ------------------------------------------------------------ loss -------

def loss_l2(image, target):
    """E_data of Eq. 1 over all pixels and channels, and its image gradient:
    (sum (I - T)^2, 2 (I - T)), float64."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return float(np.sum(d * d)), 2.0 * d


# ------------------------------------------------------ parameter chain --

def _drot(pose):
    """dR/d(rx, ry, rz) for R = Rz Ry Rx, float64."""
    rx, ry, rz = (float(x) for x in np.asarray(pose, np.float32)[:3])
    cx, sx, cy, sy, cz, sz = np.cos(rx), np.sin(rx), np.cos(ry), np.sin(ry), np.cos(rz), np.sin(rz)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    dRx = np.array([[0, 0, 0], [0, -sx, -cx], [0, cx, -sx]])
    dRy = np.array([[-sy, 0, cy], [0, 0, 0], [-cy, 0, -sy]])
    dRz = np.array([[-sz, -cz, 0], [cz, -sz, 0], [0, 0, 0]])
    return [Rz @ Ry @ dRx, Rz @ dRy @ Rx, dRz @ Ry @ Rx]


def parameter_grads(model, params, v_model, R, d_pos, d_alb):
    """Chain dL/dv (posed positions) and dL/dA into alpha, beta, delta, pose."""
    gm = R.T @ d_pos                                   # dL/dv_model, [3][V]
    flat = gm.reshape(-1)
    d_alpha = model.b_id.reshape(model.b_id.shape[0], -1).astype(np.float64) @ flat
    d_beta = model.b_exp.reshape(model.b_exp.shape[0], -1).astype(np.float64) @ flat
    d_delta = model.b_alb.reshape(model.b_alb.shape[0], -1).astype(np.float64) @ d_alb.reshape(-1)
    dR = d_pos @ v_model.T                             # sum_i d_v_i v_model_i^T
    d_pose = np.array([np.sum(dR * m) for m in _drot(params.pose)] + list(d_pos.sum(axis=1)))
    return {"d_alpha": d_alpha, "d_beta": d_beta, "d_delta": d_delta, "d_pose": d_pose}
