"""Python binding of libfacert.so (ctypes; argument marshalling only).

The functions ``fr_create`` ... ``fr_destroy`` are the C-ABI entry points of
include/facert.h with the same names and arguments.  ``Renderer`` keeps a
context and the model arrays together and passes torch device tensors (their
``data_ptr``) and the current HIP stream; ``FaceRender`` is the autograd
function whose backward is fr_backward.  Every step of the render and the
adjoint runs in the HIP kernels; if the library is missing this module raises
instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfacert.so")

FR_TIMING = 1
FR_REFIT = 2
FR_DEVICE_PTRS = 4
FR_CHUNK_MAX = 1 << 22
FR_TERM_INTERIOR, FR_TERM_PRIMARY, FR_TERM_SECONDARY = 1, 2, 4
STATUS = {0: "FR_OK", -1: "FR_EINVAL", -2: "FR_ENOMEM", -3: "FR_EDEVICE", -4: "FR_ESTATE"}


class FrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class fr_model_desc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_faces", C.c_int32), ("n_id", C.c_int32),
                ("n_exp", C.c_int32), ("n_alb", C.c_int32), ("faces", C.c_void_p),
                ("mean", C.c_void_p), ("b_id", C.c_void_p), ("b_exp", C.c_void_p),
                ("alb_mean", C.c_void_p), ("b_alb", C.c_void_p), ("uv", C.c_void_p)]


class fr_scene_desc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("cam", C.c_float * 3),
                ("pix_scale", C.c_float), ("n_lights", C.c_int32), ("light_geom", C.c_void_p),
                ("spec_res", C.c_int32)]


class fr_params(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("alpha", "beta", "delta", "pose", "lights", "spec")]


class fr_grads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("d_lights", "d_spec", "d_vertices", "d_albedo",
                                          "d_alpha", "d_beta", "d_delta", "d_pose")]


class fr_stats_t(C.Structure):
    _fields_ = [("rays_camera", C.c_uint64), ("rays_shadow", C.c_uint64),
                ("rays_edge_primary", C.c_uint64), ("rays_edge_secondary", C.c_uint64),
                ("traversal_overflow", C.c_uint64), ("box_tests", C.c_uint64), ("tri_tests", C.c_uint64),
                ("kernel_rays", C.c_uint64 * 6), ("kernel_box_tests", C.c_uint64 * 6),
                ("kernel_tri_tests", C.c_uint64 * 6), ("kernel_shades", C.c_uint64 * 6),
                ("ms_blend", C.c_float), ("ms_bvh", C.c_float),
                ("ms_edges", C.c_float), ("ms_render", C.c_float), ("ms_backward", C.c_float),
                ("ms_kernel", C.c_float * 6)]


KERNELS = ("k_cam", "k_sh_trace", "k_fwd_shade", "k_render_adj", "k_edge_primary", "k_edge_secondary")


class fr_launch(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tile", C.c_int32)]


FR_LAUNCH_FLAT, FR_LAUNCH_XCD = 0, 1

EXPORTS = ("fr_create", "fr_set_stream", "fr_set_terms", "fr_set_chunk", "fr_blend", "fr_render", "fr_backward",
           "fr_loss_l2", "fr_loss_l2_noalloc", "fr_aov", "fr_light_reg", "fr_adam", "fr_stats", "fr_last_error", "fr_destroy",
           "fr_batch_create", "fr_batch_set_stream", "fr_batch_render", "fr_batch_backward", "fr_batch_num_kinds",
           "fr_batch_kind_name", "fr_batch_get_launch", "fr_batch_set_launch", "fr_batch_tune", "fr_batch_timing",
           "fr_batch_capture_begin", "fr_batch_capture_end", "fr_batch_graph_launch", "fr_batch_last_error",
           "fr_batch_destroy")

_lib = None

# Contexts and batches still open at interpreter exit are closed by an exit
# handler registered after torch's, so it runs first: destroying them later,
# once the HIP runtime is being torn down, can stall the process.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def load():
    """Load libfacert.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with "
                                    "`python -m paper_1910_05200_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, u64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64
        L.fr_create.argtypes = [C.POINTER(fr_model_desc), C.POINTER(fr_scene_desc), u32, C.POINTER(vp)]
        L.fr_set_stream.argtypes = [vp, vp]
        L.fr_set_terms.argtypes = [vp, u32]
        L.fr_set_chunk.argtypes = [vp, i32]
        L.fr_blend.argtypes = [vp] * 7
        L.fr_render.argtypes = [vp, C.POINTER(fr_params), u64, i32, vp]
        L.fr_backward.argtypes = [vp, vp, C.POINTER(fr_grads)]
        L.fr_loss_l2.argtypes = [vp] * 5
        L.fr_loss_l2_noalloc.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
        L.fr_aov.argtypes = [vp, vp]
        L.fr_light_reg.argtypes = [vp, vp, C.c_float, vp, vp]
        L.fr_adam.argtypes = [vp, vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float, C.c_float]
        L.fr_stats.argtypes = [vp, C.POINTER(fr_stats_t)]
        L.fr_last_error.argtypes = [vp]
        L.fr_last_error.restype = C.c_char_p
        L.fr_destroy.argtypes = [vp]
        L.fr_destroy.restype = None
        L.fr_batch_create.argtypes = [i32, vp, u32, C.POINTER(vp)]
        L.fr_batch_set_stream.argtypes = [vp, vp]
        L.fr_batch_render.argtypes = [vp, vp, vp, vp, vp]
        L.fr_batch_backward.argtypes = [vp, vp, vp]
        L.fr_batch_num_kinds.argtypes = []
        L.fr_batch_kind_name.argtypes = [i32]
        L.fr_batch_kind_name.restype = C.c_char_p
        L.fr_batch_get_launch.argtypes = [vp, i32, C.POINTER(fr_launch)]
        L.fr_batch_set_launch.argtypes = [vp, i32, C.POINTER(fr_launch)]
        L.fr_batch_tune.argtypes = [vp, i32, vp]
        L.fr_batch_timing.argtypes = [vp, vp, vp, vp]
        for n in ("fr_batch_capture_begin", "fr_batch_capture_end", "fr_batch_graph_launch"):
            getattr(L, n).argtypes = [vp]
        L.fr_batch_last_error.argtypes = [vp]
        L.fr_batch_last_error.restype = C.c_char_p
        L.fr_batch_destroy.argtypes = [vp]
        L.fr_batch_destroy.restype = None
        for n in EXPORTS:
            if n not in ("fr_last_error", "fr_destroy", "fr_batch_kind_name", "fr_batch_last_error",
                         "fr_batch_destroy"):
                getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def _check(ctx, code: int):
    if code != 0:
        msg = load().fr_last_error(ctx)
        raise FrError(code, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


class Renderer:
    """One fr_ctx plus the host copies it was created from.

    model/scene: ``synth.Model`` / ``synth.Scene``.  Parameter tensors passed
    to ``render`` must be contiguous float32 on the current HIP device, except
    ``pose`` (6 floats, host).
    """

    def __init__(self, model, scene, timing: bool = False, refit: bool = False, host_ptrs: bool = False):
        import torch
        self.torch = torch
        self.host = host_ptrs
        L = load()
        self._keep = {k: np.ascontiguousarray(getattr(model, k)) for k in
                      ("faces", "mean", "b_id", "b_exp", "alb_mean", "b_alb", "uv")}
        self._keep["faces"] = np.ascontiguousarray(self._keep["faces"], np.int32)
        for k in ("mean", "b_id", "b_exp", "alb_mean", "b_alb", "uv"):
            self._keep[k] = np.ascontiguousarray(self._keep[k], np.float32)
        self._lg = np.ascontiguousarray(scene.light_geom, np.float32)
        k = self._keep
        md = fr_model_desc(model.n_vertices, model.n_faces, k["b_id"].shape[0], k["b_exp"].shape[0],
                           k["b_alb"].shape[0], *(k[n].ctypes.data for n in
                                                  ("faces", "mean", "b_id", "b_exp", "alb_mean", "b_alb", "uv")))
        sd = fr_scene_desc(scene.width, scene.height, (C.c_float * 3)(*[float(x) for x in scene.cam]),
                           float(scene.pix_scale), self._lg.shape[0], self._lg.ctypes.data, scene.spec_res)
        ctx = C.c_void_p()
        flags = (FR_TIMING if timing else 0) | (FR_REFIT if refit else 0) | (0 if host_ptrs else FR_DEVICE_PTRS)
        code = L.fr_create(C.byref(md), C.byref(sd), flags, C.byref(ctx))
        if code != 0:
            raise FrError(code, "fr_create failed")
        self.ctx = ctx
        self.V, self.F = model.n_vertices, model.n_faces
        self.W, self.H = scene.width, scene.height
        self.n_lights = self._lg.shape[0]
        self.spec_res = scene.spec_res
        self.n_id, self.n_exp, self.n_alb = md.n_id, md.n_exp, md.n_alb
        self.render_token = 0
        self._last = None
        _live.add(self)

    # -- plumbing
    def _stream(self):
        _check(self.ctx, load().fr_set_stream(self.ctx, self.torch.cuda.current_stream().cuda_stream))

    def close(self):
        if getattr(self, "ctx", None):
            load().fr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_terms(self, terms: int):
        _check(self.ctx, load().fr_set_terms(self.ctx, terms))

    def set_chunk(self, samples: int):
        _check(self.ctx, load().fr_set_chunk(self.ctx, samples))

    def _empty(self, shape, like=None):
        """An output array: numpy in host-pointer mode, else a float32 tensor
        on like's device (the current HIP device without like)."""
        if self.host:
            return np.empty(shape, np.float32)
        dev = like.device if like is not None else "cuda"
        return self.torch.empty(shape, device=dev, dtype=self.torch.float32)

    # -- calls (host-pointer mode: numpy arrays in and out, each call waits)
    def blend(self, alpha, beta, delta, pose):
        self._stream()
        v = self._empty((3, self.V), alpha)
        a = self._empty((3, self.V), alpha)
        pose_h = np.ascontiguousarray(np.asarray(pose, np.float32).reshape(6))
        _check(self.ctx, load().fr_blend(self.ctx, _ptr(alpha), _ptr(beta), _ptr(delta),
                                         pose_h.ctypes.data, _ptr(v), _ptr(a)))
        return v, a

    def render(self, p: dict, seed: int, spp: int, out=None):
        self._stream()
        if out is None:
            out = self._empty((self.H, self.W, 3), p["lights"])
        pose_h = np.ascontiguousarray(np.asarray(p["pose"], np.float32).reshape(6))
        fp = fr_params(_ptr(p["alpha"]), _ptr(p["beta"]), _ptr(p["delta"]), pose_h.ctypes.data,
                       _ptr(p["lights"]), _ptr(p["spec"]))
        _check(self.ctx, load().fr_render(self.ctx, C.byref(fp), seed, spp, _ptr(out)))
        self.render_token += 1
        self._last = (p, pose_h)          # keep the arrays alive for fr_backward
        return out

    def backward(self, dL_dimage, want=("d_lights", "d_spec", "d_vertices", "d_albedo",
                                         "d_alpha", "d_beta", "d_delta", "d_pose")):
        self._stream()
        shapes = {"d_lights": (self.n_lights, 3), "d_spec": (self.spec_res ** 2,),
                  "d_vertices": (3, self.V), "d_albedo": (3, self.V), "d_alpha": (self.n_id,),
                  "d_beta": (self.n_exp,), "d_delta": (self.n_alb,), "d_pose": (6,)}
        out = {k: self._empty(shapes[k], dL_dimage) for k in want}
        g = fr_grads(*[_ptr(out.get(k)) for k, _ in fr_grads._fields_])
        dl = np.ascontiguousarray(dL_dimage, np.float32) if self.host else dL_dimage.contiguous()
        _check(self.ctx, load().fr_backward(self.ctx, _ptr(dl), C.byref(g)))
        return out

    def loss_l2(self, image, target):
        self._stream()
        dL = self._empty(tuple(image.shape), image)
        loss = self._empty((), image)
        _check(self.ctx, load().fr_loss_l2(self.ctx, _ptr(image), _ptr(target), _ptr(dL), _ptr(loss)))
        return dL, loss

    def aov(self, out=None):
        """Albedo, shading normal and depth of the last render, [H][W][7]."""
        self._stream()
        if out is None:
            out = self._empty((self.H, self.W, 7))
        _check(self.ctx, load().fr_aov(self.ctx, _ptr(out)))
        return out

    def light_reg(self, lights, w2: float, grad=None):
        """w2 E_light (device scalar); adds its gradient to grad when given."""
        self._stream()
        loss = self._empty((), lights)
        _check(self.ctx, load().fr_light_reg(self.ctx, _ptr(lights), float(w2), _ptr(grad), _ptr(loss)))
        return loss

    def adam(self, param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        """One in-place Adam step on contiguous float32 arrays of equal size
        (device tensors, or numpy arrays in host-pointer mode)."""
        self._stream()
        if self.host:
            n = param.size
            for x in (param, grad, m, v):
                assert x.size == n and x.flags.c_contiguous and x.dtype == np.float32
        else:
            n = param.numel()
            for x in (grad, m, v):
                assert x.numel() == n and x.is_contiguous() and x.dtype == param.dtype
            assert param.is_contiguous()
        _check(self.ctx, load().fr_adam(self.ctx, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), n, step,
                                        float(lr), float(beta1), float(beta2), float(eps)))

    def stats(self) -> dict:
        s = fr_stats_t()
        _check(self.ctx, load().fr_stats(self.ctx, C.byref(s)))
        out = {}
        for k, _ in fr_stats_t._fields_:
            v = getattr(s, k)
            out[k] = list(v) if isinstance(v, C.Array) else v
        return out


def _bcheck(batch, code: int):
    if code != 0:
        msg = load().fr_batch_last_error(batch)
        raise FrError(code, msg.decode() if msg else "")


GRAD_KEYS = ("d_lights", "d_spec", "d_vertices", "d_albedo", "d_alpha", "d_beta", "d_delta", "d_pose")


class Batch:
    """Several Renderers evaluated together (fr_batch_*): one kernel launch
    per pipeline step for all of them.  Work runs on torch's current stream,
    which becomes the stream of every renderer of the batch."""

    def __init__(self, renderers, timing: bool = False):
        import torch
        self.torch = torch
        self.rs = list(renderers)
        n = len(self.rs)
        arr = (C.c_void_p * n)(*[r.ctx.value for r in self.rs])
        b = C.c_void_p()
        code = load().fr_batch_create(n, arr, FR_TIMING if timing else 0, C.byref(b))
        if code != 0:
            raise FrError(code, "fr_batch_create failed")
        self.b = b
        self.n = n
        self._keep = None
        _live.add(self)
        self.kinds = [load().fr_batch_kind_name(k).decode() for k in range(load().fr_batch_num_kinds())]

    def _stream(self):
        _bcheck(self.b, load().fr_batch_set_stream(self.b, self.torch.cuda.current_stream().cuda_stream))

    def close(self):
        if getattr(self, "b", None):
            load().fr_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def render(self, params, seeds, spps, outs=None):
        """params: list of dicts as Renderer.render takes; returns the images
        (written into outs when given)."""
        t = self.torch
        self._stream()
        n = self.n
        if outs is None:
            outs = [t.empty((r.H, r.W, 3), device="cuda", dtype=t.float32) for r in self.rs]
        poses = [np.ascontiguousarray(np.asarray(p["pose"], np.float32).reshape(6)) for p in params]
        fp = (fr_params * n)(*[fr_params(_ptr(p["alpha"]), _ptr(p["beta"]), _ptr(p["delta"]), ph.ctypes.data,
                                         _ptr(p["lights"]), _ptr(p["spec"])) for p, ph in zip(params, poses)])
        sd = (C.c_uint64 * n)(*[int(s) for s in seeds])
        sp = (C.c_int32 * n)(*[int(s) for s in spps])
        op = (C.c_void_p * n)(*[_ptr(o) for o in outs])
        _bcheck(self.b, load().fr_batch_render(self.b, fp, sd, sp, op))
        for r in self.rs:
            r.render_token += 1
        self._keep = (params, poses, outs)
        return outs

    def backward(self, dLs, want=GRAD_KEYS, outs=None):
        """dLs: image gradients; returns one dict of gradients per instance
        (written into outs, a list of such dicts, when given)."""
        t = self.torch
        self._stream()
        if outs is None:
            outs = []
            for r in self.rs:
                shapes = {"d_lights": (r.n_lights, 3), "d_spec": (r.spec_res ** 2,), "d_vertices": (3, r.V),
                          "d_albedo": (3, r.V), "d_alpha": (r.n_id,), "d_beta": (r.n_exp,), "d_delta": (r.n_alb,),
                          "d_pose": (6,)}
                outs.append({k: t.empty(shapes[k], device="cuda", dtype=t.float32) for k in want})
        g = (fr_grads * self.n)(*[fr_grads(*[_ptr(o.get(k)) for k, _ in fr_grads._fields_]) for o in outs])
        dp = (C.c_void_p * self.n)(*[_ptr(d) for d in dLs])
        _bcheck(self.b, load().fr_batch_backward(self.b, dp, g))
        self._keep_bwd = (dLs, outs)
        return outs

    def get_launch(self, kind) -> tuple:
        k = self.kinds.index(kind) if isinstance(kind, str) else kind
        L = fr_launch()
        _bcheck(self.b, load().fr_batch_get_launch(self.b, k, C.byref(L)))
        return L.mode, L.tile

    def set_launch(self, kind, mode: int, tile: int = 0):
        k = self.kinds.index(kind) if isinstance(kind, str) else kind
        L = fr_launch(mode, tile)
        _bcheck(self.b, load().fr_batch_set_launch(self.b, k, C.byref(L)))

    def tune(self, trials: int = 2) -> dict:
        """Autotune the launch of each tunable kind on the last render and
        backward; returns {kind: (launch, best ms)} of the tuned kinds."""
        ms = (C.c_float * len(self.kinds))()
        _bcheck(self.b, load().fr_batch_tune(self.b, trials, ms))
        return {k: (self.get_launch(i), ms[i]) for i, k in enumerate(self.kinds) if ms[i] > 0}

    def timing(self) -> dict:
        ms = (C.c_float * len(self.kinds))()
        r, b = C.c_float(), C.c_float()
        _bcheck(self.b, load().fr_batch_timing(self.b, ms, C.byref(r), C.byref(b)))
        out = {k: ms[i] for i, k in enumerate(self.kinds)}
        out["render"], out["backward"] = r.value, b.value
        return out

    def capture_begin(self):
        self._stream()
        _bcheck(self.b, load().fr_batch_capture_begin(self.b))

    def capture_end(self):
        _bcheck(self.b, load().fr_batch_capture_end(self.b))

    def graph_launch(self):
        self._stream()
        _bcheck(self.b, load().fr_batch_graph_launch(self.b))


def loss_l2_noalloc(image, target, dL=None, loss=None, want_dL=True):
    """fr_loss_l2_noalloc on torch's current stream: E_data and 2 (I - T) of
    n = image.numel() elements with no context and no device allocation by
    the library (outputs are written into dL / loss when given, else new
    tensors).  Returns (dL or None, loss)."""
    import torch
    assert image.is_contiguous() and target.is_contiguous() and image.numel() == target.numel()
    if want_dL and dL is None:
        dL = torch.empty_like(image)
    if loss is None:
        loss = torch.empty((), device=image.device, dtype=torch.float32)
    code = load().fr_loss_l2_noalloc(torch.cuda.current_stream().cuda_stream, _ptr(image), _ptr(target),
                                     image.numel(), _ptr(dL) if want_dL else None, _ptr(loss))
    if code != 0:
        raise FrError(code, load().fr_last_error(None).decode())
    return dL, loss


def params_to_device(params, device="cuda"):
    """synth.Params -> dict of device tensors (pose stays on the host)."""
    import torch
    d = {k: torch.from_numpy(np.ascontiguousarray(getattr(params, k), np.float32)).to(device)
         for k in ("alpha", "beta", "delta", "lights", "spec")}
    d["pose"] = np.asarray(params.pose, np.float32).copy()
    return d


def _render_inputs(alpha, beta, delta, pose, lights, spec) -> dict:
    """Renderer.render's parameter dict from tensors (pose copied to the host)."""
    return {"alpha": alpha.detach().contiguous(), "beta": beta.detach().contiguous(),
            "delta": delta.detach().contiguous(), "pose": pose.detach().cpu().numpy(),
            "lights": lights.detach().contiguous(), "spec": spec.detach().contiguous()}


def _make_autograd():
    import torch

    class FaceRender(torch.autograd.Function):
        """image = F(alpha, beta, delta, pose, lights, spec; seed, spp).

        The backward is fr_backward, which replays the forward's samples
        (same seed and spp): it reads the hit records and visibility masks
        that fr_render kept when the render fitted one chunk of samples, and
        recomputes them chunk by chunk otherwise.  If another render used the
        renderer in between, the forward is rendered again from the saved
        inputs first.  The inputs are saved with save_for_backward, so an
        in-place change to one of them between forward and backward (say an
        optimiser step) raises instead of differentiating other values."""

        @staticmethod
        def forward(ctx, renderer, seed, spp, alpha, beta, delta, pose, lights, spec):
            p = _render_inputs(alpha, beta, delta, pose, lights, spec)
            img = renderer.render(p, seed, spp)
            ctx.save_for_backward(alpha, beta, delta, pose, lights, spec)
            ctx.renderer, ctx.seed, ctx.spp = renderer, seed, spp
            ctx.token = renderer.render_token
            return img

        @staticmethod
        def backward(ctx, grad_img):
            alpha, beta, delta, pose, lights, spec = ctx.saved_tensors   # raises if modified in place
            r = ctx.renderer
            if r.render_token != ctx.token:       # another render ran since: replay this one
                r.render(_render_inputs(alpha, beta, delta, pose, lights, spec), ctx.seed, ctx.spp)
            g = r.backward(grad_img.contiguous(), want=("d_alpha", "d_beta", "d_delta", "d_pose",
                                                        "d_lights", "d_spec"))
            return (None, None, None, g["d_alpha"], g["d_beta"], g["d_delta"],
                    g["d_pose"].to(pose.device), g["d_lights"], g["d_spec"])

    return FaceRender


_face_render = None


def face_render(renderer, seed, spp, alpha, beta, delta, pose, lights, spec):
    """Differentiable render (torch autograd) through fr_render/fr_backward."""
    global _face_render
    if _face_render is None:
        _face_render = _make_autograd()
    return _face_render.apply(renderer, seed, spp, alpha, beta, delta, pose, lights, spec)
