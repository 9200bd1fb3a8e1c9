"""Learned denoiser for low-spp renders (binding of libfadenoise.so, training
and evaluation driver).

The paper names the ray tracer's sampling rate as its limitation: few
samples give a noisy render, many give slow optimisation (Results and
Conclusion paragraph).  The denoiser maps a low-spp render plus its albedo,
normal and depth buffers (fr_aov) to an estimate of the converged image.
Training pairs come from the renderer itself: a low-spp render of a random
scene and a high-spp render of the same scene.

    python -m paper_1910_05200_amd.denoise --pairs 400 --epochs 6

trains from a seeded initialisation and prints one JSON line: training time,
loss curve, and for held-out scenes the PSNR (against a 1024-spp reference)
of the denoised 2-spp image beside plain renders at 2..256 spp, with the
time each takes.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1910_05200_amd import facert, synth

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfadenoise.so")
EXPORTS = ("fd_create", "fd_create_batch", "fd_set_stream", "fd_num_params", "fd_layer_shape", "fd_set_params", "fd_get_params",
           "fd_get_state", "fd_set_state", "fd_forward", "fd_train_step", "fd_backward_input", "fd_conv3x3",
           "fd_conv3x3_wgrad", "fd_last_error", "fd_destroy")

_lib = None


def load():
    """Load libfadenoise.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with `python -m paper_1910_05200_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.fd_create.argtypes = [i32, i32, C.POINTER(vp)]
        L.fd_create_batch.argtypes = [i32, i32, i32, C.POINTER(vp)]
        L.fd_set_stream.argtypes = [vp, vp]
        L.fd_num_params.argtypes = [vp]
        L.fd_num_params.restype = C.c_int64
        L.fd_layer_shape.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.fd_set_params.argtypes = [vp, vp]
        L.fd_get_params.argtypes = [vp, vp]
        L.fd_get_state.argtypes = [vp, vp, vp, vp, C.POINTER(i32)]
        L.fd_set_state.argtypes = [vp, vp, vp, vp, i32]
        L.fd_forward.argtypes = [vp, vp, vp, vp]
        L.fd_train_step.argtypes = [vp, vp, vp, vp, C.c_float, vp, vp]
        L.fd_backward_input.argtypes = [vp, vp, vp, vp]
        L.fd_conv3x3.argtypes = [vp, i32, i32, i32, i32, vp, i32, vp, vp, i32, vp]
        L.fd_conv3x3_wgrad.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, vp]
        L.fd_last_error.argtypes = [vp]
        L.fd_last_error.restype = C.c_char_p
        L.fd_destroy.argtypes = [vp]
        L.fd_destroy.restype = None
        for n in ("fd_create", "fd_create_batch", "fd_set_stream", "fd_layer_shape", "fd_set_params", "fd_get_params", "fd_get_state",
                  "fd_set_state", "fd_forward", "fd_train_step", "fd_backward_input", "fd_conv3x3",
                  "fd_conv3x3_wgrad"):
            getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


class FdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fadenoise error {code}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else t.data_ptr()


class Denoiser:
    """One network for n images of H x W per call (n = 1: arrays [H][W][c];
    n > 1: [n][H][W][c]); tensors are float32 on the device."""

    def __init__(self, height: int, width: int, n: int = 1):
        import torch
        self.torch = torch
        self.H, self.W, self.n = height, width, n
        net = C.c_void_p()
        code = load().fd_create_batch(height, width, n, C.byref(net))
        if code != 0:
            raise FdError(code, "fd_create_batch failed")
        self.net = net
        self.n_params = int(load().fd_num_params(net))

    def close(self):
        if getattr(self, "net", None):
            load().fd_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code != 0:
            raise FdError(code, load().fd_last_error(self.net).decode())

    def _stream(self):
        self._check(load().fd_set_stream(self.net, C.c_void_p(self.torch.cuda.current_stream().cuda_stream)))

    def layer_shapes(self):
        out, i = [], 0
        ci, co, k = C.c_int32(), C.c_int32(), C.c_int32()
        while load().fd_layer_shape(self.net, i, C.byref(ci), C.byref(co), C.byref(k)) == 0:
            out.append((ci.value, co.value, k.value))
            i += 1
        return out

    def set_params(self, params):
        self._stream()
        p = params.contiguous()
        assert p.numel() == self.n_params and p.dtype == self.torch.float32 and p.is_cuda
        self._check(load().fd_set_params(self.net, _ptr(p)))

    def get_params(self):
        self._stream()
        p = self.torch.empty(self.n_params, device="cuda", dtype=self.torch.float32)
        self._check(load().fd_get_params(self.net, _ptr(p)))
        return p

    def get_state(self) -> dict:
        """Parameters, Adam moments and step count (host arrays), for checkpoints."""
        self._stream()
        t = self.torch
        p, m, v = (t.empty(self.n_params, device="cuda", dtype=t.float32) for _ in range(3))
        step = C.c_int32()
        self._check(load().fd_get_state(self.net, _ptr(p), _ptr(m), _ptr(v), C.byref(step)))
        t.cuda.current_stream().synchronize()
        return {"params": p.cpu().numpy(), "m": m.cpu().numpy(), "v": v.cpu().numpy(),
                "step": np.int32(step.value)}

    def set_state(self, st: dict):
        self._stream()
        t = self.torch
        arrs = [t.from_numpy(np.ascontiguousarray(st[k], np.float32)).cuda() for k in ("params", "m", "v")]
        for a in arrs:
            assert a.numel() == self.n_params
        self._check(load().fd_set_state(self.net, *[_ptr(a) for a in arrs], int(st["step"])))
        t.cuda.current_stream().synchronize()

    def _shape(self, c):
        return (self.H, self.W, c) if self.n == 1 else (self.n, self.H, self.W, c)

    def forward(self, rgb, aux, out=None):
        self._stream()
        for a, c in ((rgb, 3), (aux, facert_aux_channels())):
            assert a.numel() == self.n * self.H * self.W * c
        if out is None:
            out = self.torch.empty(self._shape(3), device="cuda", dtype=self.torch.float32)
        self._check(load().fd_forward(self.net, _ptr(rgb.contiguous()), _ptr(aux.contiguous()), _ptr(out)))
        return out

    def backward_input(self, rgb, dL_dout, out=None):
        """Gradient with respect to the rgb input of the last forward."""
        self._stream()
        for a in (rgb, dL_dout):
            assert a.numel() == self.n * self.H * self.W * 3
        if out is None:
            out = self.torch.empty(self._shape(3), device="cuda", dtype=self.torch.float32)
        self._check(load().fd_backward_input(self.net, _ptr(rgb.contiguous()), _ptr(dL_dout.contiguous()), _ptr(out)))
        return out

    def train_step(self, rgb, aux, target, lr: float, want_grads: bool = False):
        self._stream()
        for a, c in ((rgb, 3), (aux, facert_aux_channels()), (target, 3)):
            assert a.numel() == self.n * self.H * self.W * c
        loss = self.torch.empty((), device="cuda", dtype=self.torch.float32)
        g = self.torch.empty(self.n_params, device="cuda", dtype=self.torch.float32) if want_grads else None
        self._check(load().fd_train_step(self.net, _ptr(rgb.contiguous()), _ptr(aux.contiguous()),
                                         _ptr(target.contiguous()), float(lr), _ptr(loss), _ptr(g)))
        return (loss, g) if want_grads else loss


def facert_aux_channels() -> int:
    """Channels of fr_aov's buffers (FD_IN_AUX): albedo, normal, depth."""
    return 7


def conv3x3(x, w_bf16, bias=None, relu=False, x_is_f32=False):
    """fd_conv3x3 on torch's current stream: x [H][W][cin] (int16 bfloat16
    bit patterns, or float32 when x_is_f32), w_bf16 [cout][9][cin] int16 ->
    y [H][W][cout] float32."""
    import torch
    H, W, cin = x.shape
    cout = w_bf16.shape[0]
    y = torch.empty((H, W, cout), device=x.device, dtype=torch.float32)
    code = load().fd_conv3x3(torch.cuda.current_stream().cuda_stream, H, W, cin, cout, _ptr(x.contiguous()),
                             1 if x_is_f32 else 0, _ptr(w_bf16.contiguous()), _ptr(bias), 1 if relu else 0, _ptr(y))
    if code != 0:
        raise FdError(code, "fd_conv3x3 failed")
    return y


def conv3x3_wgrad(x_bf16, g, want_bias=True):
    """fd_conv3x3_wgrad: (dw [cout][9][cin], db [cout] or None) float32."""
    import torch
    H, W, cin = x_bf16.shape
    cout = g.shape[-1]
    dw = torch.empty((cout, 9, cin), device=g.device, dtype=torch.float32)
    db = torch.empty(cout, device=g.device, dtype=torch.float32) if want_bias else None
    code = load().fd_conv3x3_wgrad(torch.cuda.current_stream().cuda_stream, H, W, cin, cout,
                                   _ptr(x_bf16.contiguous()), _ptr(g.contiguous()), _ptr(dw), _ptr(db))
    if code != 0:
        raise FdError(code, "fd_conv3x3_wgrad failed")
    return dw, db


def init_params(shapes, seed: int = 0) -> np.ndarray:
    """He-normal weights (fan-in k*k*Cin), zero biases; the first layer's
    weights on the six unused input channels are zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (ci, co, k) in enumerate(shapes):
        w = rng.normal(0.0, math.sqrt(2.0 / (k * k * ci)), (co, k * k, ci))
        if i == len(shapes) - 1:
            w *= 0.1                        # start the output near zero
        if i == 0:
            w[:, :, 10:] = 0.0
        parts += [w.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def psnr(img, ref) -> float:
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    mse = float(np.mean((img - ref) ** 2))
    peak = float(ref.max())
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def scene_params(i: int) -> synth.Params:
    """Training/evaluation scene i: a fresh identity, expression, albedo,
    pose and light set from the generator's parameter distribution."""
    return synth.make_params(10_000 + i)


def render_pair(r: facert.Renderer, i: int, spp_in: int, spp_ref: int, seed: int):
    """(low-spp render, its auxiliary buffers, high-spp render) of scene i."""
    p = facert.params_to_device(scene_params(i))
    ref = r.render(p, seed + 1, spp_ref).clone()
    rgb = r.render(p, seed, spp_in).clone()
    aux = r.aov()
    return rgb, aux, ref


def train(r: facert.Renderer, dn: Denoiser, pairs: int, epochs: int, spp_in: int = 2, spp_target: int = 256,
          lr: float = 1e-3, seed: int = 0, log=sys.stderr, first_pair: int = 0, state: dict | None = None,
          total_steps: int | None = None):
    """Renderer-generated pairs first_pair .. first_pair + pairs - 1, then
    epochs passes over them with Adam and a cosine-decaying step over
    total_steps (default: this call's steps).  Starts from a seeded
    initialisation, or from state (a checkpoint of get_state; its step count
    continues the schedule).  Returns (data seconds, training seconds, loss
    per epoch)."""
    import torch
    if state is None:
        dn.set_params(torch.from_numpy(init_params(dn.layer_shapes(), seed)).cuda())
        step0 = 0
    else:
        dn.set_state(state)
        step0 = int(state["step"])
    t0 = time.perf_counter()
    data = []
    for i in range(first_pair, first_pair + pairs):
        data.append(render_pair(r, i, spp_in, spp_target, 50_000 + 7 * i))
        if log and (i - first_pair + 1) % 500 == 0:
            torch.cuda.synchronize()
            print(f"rendered {i - first_pair + 1}/{pairs} pairs ({time.perf_counter() - t0:.0f} s)", file=log,
                  flush=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    rng = np.random.default_rng(seed + first_pair)
    losses = []
    steps = epochs * pairs
    total = total_steps or (step0 + steps)
    t0 = time.perf_counter()
    for ep in range(epochs):
        for k in rng.permutation(pairs):
            step = step0 + len(losses)
            rgb, aux, ref = data[k]
            losses.append(dn.train_step(rgb, aux, ref, lr * 0.5 * (1.0 + math.cos(math.pi * min(step, total) / total))))
        if log:
            print(f"epoch {ep}: loss {float(torch.stack(losses[-pairs:]).mean()):.5f} "
                  f"({time.perf_counter() - t0:.0f} s)", file=log, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    curve = [float(x) for x in torch.stack(losses).reshape(epochs, -1).mean(1)]
    return t_data, t_train, curve


def conv_flops(shapes, H: int, W: int) -> float:
    """Multiply-add FLOPs (2 per MAC) of one forward pass at H x W."""
    levels = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0]
    return float(sum(2.0 * (H >> lv) * (W >> lv) * k * k * ci * co for (ci, co, k), lv in zip(shapes, levels)))


def bench(H: int = 256, W: int = 256, reps: int = 20, n: int = 1) -> dict:
    """Time fd_forward, fd_backward_input and fd_train_step on n H x W images
    per call (seeded weights and inputs) with HIP events on the network's
    stream; times and FLOP rates are per call."""
    import torch
    dn = Denoiser(H, W, n=n)
    shapes = dn.layer_shapes()
    dn.set_params(torch.from_numpy(init_params(shapes, 0)).cuda())
    g = torch.Generator(device="cpu").manual_seed(0)
    shape = (H, W) if n == 1 else (n, H, W)
    rgb = (torch.rand(shape + (3,), generator=g) * 0.05).cuda()
    aux = torch.rand(shape + (7,), generator=g).cuda()
    tgt = (torch.rand(shape + (3,), generator=g) * 0.05).cuda()
    out = torch.empty_like(rgb)
    flops = n * conv_flops(shapes, H, W)

    def timed(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_f = timed(lambda: dn.forward(rgb, aux, out))
    ms_b = timed(lambda: dn.backward_input(rgb, out))
    ms_t = timed(lambda: dn.train_step(rgb, aux, tgt, 0.0))
    dn.close()
    # a training step runs the forward, the input-gradient and the weight-gradient GEMMs: 3x the forward's FLOPs
    return {"H": H, "W": W, "n": n, "gflop_forward": flops / 1e9, "ms_forward": ms_f, "ms_backward_input": ms_b,
            "ms_train_step": ms_t, "tflops_forward": flops / ms_f / 1e9, "tflops_train_step": 3 * flops / ms_t / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=400)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--spp-in", type=int, default=2)
    ap.add_argument("--spp-target", type=int, default=256)
    ap.add_argument("--spp-ref", type=int, default=1024)
    ap.add_argument("--eval", type=int, default=4, help="held-out scenes")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--first-pair", type=int, default=0, help="index of the first training scene of this run")
    ap.add_argument("--resume", default=None, help="checkpoint (.npz) to continue from")
    ap.add_argument("--save", default=None, help="write the training state (.npz) here")
    ap.add_argument("--total-steps", type=int, default=None, help="length of the cosine schedule across runs")
    ap.add_argument("--bench", action="store_true", help="only time the network's calls: one, 8 and 64 "
                    "images of 256x256 per call, and 64 of 512x512 (the sequence fit's frames)")
    ap.add_argument("--bench-n", type=int, default=0, help="with --bench: only n images of 256x256 per call")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the denoiser needs a HIP device"
    if args.bench:
        if args.bench_n:
            print(json.dumps(bench(n=args.bench_n)), flush=True)
            return
        print(json.dumps(bench()), flush=True)
        for n in (8, 64):          # several images per call: the deep layers fill the chip
            print(json.dumps(bench(n=n, reps=5)), flush=True)
        print(json.dumps(bench(512, 512, reps=3, n=64)), flush=True)
        return
    model, scene, _, _ = synth.workload("paper")
    r = facert.Renderer(model, scene)
    dn = Denoiser(scene.height, scene.width)
    state = None
    if args.resume:
        with np.load(args.resume, allow_pickle=False) as z:
            state = {k: z[k] for k in ("params", "m", "v", "step")}
    steps = args.epochs * args.pairs
    t_data, t_train, curve = (0.0, 0.0, [])
    if args.pairs > 0:
        t_data, t_train, curve = train(r, dn, args.pairs, args.epochs, args.spp_in, args.spp_target, args.lr,
                                       args.seed, first_pair=args.first_pair, state=state,
                                       total_steps=args.total_steps)
    elif state is not None:
        dn.set_state(state)
    if args.save:
        st = dn.get_state()
        np.savez(args.save, **st)

    # held-out evaluation against a 1024-spp reference
    spps = [2, 4, 8, 16, 32, 64, 128, 256]
    res = {"plain": {s: [] for s in spps}, "denoised": []}
    timing = {}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3

    for e in range(args.eval):
        i = 1_000_000 + e
        p = facert.params_to_device(scene_params(i))
        ref = r.render(p, 7, args.spp_ref).cpu().numpy()
        for s in spps:
            res["plain"][s].append(psnr(r.render(p, 99, s).cpu().numpy(), ref))
        rgb = r.render(p, 99, args.spp_in).clone()
        aux = r.aov()
        res["denoised"].append(psnr(dn.forward(rgb, aux).cpu().numpy(), ref))
        if e == 0:
            for s in spps:
                timing[f"render_{s}spp_ms"] = timed(lambda: r.render(p, 99, s))
            timing["denoise_ms"] = timed(lambda: dn.forward(rgb, aux))

            def low_spp_path():
                r.render(p, 99, args.spp_in, out=rgb)
                r.aov(out=aux)
                dn.forward(rgb, aux)
            timing[f"render_{args.spp_in}spp_aov_denoise_ms"] = timed(low_spp_path)
    plain = {s: float(np.mean(v)) for s, v in res["plain"].items()}
    den = float(np.mean(res["denoised"]))
    # the plain sample count whose PSNR the denoised 2-spp image matches (log-linear interpolation)
    equiv = None
    for a, b in zip(spps, spps[1:]):
        if plain[a] <= den <= plain[b]:
            f = (den - plain[a]) / (plain[b] - plain[a])
            equiv = float(2 ** (math.log2(a) + f * (math.log2(b) - math.log2(a))))
    if equiv is None and den > plain[spps[-1]]:
        equiv = f">{spps[-1]}"
    out = {"pairs": args.pairs, "epochs": args.epochs, "spp_in": args.spp_in, "spp_target": args.spp_target,
           "first_pair": args.first_pair, "resumed": bool(args.resume),
           "data_s": t_data, "train_s": t_train, "ms_per_train_step": t_train / max(steps, 1) * 1e3,
           "loss_per_epoch": curve,
           "psnr_db": {"denoised_2spp": den, "plain": plain}, "equal_psnr_plain_spp": equiv, "timing": timing}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
