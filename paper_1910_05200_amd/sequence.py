"""Sequence fitting: several frames of one face share identity alpha, albedo
delta, the light colours and the specular texels; each frame has its own
expression beta and pose (a random walk over the sequence in the synthetic
truth).  The objective is Eq. 1 without E_prior summed over frames; Adam on
the shared groups with the frames' gradients summed, and on each frame's
own groups.

Three ways to get each frame's data-term gradient:
  plain        render at N spp, E_data against the target, fr_backward;
  denoised     render at 2 spp, its auxiliary buffers (fr_aov), the
               denoiser, E_data on the denoised image, the gradient through
               the denoiser to the 2-spp render (fd_backward_input),
               fr_backward;
  denoised-st  as denoised, but the image gradient of E_data on the
               denoised image goes to the 2-spp render's adjoint as it is
               (the denoiser treated as the identity in the backward pass).
The denoiser is trained first on renderer-generated pairs (denoise.py).

With one renderer per frame (``frame_renderers``), an iteration renders
all frames in one batched call and differentiates them in another
(fr_batch_*, the same results as one frame after another); a frame count
and spp whose frames exceed one chunk of samples each run frame by frame.

    python -m paper_1910_05200_amd.sequence --frames 8 --iters 150 --modes plain:256,plain:16,denoised:2

prints one JSON line per mode: seconds per iteration, parameter errors and
the frames' mean PSNR (256 spp evaluation) against their targets, logged
along the run, so that the modes can be compared at equal error.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1910_05200_amd import denoise, facert, fit, synth

SHARED = ("alpha", "delta", "lights", "spec")
LR = dict(fit.LR)


def make_truth(n_frames: int, seed: int = synth.TARGET_SCENE_SEED):
    """Shared parameters of one face, and per-frame (beta, pose) on a random walk."""
    base = synth.make_params(seed)
    rng = np.random.default_rng(4242 + seed)
    d2r = math.pi / 180.0
    frames, beta, pose = [], base.beta.astype(np.float64), base.pose.astype(np.float64)
    for _ in range(n_frames):
        frames.append((beta.astype(np.float32), pose.astype(np.float32)))
        beta = beta + rng.normal(0, 0.15, beta.shape)
        pose = pose + np.concatenate([rng.normal(0, 1.0, 3) * d2r, rng.normal(0, 0.001, 3)])
    return base, frames


def make_start(base: synth.Params, frames, seed: int = fit.START_SEED):
    """Perturbed shared parameters and per-frame (beta, pose), as synth.perturb."""
    start = synth.perturb(base, seed)
    out = []
    for f, (beta, pose) in enumerate(frames):
        q = base.copy()
        q.beta, q.pose = beta.copy(), pose.copy()
        q = synth.perturb(q, 1000 + 17 * seed + f)
        out.append((q.beta, q.pose))
    return start, out


def frame_params(shared: dict, beta, pose) -> dict:
    d = dict(shared)
    d["beta"] = beta
    d["pose"] = pose
    return d


def errors(shared: dict, betas, poses, base: synth.Params, frames) -> dict:
    e = {}
    for k in SHARED:
        a = shared[k].detach().cpu().numpy() if hasattr(shared[k], "detach") else np.asarray(shared[k])
        e[k] = float(np.sqrt(np.mean((a - getattr(base, k)) ** 2)))
    b = np.concatenate([np.asarray(x.cpu().numpy() if hasattr(x, "cpu") else x) - t[0] for x, t in zip(betas, frames)])
    e["beta"] = float(np.sqrt(np.mean(b ** 2)))
    P = np.array([np.asarray(p.cpu().numpy() if hasattr(p, "cpu") else p, np.float64) for p in poses])
    T = np.array([t[1] for t in frames], np.float64)
    e["rot_deg"] = float(np.degrees(np.sqrt(np.mean((P[:, :3] - T[:, :3]) ** 2))))
    e["trans_mm"] = float(1e3 * np.sqrt(np.mean((P[:, 3:] - T[:, 3:]) ** 2)))
    return e


def frame_renderers(model, scene, n: int):
    """One renderer (context) per frame, for batched iterations."""
    return [facert.Renderer(model, scene) for _ in range(n)]


def _state_out(shared, betas, poses, st, stf, it, elapsed, log, nonfinite) -> dict:
    """Host copy of a run's state, for a checkpoint (see run)."""
    h = lambda t: t.detach().cpu().numpy()
    d = {"iter": np.int64(it), "elapsed": np.float64(elapsed),
         "log": np.frombuffer(json.dumps({"log": log, "nonfinite": nonfinite}).encode(), np.uint8)}
    for k in SHARED:
        d[f"p_{k}"], d[f"m_{k}"], d[f"v_{k}"] = h(shared[k]), h(st[k][0]), h(st[k][1])
    d["betas"] = np.stack([h(b) for b in betas])
    d["poses"] = np.stack([h(q) for q in poses])
    d["mb"] = np.stack([h(x[0][0]) for x in stf]); d["vb"] = np.stack([h(x[0][1]) for x in stf])
    d["mp"] = np.stack([h(x[1][0]) for x in stf]); d["vp"] = np.stack([h(x[1][1]) for x in stf])
    return d


def run(r: facert.Renderer, targets, base, frames, start, start_frames, iters: int, mode: str, spp: int,
        dn: denoise.Denoiser = None, eval_spp: int = synth.TARGET_SPP, log_every: int = 25, decay: float = fit.DECAY,
        rs=None, seed: int = 0, state: dict | None = None, stop_after_s: float | None = None):
    """Fit for iterations [state's iteration or 0, iters) (the step-size
    schedule spans all iters).  seed offsets the render seeds.  state
    resumes a checkpoint written by an earlier call (the "state" entry of the
    result, present when the run stopped early at stop_after_s seconds of
    fitting)."""
    import torch
    shared = facert.params_to_device(start)
    shared.pop("beta"), shared.pop("pose")
    betas = [torch.from_numpy(b.copy()).cuda() for b, _ in start_frames]
    poses = [torch.from_numpy(np.asarray(p, np.float32).copy()).cuda() for _, p in start_frames]
    st = {k: (torch.zeros_like(shared[k]), torch.zeros_like(shared[k])) for k in SHARED}
    stf = [((torch.zeros_like(b), torch.zeros_like(b)), (torch.zeros(6, device="cuda"), torch.zeros(6, device="cuda")))
           for b in betas]
    want = ("d_alpha", "d_beta", "d_delta", "d_lights", "d_spec", "d_pose")
    n = len(targets)
    log, elapsed = [], 0.0
    nonfinite = {}                       # parameter group -> skipped updates
    it0 = 0
    if state is not None:
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        for k in SHARED:
            shared[k].copy_(dev(state[f"p_{k}"]).reshape(shared[k].shape))
            st[k][0].copy_(dev(state[f"m_{k}"]).reshape(shared[k].shape))
            st[k][1].copy_(dev(state[f"v_{k}"]).reshape(shared[k].shape))
        for f in range(n):
            betas[f].copy_(dev(state["betas"][f])); poses[f].copy_(dev(state["poses"][f]))
            stf[f][0][0].copy_(dev(state["mb"][f])); stf[f][0][1].copy_(dev(state["vb"][f]))
            stf[f][1][0].copy_(dev(state["mp"][f])); stf[f][1][1].copy_(dev(state["vp"][f]))
        it0, elapsed = int(state["iter"]), float(state["elapsed"])
        meta = json.loads(bytes(state["log"]).decode())
        log, nonfinite = meta["log"], meta["nonfinite"]
    batch = None
    if rs is not None and len(rs) == n and r.W * r.H * spp <= facert.FR_CHUNK_MAX:
        batch = facert.Batch(rs)

    def evaluate(it):
        psnrs = []
        for f in range(n):
            img = r.render(frame_params(shared, betas[f], poses[f].cpu().numpy()), 99, eval_spp)
            psnrs.append(fit.psnr(img.cpu().numpy(), targets[f].cpu().numpy()))
        e = errors(shared, betas, poses, base, frames)
        log.append({"iter": it, "seconds": elapsed, "psnr_db": float(np.mean(psnrs)), "errors": e})
        print(f"{mode}:{spp} iteration {it}: {elapsed:.2f} s, {log[-1]['psnr_db']:.2f} dB", file=sys.stderr, flush=True)

    if it0 == 0:
        evaluate(0)
    stopped = None
    for it in range(it0, iters):
        if stop_after_s is not None and elapsed - (float(state["elapsed"]) if state is not None else 0.0) > stop_after_s:
            stopped = it
            break
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = {k: torch.zeros_like(shared[k]) for k in SHARED}
        f_lr = decay ** (it / max(1, iters - 1))
        pose_h = torch.stack(poses).cpu().numpy()
        ps = [frame_params(shared, betas[f], pose_h[f]) for f in range(n)]
        seeds = [1000 + 10_000_000 * seed + it * n + f for f in range(n)]

        def data_grad(rf, img, f):
            if mode in ("denoised", "denoised-st"):
                den = dn.forward(img, rf.aov())
                dL, _ = rf.loss_l2(den, targets[f])
                return dn.backward_input(img, dL) if mode == "denoised" else dL
            return rf.loss_l2(img, targets[f])[0]

        def data_grads_stacked(imgs):
            # a denoiser made for all n frames: one forward and one input
            # gradient for the stack instead of n of each
            rgb = torch.stack(imgs)
            aux = torch.empty((n, r.H, r.W, denoise.facert_aux_channels()), device="cuda", dtype=torch.float32)
            for f in range(n):
                rs[f].aov(out=aux[f])
            den = dn.forward(rgb, aux)
            dL = torch.stack([rs[f].loss_l2(den[f], targets[f])[0] for f in range(n)])
            if mode == "denoised":
                dL = dn.backward_input(rgb, dL)
            return [dL[f] for f in range(n)]

        if batch is not None:
            imgs = batch.render(ps, seeds, [spp] * n)
            if mode in ("denoised", "denoised-st") and dn.n == n > 1:
                dls = data_grads_stacked(imgs)
            else:
                dls = [data_grad(rs[f], imgs[f], f) for f in range(n)]
            gs = batch.backward(dls, want=want)
        else:
            gs = []
            for f in range(n):
                img = r.render(ps[f], seeds[f], spp)
                gs.append(r.backward(data_grad(r, img, f), want=want))
        for f in range(n):
            for k in SHARED:
                acc[k] += gs[f]["d_" + k].reshape(acc[k].shape)
        r.light_reg(shared["lights"], fit.W2, acc["lights"])
        named = [(k, acc[k]) for k in SHARED]
        for f in range(n):
            named += [(f"beta{f}", gs[f]["d_beta"]), (f"pose{f}", gs[f]["d_pose"])]
        ok = fit.finite_groups(named, nonfinite)
        for f in range(n):
            g = gs[f]
            (mb, vb), (mp, vp) = stf[f]
            if ok[f"beta{f}"]:
                r.adam(betas[f], g["d_beta"], mb, vb, it + 1, LR["beta"] * f_lr)
            if ok[f"pose{f}"]:
                r.adam(poses[f][:3], g["d_pose"][:3], mp[:3], vp[:3], it + 1, LR["rot"] * f_lr)
                r.adam(poses[f][3:], g["d_pose"][3:], mp[3:], vp[3:], it + 1, LR["trans"] * f_lr)
        for k in SHARED:
            m, v = st[k]
            if ok[k]:
                r.adam(shared[k], acc[k], m, v, it + 1, LR[k] * f_lr)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        if (it + 1) % log_every == 0 or it == iters - 1:
            evaluate(it + 1)
    if batch is not None:
        batch.close()
    done = stopped if stopped is not None else iters
    out = {"mode": mode, "spp": spp, "frames": n, "iters": iters, "iters_done": done, "seed": seed,
           "s_per_iter": elapsed / max(1, done), "batched": batch is not None,
           "nonfinite_updates_skipped": nonfinite, "log": log}
    if stopped is not None:
        out["state"] = _state_out(shared, betas, poses, st, stf, stopped, elapsed, log, nonfinite)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--iters", type=int, default=150)
    ap.add_argument("--modes", default="plain:256,plain:16,plain:2,denoised:2")
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny", "sequence512"])
    ap.add_argument("--dn-workload", default=None, choices=["paper", "tiny", "sequence512"],
                    help="train the denoiser on this workload's scenes (default: --workload); the network is "
                         "convolutional, so its parameters then serve the fit's image size")
    ap.add_argument("--dn-pairs", type=int, default=2000)
    ap.add_argument("--dn-epochs", type=int, default=10)
    ap.add_argument("--log-every", type=int, default=25)
    ap.add_argument("--sequential", action="store_true", help="render and differentiate frame by frame")
    ap.add_argument("--seed", type=int, default=0, help="start perturbation and render seeds of the run")
    ap.add_argument("--dn-ckpt", default=None, help="denoiser checkpoint (.npz from denoise.py --save) to use "
                                                    "instead of training one")
    ap.add_argument("--resume", default=None, help="continue the (single) mode from this checkpoint (.npz)")
    ap.add_argument("--save-state", default=None, help="where to write the checkpoint if the run stops early")
    ap.add_argument("--stop-after", type=float, default=None, help="stop after this many seconds of fitting")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "sequence fitting needs a HIP device"
    model, scene, _, _ = synth.workload(args.workload)
    r = facert.Renderer(model, scene)
    rs = None if args.sequential else frame_renderers(model, scene, args.frames)
    base, frames = make_truth(args.frames)
    start, start_frames = make_start(base, frames, seed=fit.START_SEED + args.seed)
    targets = [r.render(facert.params_to_device(frame_params_np(base, b, p)), synth.TARGET_RENDER_SEED + f,
                        synth.TARGET_SPP).clone() for f, (b, p) in enumerate(frames)]
    dn = None
    modes = [(m.split(":")[0], int(m.split(":")[1])) for m in args.modes.split(",")]
    # with batched frames, one network runs all of them per call
    dn_n = args.frames if rs is not None and args.frames > 1 and scene.height % 64 == 0 else 1
    if any(m.startswith("denoised") for m, _ in modes) and args.dn_ckpt:
        dn = denoise.Denoiser(scene.height, scene.width, n=dn_n)
        with np.load(args.dn_ckpt, allow_pickle=False) as z:
            dn.set_params(torch.from_numpy(np.ascontiguousarray(z["params"], np.float32)).cuda())
        print(json.dumps({"denoiser": args.dn_ckpt}), flush=True)
    elif any(m.startswith("denoised") for m, _ in modes):
        t0 = time.perf_counter()
        dn = denoise.Denoiser(scene.height, scene.width, n=dn_n)
        dw = args.dn_workload or args.workload
        if dw == args.workload:
            dn1 = denoise.Denoiser(scene.height, scene.width) if dn_n > 1 else dn
            denoise.train(r, dn1, args.dn_pairs, args.dn_epochs, spp_in=2, spp_target=synth.TARGET_SPP)
            if dn1 is not dn:
                dn.set_params(dn1.get_params())
                dn1.close()
        else:
            m2, s2, _, _ = synth.workload(dw)
            r2 = facert.Renderer(m2, s2)
            dn2 = denoise.Denoiser(s2.height, s2.width)
            denoise.train(r2, dn2, args.dn_pairs, args.dn_epochs, spp_in=2, spp_target=synth.TARGET_SPP)
            dn.set_params(dn2.get_params())
            dn2.close()
            r2.close()
        torch.cuda.synchronize()
        print(json.dumps({"denoiser_training_s": time.perf_counter() - t0, "pairs": args.dn_pairs,
                          "epochs": args.dn_epochs, "trained_on": dw}), flush=True)
    state = None
    if args.resume:
        assert len(modes) == 1, "--resume continues one mode"
        with np.load(args.resume, allow_pickle=False) as z:
            state = {k: z[k] for k in z.files}
    for m, spp in modes:
        out = run(r, targets, base, frames, start, start_frames, args.iters, m, spp, dn, log_every=args.log_every,
                  rs=rs, seed=args.seed, state=state, stop_after_s=args.stop_after)
        st = out.pop("state", None)
        if st is not None and args.save_state:
            np.savez(args.save_state, **st)
            out["saved_state"] = args.save_state
        print(json.dumps(out), flush=True)


def frame_params_np(base: synth.Params, beta, pose) -> synth.Params:
    q = base.copy()
    q.beta, q.pose = beta, pose
    return q


if __name__ == "__main__":
    main()
