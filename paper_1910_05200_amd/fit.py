"""Fitting loop: the objective of Eq. 1 without the landmark/statistical
prior, argmin E_data + w2 E_light, over identity alpha, expression beta,
albedo delta, light colours l_j, specular texels c_spec and pose [R t].

Each iteration runs on the device through the C-ABI: fr_render (a fresh
Monte-Carlo seed per iteration), fr_loss_l2 (E_data and its image
gradient), fr_backward (all gradient terms), fr_light_reg (adds w2 E_light's
gradient to the light gradient) and one fr_adam call per parameter group.
The pose goes back to the host once per iteration because fr_render builds
R from it in double precision on the host.

    python -m paper_1910_05200_amd.fit --workload paper --iters 200

prints one JSON line: time per iteration, E_data along the way, PSNR of the
fitted render against the target and the parameter errors before and after.
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

from paper_1910_05200_amd import facert, synth

# initial Adam step sizes, in each group's own units (coefficients, light
# intensity, texel value, radians, metres); they decay by DECAY over the run.
# Adam turns Monte-Carlo gradient noise into a random walk of about
# lr * sqrt(iterations) on parameters the image barely constrains (the
# specular texels), hence their small step.
LR = {"alpha": 0.03, "beta": 0.03, "delta": 0.02, "lights": 0.01, "spec": 0.004, "rot": 1e-3, "trans": 2.5e-4}
DECAY = 0.1
W2 = 1e-3          # weight of E_light
START_SEED = 3     # seed of the perturbation that gives the fitting start


def finite_groups(named, counts: dict) -> dict:
    """{name: every component finite} for (name, tensor) pairs, read back
    with one synchronisation; a non-finite group's count goes up (a fitting
    loop then leaves that group unchanged for the iteration: one non-finite
    component would make Adam's moments, and so the parameters, non-finite
    for good)."""
    import torch
    flags = torch.stack([torch.isfinite(t).all() for _, t in named]).cpu().tolist()
    out = {}
    for (name, _), ok in zip(named, flags):
        out[name] = bool(ok)
        if not ok:
            counts[name] = counts.get(name, 0) + 1
    return out


def psnr(img, ref) -> float:
    """Peak signal-to-noise ratio in dB, peak = max of the reference."""
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    mse = float(np.mean((img - ref) ** 2))
    peak = float(ref.max())
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def param_errors(p: dict, truth: synth.Params) -> dict:
    """RMS error per parameter group against the target parameters."""
    out = {}
    for k in ("alpha", "beta", "delta", "lights", "spec"):
        a = p[k].detach().cpu().numpy() if hasattr(p[k], "detach") else np.asarray(p[k])
        out[k] = float(np.sqrt(np.mean((a - getattr(truth, k)) ** 2)))
    pose = np.asarray(p["pose"], np.float64)
    out["rot_deg"] = float(np.degrees(np.sqrt(np.mean((pose[:3] - truth.pose[:3]) ** 2))))
    out["trans_mm"] = float(1e3 * np.sqrt(np.mean((pose[3:] - truth.pose[3:]) ** 2)))
    return out


def fit(r: facert.Renderer, target, start: synth.Params, iters: int, spp: int, w2: float = W2,
        lr: dict = None, decay: float = DECAY, seed0: int = 1000, log_every: int = 0):
    """Run the loop from `start`; returns (params dict, per-iteration E_data
    list, seconds per iteration)."""
    import torch
    lr = dict(LR if lr is None else lr)
    p = facert.params_to_device(start)
    pose_d = torch.from_numpy(np.asarray(start.pose, np.float32).copy()).cuda()
    groups = ("alpha", "beta", "delta", "lights", "spec")
    state = {k: (torch.zeros_like(p[k]), torch.zeros_like(p[k])) for k in groups}
    state["pose"] = (torch.zeros_like(pose_d), torch.zeros_like(pose_d))
    losses = []
    nonfinite = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        p["pose"] = pose_d.cpu().numpy()
        img = r.render(p, seed0 + it, spp)
        dL, loss = r.loss_l2(img, target)
        g = r.backward(dL, want=("d_alpha", "d_beta", "d_delta", "d_lights", "d_spec", "d_pose"))
        r.light_reg(p["lights"], w2, g["d_lights"])
        f = decay ** (it / max(1, iters - 1))
        step = it + 1
        ok = finite_groups([(k, g["d_" + k]) for k in groups + ("pose",)], nonfinite)
        for k in groups:
            m, v = state[k]
            if ok[k]:
                r.adam(p[k], g["d_" + k].reshape(p[k].shape), m, v, step, lr[k] * f)
        m, v = state["pose"]
        if ok["pose"]:
            r.adam(pose_d[:3], g["d_pose"][:3], m[:3], v[:3], step, lr["rot"] * f)
            r.adam(pose_d[3:], g["d_pose"][3:], m[3:], v[3:], step, lr["trans"] * f)
        losses.append(loss)
        if log_every and (it % log_every == 0 or it == iters - 1):
            print(f"it {it:4d}  E_data {float(loss):.6g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(1, iters)
    p["pose"] = pose_d.cpu().numpy()
    if nonfinite:
        print(f"updates skipped for non-finite gradients: {nonfinite}", file=sys.stderr, flush=True)
    return p, [float(x) for x in losses], sec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny"])
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--spp", type=int, default=0, help="samples per pixel while fitting (default: the workload's)")
    ap.add_argument("--eval-spp", type=int, default=synth.TARGET_SPP)
    ap.add_argument("--log-every", type=int, default=20)
    ap.add_argument("--lr", action="append", default=[], metavar="GROUP=VALUE",
                    help=f"override an initial step size (groups: {', '.join(LR)})")
    ap.add_argument("--decay", type=float, default=DECAY)
    args = ap.parse_args()
    lr = dict(LR)
    for kv in args.lr:
        k, v = kv.split("=")
        if k not in lr:
            ap.error(f"unknown group {k}")
        lr[k] = float(v)
    import torch
    assert torch.cuda.is_available(), "the fitting loop needs a HIP device"
    model, scene, _, spp = synth.workload(args.workload)
    spp = args.spp or spp
    truth = synth.make_params(synth.TARGET_SCENE_SEED)
    start = synth.perturb(truth, START_SEED)
    r = facert.Renderer(model, scene)
    target = r.render(facert.params_to_device(truth), synth.TARGET_RENDER_SEED, synth.TARGET_SPP).clone()
    tgt = target.cpu().numpy()
    p0 = facert.params_to_device(start)
    psnr0 = psnr(r.render(p0, 99, args.eval_spp).cpu().numpy(), tgt)
    err0 = param_errors(p0, truth)
    p, losses, sec = fit(r, target, start, args.iters, spp, lr=lr, decay=args.decay, log_every=args.log_every)
    psnr1 = psnr(r.render(p, 99, args.eval_spp).cpu().numpy(), tgt)
    err1 = param_errors(p, truth)
    # reference point: the target parameters themselves, rendered with another seed
    psnr_truth = psnr(r.render(facert.params_to_device(truth), 99, args.eval_spp).cpu().numpy(), tgt)
    out = {"workload": args.workload, "iters": args.iters, "spp": spp, "ms_per_iter": sec * 1e3,
           "E_data_first": losses[0], "E_data_last": float(np.mean(losses[-10:])),
           "psnr_db": {"start": psnr0, "fitted": psnr1, "target_params": psnr_truth, "eval_spp": args.eval_spp},
           "param_rms_error": {"start": err0, "fitted": err1}, "w2": W2, "lr": lr, "decay": args.decay}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
