"""Benchmark: one forward + adjoint iteration of the light-stage face render.

A step is the whole hot path on one batch: morphable blend, BVH refit, edge
tables, Monte-Carlo render (256x256, 16 spp, 20 lights), squared-L2 loss and
its image gradient, adjoint with both edge-sampling terms, normal chain and
the transposed blend/pose reductions to alpha, beta, delta and pose.  Inputs
are resident on the device before timing starts.

Prints one JSON line (see the fields below).  --gpus above 1 is refused: the
build targets one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/iter & Mrays/s at 256x256; denoised-2spp vs plain-256spp at equal PSNR"

# Algorithmic VALU work per unit, in fp32 lane operations, at fixed costs
# that do not depend on how the kernels compile: a box (slab) test 15 (six
# fused subtract-multiply slab times, six min/max, the entry/exit compare),
# a Moller-Trumbore triangle test 50 (two cross products, three dot
# products, the reciprocal, the bound tests).  These price the roofline.
OPS_BOX = 15
OPS_TRI = 50
# The same units as the compiled gfx950 code issues them (VALU instructions
# per lane in the compiled loop, address arithmetic included): a node visit
# of the any-hit walk 23 (three byte permutations pick the near and far
# bounds, the binary16 decode is folded into v_fma_mix_f32; the loop's exit
# and queue tests included), a full triangle test with its hit-box check 95, one light
# sample's shading 215, one light sample's shading plus reverse-mode
# adjoint 590.  Reported beside the fixed-cost fraction, never in its place.
ISA_BOX = 23
ISA_TRI = 95
OPS_SHADE_FWD = 215
OPS_SHADE_ADJ = 590
# fp32 VALU issue ceiling: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz, one
# non-packed, non-fused operation per lane per clock
PEAK_VALU = 39.3      # T lane-ops/s
VALU_UNIT = "Tlane-ops/s"
# the renderer's kernel sources (a traffic figure is valid while they hash as when it was taken)
KERNEL_SOURCES = ("facert.hip", "fr_device.hpp", "fr_lbvh.hpp", "fr_batch.hpp")


def _profile_fields(name: str, workload: str):
    """key: value lines of a committed rocprofv3 summary, or None when the
    kernel sources changed since its counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"fwd_bwd_{workload}_{name}.md")
    if not os.path.exists(path):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_1910_05200_amd", "csrc", f), "rb").read()
                   for f in KERNEL_SOURCES)
    fields = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l and not l.startswith("|"))
    if fields.get("kernel_source_sha256", "").strip() != hashlib.sha256(src).hexdigest():
        return None
    return fields


def profiled_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE, calibrated), or None when it is stale."""
    f = _profile_fields("traffic", workload)
    v = f.get(f"{kernel}_traffic_bytes_per_launch") if f else None
    return float(v) if v else None


def profiled_valu(kernel: str, workload: str):
    """VALU counters per launch from the committed PMC summary: wave-level
    VALU instructions (SQ_INSTS_VALU) and active lanes per VALU instruction
    (SQ_THREAD_CYCLES_VALU / SQ_ACTIVE_INST_VALU), or None when stale."""
    f = _profile_fields("valu", workload)
    if not f or not f.get(f"{kernel}_sq_insts_valu"):
        return None
    return {"sq_insts_valu": float(f[f"{kernel}_sq_insts_valu"]),
            "active_lanes_per_valu_inst": float(f[f"{kernel}_active_lanes_per_valu_inst"])}


def host_cpu() -> dict:
    """The host's logical CPU count, the cores this process may use, and the CPU model."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


def oracle_threads(requested: int = 0) -> int:
    """All the cores this process may use, up to 16 (the CPU share of one GPU
    on the GPU machines; there nproc and the affinity are both 16)."""
    return requested or max(1, min(16, host_cpu()["usable"]))


def roofline_entry(kernel: str, box: float, tri: float, shade: float, shade_cost: int, sec: float, workload: str):
    """The roofline object of one kernel's launch: work at the fixed unit
    costs over its measured time against the VALU ceiling, the same work at
    the compiled code's instruction costs, and the VALU counters of the committed
    profile (issue rate of wave-level VALU instructions, as lane slots, and
    the active lanes per instruction)."""
    ops = box * OPS_BOX + tri * OPS_TRI + shade * shade_cost
    ops_isa = box * ISA_BOX + tri * ISA_TRI + shade * shade_cost
    achieved = ops / sec / 1e12
    out = {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": PEAK_VALU, "unit": VALU_UNIT,
           "frac": achieved / PEAK_VALU, "traffic": profiled_traffic(kernel, workload),
           "ops_per_launch": ops, "ms_per_launch": sec * 1e3,
           "unit_costs": {"box": OPS_BOX, "tri": OPS_TRI, "shade": shade_cost},
           "frac_at_isa_costs": ops_isa / sec / 1e12 / PEAK_VALU,
           "isa_costs": {"box": ISA_BOX, "tri": ISA_TRI, "shade": shade_cost}}
    v = profiled_valu(kernel, workload)
    if v:
        out["counters"] = {"valu_lane_slots_per_launch": v["sq_insts_valu"] * 64,
                           "valu_issue_frac": v["sq_insts_valu"] * 64 / sec / 1e12 / PEAK_VALU,
                           "active_lanes_per_valu_inst": v["active_lanes_per_valu_inst"],
                           "active_lane_ops_per_launch": v["sq_insts_valu"] * v["active_lanes_per_valu_inst"]}
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny", "batch"],
                    help="paper / tiny: one face per step; batch: 32 faces of 5k-40k vertices at 128^2-512^2 and "
                         "4-16 spp per step, one launch per kernel for all of them")
    ap.add_argument("--bvh", default="lbvh", choices=["lbvh", "refit"],
                    help="lbvh: Morton-code tree rebuilt from the posed mesh every step; refit: tree shape built "
                         "once over the mean shape, boxes refitted every step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu-single", action="store_true", help="skip the one-thread oracle timing")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (scale for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(model, scene, params, target, seed, spp, threads):
    """The CPU oracle on one full iteration of the same workload."""
    import oracle
    oracle.build(force=not os.path.exists(oracle.LIB_PATH))
    osc, vm, R = oracle.scene_from_model(model, scene, params)
    t0 = time.perf_counter()
    img, c1 = oracle.render(osc, seed, spp, threads=threads, counts=True)
    dL = 2.0 * (img - target)
    g, c2 = oracle.backward(osc, seed, spp, dL, flags=7, threads=threads, counts=True)
    oracle.parameter_grads(model, params, vm, R, g["d_pos"], g["d_alb"])
    dt = time.perf_counter() - t0
    rays = c1.total() + c2.total()
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "ms_per_iter": dt * 1e3, "host": host_cpu(),
            "sample": "one full forward+adjoint iteration (all terms) of the same paper-scale workload, "
                      "same seed and spp"}


def _rays(st) -> int:
    return st["rays_camera"] + st["rays_shadow"] + st["rays_edge_primary"] + st["rays_edge_secondary"]


def bench_batch(args):
    """Many faces per step (fr_batch_*): render, per-face loss, adjoint.
    Timed four ways: eager batched calls; a HIP graph captured per step (the
    reported value); replay of one captured step; the single-context calls
    one face after another (the same work without batching)."""
    import ctypes as C
    import torch
    from paper_1910_05200_amd import facert, synth
    lib = facert.load()
    if args.calibrate_copy:
        src = torch.ones(64 << 20, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    inst = synth.batch_workload()
    n = len(inst)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rs = [facert.Renderer(m, sc) for m, sc, _, _ in inst]
        ps = [facert.params_to_device(p) for _, _, p, _ in inst]
        spps = [spp for *_, spp in inst]
        batch = facert.Batch(rs, timing=True)
        tg = [facert.params_to_device(synth.make_params(900 + i)) for i in range(n)]
        tgts = [t.clone() for t in batch.render(tg, [77 + i for i in range(n)], spps)]
        imgs = [torch.empty_like(t) for t in tgts]
        dls = [torch.empty_like(t) for t in tgts]
        losses = [torch.empty((), device="cuda") for _ in range(n)]
        grads = [{k: torch.empty(v, device="cuda") for k, v in
                  {"d_lights": (r.n_lights, 3), "d_spec": (r.spec_res ** 2,), "d_vertices": (3, r.V),
                   "d_albedo": (3, r.V), "d_alpha": (r.n_id,), "d_beta": (r.n_exp,), "d_delta": (r.n_alb,),
                   "d_pose": (6,)}.items()} for r in rs]

        def step(it):
            batch.render(ps, [1000 + 97 * it + i for i in range(n)], spps, outs=imgs)
            for r, im, t, d, l in zip(rs, imgs, tgts, dls, losses):
                facert._check(r.ctx, lib.fr_loss_l2(r.ctx, im.data_ptr(), t.data_ptr(), d.data_ptr(), l.data_ptr()))
            batch.backward(dls, outs=grads)

        for it in range(args.warmup):
            step(it)
        tuned = batch.tune(trials=2)
        step(0)
        tm = batch.timing()
        rays = sum(_rays(r.stats()) for r in rs)
        stats = [r.stats() for r in rs]

        def timed(fn, k):
            stream.synchronize()
            t0 = time.perf_counter()
            for it in range(k):
                fn(it)
            stream.synchronize()
            return (time.perf_counter() - t0) / k * 1e3

        ms_eager = timed(lambda it: step(args.warmup + it), args.steps)

        def graph_step(it):
            batch.capture_begin()
            step(args.warmup + args.steps + it)
            batch.capture_end()
            batch.graph_launch()

        graph_step(0)
        ms_graph = timed(graph_step, args.steps)
        ms_replay = timed(lambda it: batch.graph_launch(), args.steps)

        def sequential(it):
            for i, r in enumerate(rs):
                img = r.render(ps[i], 5000 + 97 * it + i, spps[i], out=imgs[i])
                facert._check(r.ctx, lib.fr_loss_l2(r.ctx, img.data_ptr(), tgts[i].data_ptr(), dls[i].data_ptr(),
                                                    losses[i].data_ptr()))
                r.backward(dls[i])

        sequential(0)
        ms_seq = timed(sequential, max(2, args.steps // 4))
    k_sh = facert.KERNELS.index("k_sh_trace")
    box_sh = sum(st["kernel_box_tests"][k_sh] for st in stats)
    tri_sh = sum(st["kernel_tri_tests"][k_sh] for st in stats)
    ms_sh = tm["sh_trace"]
    V = [m.n_vertices for m, *_ in inst]
    out = {
        "metric": METRIC,
        "value": rays / (ms_graph * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch: {n} faces per step ({min(V)}-{max(V)} vertices, images "
                               f"{min(sc.width for _, sc, _, _ in inst)}^2-{max(sc.width for _, sc, _, _ in inst)}^2, "
                               f"{min(spps)}-{max(spps)} spp, 20 area lights each), render + per-face loss + "
                               "adjoint (all terms), HIP graph captured per step",
                   "samples_per_step": int(sum(sc.width * sc.height * spp for _, sc, _, spp in inst)),
                   "rays_per_step": rays,
                   "ms_eager": round(ms_eager, 3), "ms_graph_per_step_capture": round(ms_graph, 3),
                   "ms_graph_replay": round(ms_replay, 3), "ms_sequential_single_context": round(ms_seq, 3),
                   "batching_speedup_vs_sequential": round(ms_seq / ms_graph, 3),
                   "ms_render": round(tm["render"], 3), "ms_backward": round(tm["backward"], 3),
                   "ms_kinds": {k: round(v, 3) for k, v in tm.items() if v > 0.05 and k not in ("render", "backward")},
                   "tuned": {k: {"mode": ["flat", "xcd"][v[0][0]], "tile": v[0][1], "ms": round(v[1], 3)}
                             for k, v in tuned.items()}},
        "roofline": roofline_entry("k_multi_KShTrace", box_sh, tri_sh, 0, 0, ms_sh * 1e-3, "batch"),
    }
    out["roofline"]["kernel"] = "sh_trace (batched, k_multi_KShTrace)"
    if not args.no_cpu_baseline:
        threads = oracle_threads(args.cpu_threads)
        i = min(range(n), key=lambda k: inst[k][1].width * inst[k][1].height * inst[k][3])
        m, sc, p, spp = inst[i]
        cb = cpu_baseline(m, sc, p, np.zeros((sc.height, sc.width, 3)), 1000, spp, threads)
        cb["sample"] = (f"one full forward+adjoint iteration (all terms) of the batch's smallest face "
                        f"({m.n_vertices} vertices, {sc.width}x{sc.height}, {spp} spp), same seed and spp")
        out["cpu_baseline"] = cb
    batch.close()
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path would shard by image "
              "rows with one gradient all-reduce; the library implements one GPU's share)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    import torch
    from paper_1910_05200_amd import facert, synth

    assert torch.cuda.is_available(), "bench needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    model, scene, params, spp = synth.workload(args.workload)
    r = facert.Renderer(model, scene, timing=True, refit=args.bvh == "refit")
    p = facert.params_to_device(params)
    pt = facert.params_to_device(synth.make_params(synth.TARGET_SCENE_SEED))
    target = r.render(pt, synth.TARGET_RENDER_SEED, synth.TARGET_SPP).clone()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    want = ("d_lights", "d_spec", "d_vertices", "d_albedo", "d_alpha", "d_beta", "d_delta", "d_pose")

    def step(it, ctx=r):
        img = ctx.render(p, 1000 + it, spp)
        dL, loss = ctx.loss_l2(img, target)
        return ctx.backward(dL, want=want), loss

    for it in range(args.warmup):
        step(it)
    torch.cuda.synchronize()
    # per-step kernel timings and work counters (fr_stats synchronises, so
    # this loop is not the timed one)
    per_step = []
    for it in range(args.steps):
        step(args.warmup + it)
        per_step.append(r.stats())
    # the timed bracket: K steps back to back, on a second context of the
    # same face without the per-kernel timing events (their event records,
    # about 0.08 ms per step, are instrumentation, not work).  The first
    # context goes first: each context runs three streams, and the GPU's
    # four hardware queues must not be shared between streams that overlap.
    r.close()
    r_run = facert.Renderer(model, scene, refit=args.bvh == "refit")
    for it in range(args.warmup):
        step(it, r_run)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for it in range(args.steps):
        step(args.warmup + args.steps + it, r_run)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    rays = [st["rays_camera"] + st["rays_shadow"] + st["rays_edge_primary"] + st["rays_edge_secondary"]
            for st in per_step]
    rays_per_iter = float(np.mean(rays))
    kern = {}
    for k, name in enumerate(facert.KERNELS):
        mean = lambda key: float(np.mean([st[key][k] for st in per_step]))
        kern[name] = (mean("kernel_box_tests"), mean("kernel_tri_tests"), mean("kernel_shades"),
                      mean("ms_kernel") * 1e-3, OPS_SHADE_ADJ if name == "k_render_adj" else OPS_SHADE_FWD)
    # The roofline kernel is the shadow-ray trace: the largest single kernel
    # by GPU time, and one that runs alone on the chip, so that its event
    # time is its own.  (The adjoint's kernels share the chip across three
    # streams, and the silhouette entry times a phase of several kernels.)
    dom = "k_sh_trace"
    last = per_step[-1]
    out = {
        "metric": METRIC,
        "value": rays_per_iter / (ms * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {model.n_vertices}-vertex / {model.n_faces}-triangle "
                               f"morphable face, {scene.width}x{scene.height}, {spp} spp, 20 area lights, "
                               "forward + adjoint (interior, camera-silhouette and shadow-boundary terms)",
                   "bvh": args.bvh,
                   "ms_bvh": round(float(np.mean([st["ms_bvh"] for st in per_step])), 4),
                   "rays_per_iter": rays_per_iter,
                   "traversal_overflow": int(last["traversal_overflow"]),
                   "ms_kernels": {n: round(kern[n][3] * 1e3, 3) for n in facert.KERNELS},
                   "box_tests_per_ray": {n: round(last["kernel_box_tests"][k] / max(1, last["kernel_rays"][k]), 2)
                                         for k, n in enumerate(facert.KERNELS)},
                   "tri_tests_per_ray": {n: round(last["kernel_tri_tests"][k] / max(1, last["kernel_rays"][k]), 2)
                                         for k, n in enumerate(facert.KERNELS)}},
        "roofline": roofline_entry(dom, kern[dom][0], kern[dom][1], kern[dom][2], kern[dom][4], kern[dom][3],
                                   args.workload),
    }
    if not args.no_cpu_baseline:
        threads = oracle_threads(args.cpu_threads)
        # the oracle gets its own inputs only: a zero target (dL/dI = 2 I)
        zero = np.zeros((scene.height, scene.width, 3))
        out["cpu_baseline"] = cpu_baseline(model, scene, params, zero, 1000, spp, threads)
        if threads > 1 and not args.no_cpu_single:
            one = cpu_baseline(model, scene, params, zero, 1000, spp, 1)
            out["cpu_baseline"]["one_thread"] = {"value": one["value"], "ms_per_iter": one["ms_per_iter"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
