#!/usr/bin/env python3
"""Benchmark: batched forward + backward GES rendering on one MI355X.

One step = the whole hot path over every view of the workload: projection,
tile binning (radix sort), forward compositing, the L1 loss gradient, the
per-tile render adjoint and the projection adjoint, all in the HIP library,
captured once in a HIP graph and replayed.  The default workload is the
dynamic-resolution batch: 500,000 splats, 8 ring views at 1/8 .. 1 of
1600x1064 (6,304,200 pixels).

Printed: one JSON line with Mpix/s (pixels of all views per second of
fwd+bwd), the per-view comparison, per-stage times from HIP events on the
launch stream, the roofline of the dominant kernel, the FP64 oracle timed
on the host cores over a bounded sample, a training-step leg (the same
graph followed by the fused Adam step, with the Adam kernel's HBM roofline),
a surface-points leg on the sphere-shell workload (level-set points along
depth-map rays) and a surface-regulariser leg (neighbour lists, losses and
gradients); then every other workload's batched step in the same run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd render Mpix/s, batched vs per-view, at ≤1e-4 rel err vs FP64 oracle"
WORKLOADS = {"plain": 1, "spheres": 2, "drt": 3, "surfels": 4, "blobs": 5}

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.3e12 non-packed FP32 VALU
# lane-slots per second.  A transcendental (v_exp/v_log/v_rcp) occupies 2 slots of
# the same pipe (measured on gfx950: v_fma_f32 sustains 14.3 lanes/cycle/SIMD,
# v_exp_f32 7.6, and mixes of the two add up to the FMA rate).  HBM3E 8 TB/s.
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9
HBM_BYTES_PER_S = 8.0e12

# Algorithmic VALU slots per fragment (see the design notes for the count):
#   forward : 8 per listed fragment, +18 per hit (3 transcendentals x 2)
#   backward: 9 per listed fragment, +48 per hit (5 transcendentals x 2, sums fused
#             into multiply-adds)
FWD_LISTED, FWD_HIT = 8, 18
BWD_LISTED, BWD_HIT = 9, 48
# with the extended depth and alpha channels (--channels): the forward adds one
# depth multiply-add per hit; the adjoint adds the two channels' dL/dalpha terms
# (2 differences, a multiply and 2 multiply-adds), the dz term and the two
# behind-accumulator updates (8)
FWD_HIT_CHANNELS, BWD_HIT_CHANNELS = 19, 56
# surface points (--surface): per (candidate splat, sample) the affine Mahalanobis
# vector and its square (6 multiply-adds), log2, scale, exp2, scale, exp2
# (3 transcendentals x 2 + 2), the opacity and the accumulation: 16 slots
SURFACE_SLOTS_PER_SAMPLE = 16

# HBM bytes per launch of the tile adjoint on the default workload, from two
# rocprofv3 counter passes (FETCH_SIZE x2.0, WRITE_SIZE x1.0 after calibration
# against a 1 GiB copy; profiles/drt-500k-8views_hbm_counters.md).  Valid only
# for the kernel source it was measured on (fingerprint below: the kernel, the
# projection and binning that build the records and tile lists it walks, and the
# record layout); otherwise null.
MEASURED_TRAFFIC = {"kernel": "render_bwd_tiles", "workload": "drt-batch-500k-8views",
                    "fingerprint": "3a21a60edd1f05f5", "bytes": 2078642230,
                    "settings": (16, 16, 0, 64)}  # tile_w, tile_h, variant, batch of the measured run


def kernel_fingerprint():
    """First 16 hex digits of the sha256 of the sources with comments and blank
    lines removed (a comment edit does not change what was measured)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("paper_2411_09156_amd/csrc/gesr_render.hip", "paper_2411_09156_amd/csrc/gesr_device.h",
              "paper_2411_09156_amd/csrc/gesr_bin.hip", "paper_2411_09156_amd/csrc/gesr_project.hip",
              "paper_2411_09156_amd/csrc/gesr_kernels.h", "include/gesr.h"):
        with open(os.path.join(ROOT, f)) as fh:
            t = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        t = re.sub(r"//[^\n]*", "", t)
        h.update("\n".join(line.rstrip() for line in t.split("\n") if line.strip()).encode())
    return h.hexdigest()[:16]


def parse_args():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="drt", choices=sorted(WORKLOADS))
    p.add_argument("--tile", default="16x16")
    p.add_argument("--batch", type=int, default=0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-per-view", action="store_true")
    p.add_argument("--no-graph", action="store_true")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep --tile/--batch instead of the autotuner's choice")
    p.add_argument("--cpu-sample-views", default="0,1,2,3,4,5")
    p.add_argument("--surface", type=int, default=65536,
                   help="time level-set surface points for this many covered pixels (32 samples per ray; 0: skip)")
    p.add_argument("--surface-workload", type=int, default=2,
                   help="workload of the surface-points leg (default: the sphere shells)")
    p.add_argument("--no-train", action="store_true",
                   help="skip the training-step leg (fwd+bwd graph followed by the fused Adam step)")
    p.add_argument("--no-gsr", action="store_true",
                   help="skip the surface-regulariser leg (neighbour lists, losses and gradients)")
    p.add_argument("--entropy", type=float, default=0.0,
                   help="weight of the opacity-entropy term in the training-step leg")
    p.add_argument("--channels", action="store_true",
                   help="extended rasterizer: depth and alpha maps in the forward and seeded synthetic upstream "
                        "gradients for them in the backward (16x16 one-wave renderer; implies --no-autotune)")
    p.add_argument("--workloads", default="1,2,4,5",
                   help="other configurations timed in the same run after the headline (comma list of 1..5; "
                        "'' for none)")
    p.add_argument("--workload-steps", type=int, default=10, help="timed steps of each other workload")
    p.add_argument("--calibrate-copy", type=int, default=0,
                   help="also run a plain device copy of this many MiB (hardware counter calibration)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_step_fn(scene):
    """Step builder for the workload's loss: "l1" (mean |X - Y| over all
    values), "l1+dssim" (Eq. 8 per view, lambda 0.2, the loss kernel) or
    "l1+surface" (L1 plus the surface-alignment regulariser, weights 0.1,
    whose gradient is added to the parameter gradients)."""
    import numpy as np
    import torch
    normals = None
    if scene.loss == "l1+surface":
        normals = torch.as_tensor(np.ascontiguousarray(np.asarray(scene.normals, np.float32).T), device="cuda")
    if scene.loss not in ("l1", "l1+dssim", "l1+surface"):
        raise ValueError(f"unsupported loss {scene.loss!r}")

    def make_step(rast, sp, target, m_cap, events=None, chan=None):
        n = sp.n
        scale = 1.0 / float(target.numel())
        loss_ws = rast.alloc_loss_workspace() if scene.loss == "l1+dssim" else None

        def rec(i):
            if events is not None:
                events[i].record()

        def step():
            rec(0)
            proj = rast.project(sp)
            rec(1)
            bins = rast.bin(proj, n, m_cap=m_cap, sync=False)
            rec(2)
            f = rast.render_fwd(proj, bins, n, channels=chan is not None)
            rec(3)
            if scene.loss == "l1+dssim":
                dL, _ = rast.loss_eq8(f["image"], target, 0.2, want_loss=False, workspace=loss_ws)
            else:
                dL = rast.l1_grad(f["image"], target, scale)
            rec(4)
            ws = rast.render_bwd_tiles(proj, bins, n, f["final_T"], f["n_contrib"], dL,
                                       dL_ddepth=None if chan is None else chan[0],
                                       dL_dalpha=None if chan is None else chan[1])
            rec(5)
            g = rast.project_bwd(sp, proj, bins, ws)
            if normals is not None:
                rast.surface_align(sp, normals, g, 0.1, 0.1, want_losses=False)
            rec(6)
            return f, g, bins
        return step
    return make_step


def time_step(step, steps, warmup, graph=True):
    """ms per step of `step` (captured in a HIP graph and replayed unless
    graph=False), HIP events on the launch stream around `steps` replays after
    `warmup`; returns (ms, wall seconds of the timed loop, the captured
    outputs or None)."""
    import torch
    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    res = None
    run = step
    if graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            res = step()
        run = g.replay
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, time.perf_counter() - t0, res


def stage_times(make_step, rast, sp, target, m_cap, chan, steps, names):
    """Per-stage milliseconds (eager, HIP events between the stages on the
    launch stream) and their sum."""
    import numpy as np
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    tstep = make_step(rast, sp, target, m_cap, evs, chan=chan)
    tstep()
    torch.cuda.synchronize()
    acc = np.zeros(6)
    for _ in range(steps):
        tstep()
        torch.cuda.synchronize()
        acc += [evs[i].elapsed_time(evs[i + 1]) for i in range(6)]
    return dict(zip(names, (acc / steps).round(4).tolist())), float(acc.sum() / steps)


def per_view_times(scene, rs, sp, target, chan, make_step, steps, warmup, graph=True):
    """The same pipeline view by view (V sequential one-view pipelines, the
    parameter gradients summed), eager and captured in one graph."""
    import torch
    from paper_2411_09156_amd import Rasterizer
    rasts, vsteps = [], []
    off = offp = 0
    P = scene.n_pixels
    for cam in scene.cameras:
        r = Rasterizer([cam], rs, store_tile_ids=False)
        npx = 3 * cam.width * cam.height
        tv = target[off:off + npx]
        cv = None if chan is None else tuple(c[offp:offp + npx // 3] for c in chan)
        off += npx
        offp += npx // 3
        fv = r.forward(sp, sync=True)
        mv = int(fv["bins"]["M"])
        del fv
        rasts.append(r)
        vsteps.append(make_step(r, sp, tv, mv, chan=cv))

    def per_view_step():
        total = None
        for st_ in vsteps:
            f, g, _ = st_()
            if total is None:
                total = {k2: v2.clone() for k2, v2 in g.items()}
            else:
                for k2 in total:
                    total[k2].add_(g[k2])
        return total
    pv_ms, _, _ = time_step(per_view_step, steps, warmup, graph=False)
    pv_graph_ms = time_step(per_view_step, steps, warmup, graph=True)[0] if graph else None
    del rasts, vsteps
    return {"eager_ms_per_step": round(pv_ms, 4), "eager_mpix_s": round(P / (pv_ms * 1e-3) / 1e6, 2),
            "graph_ms_per_step": None if pv_graph_ms is None else round(pv_graph_ms, 4),
            "graph_mpix_s": None if pv_graph_ms is None else round(P / (pv_graph_ms * 1e-3) / 1e6, 2)}


def workload_leg(k, args, rs):
    """Workload k (one of the other configurations) timed in this same run:
    batched fwd+bwd in a graph vs the per-view pipelines, its own autotuned
    settings (the headline's with --no-autotune), its own loss; the peak
    device memory of its sizing run and batched step above what was allocated
    before (torch's allocator: splats, targets, lists, workspaces, outputs)
    and the sizes of the binning and backward buffers."""
    import numpy as np
    import torch

    import gesr_inputs as gi
    from paper_2411_09156_amd import Rasterizer, RasterSettings, Splats
    from paper_2411_09156_amd._lib import REC_FLOATS
    log(f"[bench] workload {k}: building")
    scene = gi.make_workload(k)
    N, V, P = scene.n, scene.n_views, scene.n_pixels
    rsk = RasterSettings(sh_degree=scene.sh_degree, tile_w=rs.tile_w, tile_h=rs.tile_h, batch=rs.batch,
                         radix_bits=rs.radix_bits, variant=rs.variant)
    sp = Splats.from_aos(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas, scene.sh)
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in gi.target_images(scene, k)]), device="cuda")
    rast = Rasterizer(scene.cameras, rsk, store_tile_ids=False)
    tune = None
    if not args.no_autotune:
        tune = rast.autotune(sp, reps=2)
        rsk = rast.settings
        log(f"[bench] workload {k}: autotune chose tile {tune['tile']} variant {tune['variant']} batch "
            f"{tune['batch']} radix {tune['radix_bits']}")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    mem0 = torch.cuda.memory_allocated()
    first = rast.forward(sp, sync=True, counts=True)
    M = int(first["bins"]["M"])
    listed_inst = int(first["bins"]["counters"][3].item())
    n_listed = int(first["n_listed"].to(torch.int64).sum().item())
    n_hit = int(first["n_hit"].to(torch.int64).sum().item())
    del first
    make_step = make_step_fn(scene)
    step = make_step(rast, sp, target, M)
    ms, _, res = time_step(step, args.workload_steps, args.warmup, graph=not args.no_graph)
    if res is not None:
        assert res[2]["counters"].cpu().numpy().view(np.uint32)[1] == 0, "instance capacity overflowed"
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - mem0
    sz = rast.sizes(N, M)
    T = int(sz.total_tiles)
    names = ["project", "bin", "render_fwd", "loss_grad", "render_bwd_tiles", "seg_reduce+project_bwd"]
    stage_ms, _ = stage_times(make_step, rast, sp, target, M, None, max(args.workload_steps // 2, 2), names)
    del res, step
    pv = per_view_times(scene, rsk, sp, target, None, make_step, args.workload_steps, args.warmup,
                        graph=not args.no_graph)
    value = P / (ms * 1e-3) / 1e6
    log(f"[bench] workload {k} ({scene.name}): {ms:.3f} ms per step, {value:.1f} Mpix/s; per view "
        f"{pv['eager_ms_per_step']:.3f} ms eager, {pv['graph_ms_per_step']} ms graph")
    out = {"workload": scene.name, "splats": N, "views": V, "pixels": P, "sh_degree": scene.sh_degree,
           "loss": scene.loss, "value": round(value, 2), "unit": "Mpix/s", "ms_per_step": round(ms, 4),
           "steps": args.workload_steps, "instances": M, "listed_instances": listed_inst,
           "fragments": {"listed": n_listed, "hit": n_hit, "listed_per_s": round(n_listed / (ms * 1e-3), 1),
                         "hit_per_s": round(n_hit / (ms * 1e-3), 1)},
           "stages_ms": stage_ms, "per_view": pv,
           "batched_speedup_vs_eager": round(pv["eager_ms_per_step"] / ms, 3),
           "batched_speedup_vs_graph": None if pv["graph_ms_per_step"] is None
           else round(pv["graph_ms_per_step"] / ms, 3),
           "settings": {"tile": f"{rsk.tile_w}x{rsk.tile_h}", "variant": rsk.variant, "batch": rsk.batch or 64,
                        "radix_bits": rsk.radix_bits, "autotuned": tune is not None},
           "memory": {"peak_step_bytes": int(peak), "bin_scratch_bytes": int(sz.bin_scratch_bytes),
                      "sort_buffer_bytes": 16 * V * N,  # depth/view sort ping-pong keys and values, in the scratch
                      "sorted_list_bytes": 4 * M, "ranges_worklist_bytes": 12 * T,
                      "bwd_workspace_bytes": int(sz.bwd_workspace_bytes),
                      "projection_bytes": V * N * (REC_FLOATS * 4 + 16)}}  # record, count, rectangle, depth key
    del rast, sp, target
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU design "
              "(views sharded across GPUs, one gradient all-reduce) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gesr_inputs as gi
    from paper_2411_09156_amd import Rasterizer, RasterSettings, Splats

    torch.cuda.init()
    k = WORKLOADS[args.workload]
    tw, th = (int(x) for x in args.tile.split("x"))
    log(f"[bench] building workload {args.workload}")
    scene = gi.make_workload(k)
    N, V, P = scene.n, scene.n_views, scene.n_pixels
    rs = RasterSettings(sh_degree=scene.sh_degree, tile_w=tw, tile_h=th, batch=args.batch)
    sp = Splats.from_aos(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas, scene.sh)
    target = torch.as_tensor(np.concatenate([t.reshape(-1) for t in gi.target_images(scene, k)]), device="cuda")
    chan = None
    if args.channels:
        # upstream gradients of the depth and alpha maps (a stand-in for a depth
        # or mask loss): seeded normals scaled like the L1 image gradient
        rng = np.random.default_rng([k, 77])
        chan = tuple(torch.as_tensor((rng.standard_normal(P) / (3 * P)).astype(np.float32), device="cuda")
                     for _ in range(2))
        if not args.no_autotune:
            log("[bench] --channels: the extended channels run in the 16x16 one-wave renderer; autotuning is skipped")
            args.no_autotune = True

    make_step = make_step_fn(scene)

    if args.calibrate_copy > 0:
        # plain device-to-device copy of known size, for scaling HBM byte counters
        src = torch.empty(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst

    # ------------------------------------------------------------ sizing
    rast = Rasterizer(scene.cameras, rs, store_tile_ids=False)
    tune = None
    if not args.no_autotune:
        log("[bench] autotuning tile shape, renderer, LDS batch and depth-sort digit width")
        tune = rast.autotune(sp, reps=3)
        rs = rast.settings
        log(f"[bench] autotune chose tile {tune['tile']} variant {tune['variant']} batch {tune['batch']} "
            f"radix {tune['radix_bits']}")
    log("[bench] sizing run (eager, synchronous count)")
    first = rast.forward(sp, sync=True, counts=True)
    M = int(first["bins"]["M"])
    listed_inst = int(first["bins"]["counters"][3].item())
    m_cap = M
    n_listed = int(first["n_listed"].to(torch.int64).sum().item())
    n_hit = int(first["n_hit"].to(torch.int64).sum().item())
    del first
    torch.cuda.synchronize()
    log(f"[bench] M={M} instance slots, {listed_inst} in the tile lists, listed={n_listed}, hit={n_hit}")

    # ---------------------------------------------------- batched, graph
    step = make_step(rast, sp, target, m_cap, chan=chan)
    ms, wall, res = time_step(step, args.steps, args.warmup, graph=not args.no_graph)
    if res is not None:
        cnt = res[2]["counters"].cpu().numpy().view(np.uint32)
        assert cnt[1] == 0, "instance capacity overflowed inside the graph"
    value = P / (ms * 1e-3) / 1e6
    log(f"[bench] batched: {ms:.4f} ms per step, {value:.1f} Mpix/s")

    # ------------------------------------- per-stage times (eager, events)
    names = ["project", "bin", "render_fwd", "loss_grad", "render_bwd_tiles", "seg_reduce+project_bwd"]
    stage_ms, eager_ms = stage_times(make_step, rast, sp, target, m_cap, chan, args.steps, names)

    # -------------------------------------------------- per-view baseline
    per_view = None
    if not args.no_per_view:
        log("[bench] per-view pipelines")
        per_view = per_view_times(scene, rs, sp, target, chan, make_step, args.steps, args.warmup,
                                  graph=not args.no_graph)
        per_view["batched_speedup_vs_eager"] = round(per_view["eager_ms_per_step"] / ms, 3)
        if per_view["graph_ms_per_step"] is not None:
            per_view["batched_speedup_vs_graph"] = round(per_view["graph_ms_per_step"] / ms, 3)

    # ------------------------------------------------------------ roofline
    fwd_hit, bwd_hit = (FWD_HIT_CHANNELS, BWD_HIT_CHANNELS) if args.channels else (FWD_HIT, BWD_HIT)
    fwd_slots = FWD_LISTED * n_listed + fwd_hit * n_hit
    bwd_slots = BWD_LISTED * n_listed + bwd_hit * n_hit
    kern = {"render_fwd": fwd_slots, "render_bwd_tiles": bwd_slots}
    dom = max(kern, key=lambda kk: stage_ms[kk])
    achieved = kern[dom] / (stage_ms[dom] * 1e-3) / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    traffic = None
    if (not args.channels and dom == MEASURED_TRAFFIC["kernel"] and scene.name == MEASURED_TRAFFIC["workload"]
            and kernel_fingerprint() == MEASURED_TRAFFIC["fingerprint"]
            and (rs.tile_w, rs.tile_h, rs.variant, rs.batch or 64) == MEASURED_TRAFFIC["settings"]):
        traffic = MEASURED_TRAFFIC["bytes"]
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "Tslot/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "algorithmic_slots_per_launch": int(kern[dom])}

    # ------------------------------------------------------ surface points
    surface = surface_leg(args) if args.surface > 0 else None

    # ------------------------------------------- training step with Adam
    train = None
    if not args.no_train:
        train = train_leg(args, scene, rast, target, M, make_step, P)

    # ------------------------------------------- surface regulariser (GSR)
    gsr_out = None
    if not args.no_gsr:
        gsr_out = gsr_leg(args, scene, sp, rs)

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, k, [int(x) for x in args.cpu_sample_views.split(",")], rs, args.channels)

    # --------------------------------------- the other workloads, same run
    others = {}
    wl = [int(x) for x in args.workloads.split(",") if x.strip()]
    if wl:
        del rast, sp, target, res, step
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for kk in wl:
            if kk == k:
                continue
            others[f"cfg{kk}"] = workload_leg(kk, args, rs)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": scene.name, "splats": N, "views": V, "pixels": P,
                   "resolutions": [f"{c.width}x{c.height}" for c in scene.cameras], "sh_degree": scene.sh_degree,
                   "tile": f"{rs.tile_w}x{rs.tile_h}", "variant": rs.variant, "batch": rs.batch or 64,
                   "radix_bits": rs.radix_bits, "graph": not args.no_graph, "instances": M,
                   "listed_instances": listed_inst,
                   "channels": bool(args.channels)},
        "fragments": {"listed": n_listed, "hit": n_hit,
                      "listed_per_s": round(n_listed / (ms * 1e-3), 1), "hit_per_s": round(n_hit / (ms * 1e-3), 1)},
        "stages_ms": stage_ms, "eager_ms_per_step": round(eager_ms, 4), "per_view": per_view,
        "roofline": roofline, "cpu_baseline": cpu, "wall_s_timed": round(wall, 3),
        "autotune": tune,
    }
    if surface is not None:
        out["surface"] = surface
    if train is not None:
        out["train"] = train
    if gsr_out is not None:
        out["gsr"] = gsr_out
    if others:
        out["workloads"] = others
    print(json.dumps(out), flush=True)


def train_leg(args, scene, rast, target, M, make_step, P):
    """Training step of the schedule (Sec. 4.2): the batched fwd+bwd graph on
    the optimiser's activated parameters, then one fused Adam step of the raw
    parameters (with the opacity-entropy term), repeated; and the Adam kernel
    alone against the HBM roofline."""
    import numpy as np
    import torch

    from paper_2411_09156_amd.optim import AdamConfig, RawParams, SplatAdam
    log("[bench] training steps: fwd+bwd graph, then the fused Adam step")
    op = np.clip(np.asarray(scene.opacities, np.float64), 1e-6, 1 - 1e-6)
    raw = RawParams.from_aos(scene.means, np.log(np.asarray(scene.scales, np.float64)), scene.quats,
                             np.log(op / (1 - op)), scene.betas, scene.sh)
    opt = SplatAdam(raw, AdamConfig(entropy_weight=args.entropy))
    m_cap = int(M * 1.5) + 4096  # the footprints move while training
    step = make_step(rast, opt.splats, target, m_cap)
    step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        f, g, bins = step()

    def l1():
        return float((f["image"][:3 * P] - target).abs().mean().item())
    graph.replay()
    torch.cuda.synchronize()
    l1_first = l1()
    for _ in range(args.warmup):
        graph.replay()
        opt.step(g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
        opt.step(g)
    e1.record()
    torch.cuda.synchronize()
    tr_ms = e0.elapsed_time(e1) / args.steps
    graph.replay()
    torch.cuda.synchronize()
    l1_last = l1()
    overflow = int(bins["counters"].cpu().numpy().view(np.uint32)[1])
    # the Adam kernel alone (events on the stream it is launched on)
    e0.record()
    for _ in range(args.steps):
        opt.step(g)
    e1.record()
    torch.cuda.synchronize()
    adam_ms = e0.elapsed_time(e1) / args.steps
    # one pruning pass of the trained state (opacity and shape thresholds 0.5);
    # the interval includes the read-back of the kept count; a first pass
    # leaves the allocator holding blocks of the output sizes
    from paper_2411_09156_amd.optim import prune
    prune(opt.raw, opt.m, opt.v, 0.5, 0.5)
    torch.cuda.synchronize()
    e0.record()
    kept = prune(opt.raw, opt.m, opt.v, 0.5, 0.5)[0].n
    e1.record()
    torch.cuda.synchronize()
    prune_ms = e0.elapsed_time(e1)
    n, K = scene.n, opt.raw.sh_coeffs
    rows = 12 + 3 * K
    # per splat: read p, m, v, g and write p, m, v for every row; write the
    # activated scale (3 rows) and opacity
    bytes_launch = n * (rows * 7 * 4 + 4 * 4)
    ach = bytes_launch / (adam_ms * 1e-3)
    log(f"[bench] train step {tr_ms:.3f} ms (Adam {adam_ms:.4f} ms), L1 {l1_first:.5f} -> {l1_last:.5f}")
    return {"ms_per_step": round(tr_ms, 4), "mpix_s": round(P / (tr_ms * 1e-3) / 1e6, 2),
            "steps": args.steps + args.warmup, "l1_first": round(l1_first, 6), "l1_last": round(l1_last, 6),
            "instance_overflow": bool(overflow), "entropy_weight": args.entropy,
            "prune": {"ms_incl_readback": round(prune_ms, 4), "kept": kept, "of": scene.n},
            "adam": {"ms": round(adam_ms, 4), "rows": rows,
                     "roofline": {"bound": "hbm", "kernel": "adam_step", "achieved": round(ach / 1e9, 1),
                                  "peak": HBM_BYTES_PER_S / 1e9, "unit": "GB/s",
                                  "frac": round(ach / HBM_BYTES_PER_S, 4), "traffic": None,
                                  "algorithmic_bytes_per_launch": bytes_launch}}}


def gsr_leg(args, scene, sp, rs):
    """Surface regulariser of Sec. 3.3 (Eq. 9-13) on the workload's splats:
    the 16-neighbour lists with their inverse (one refresh), then one sample
    per splat with losses and gradients, against the HBM roofline of its
    algorithmic bytes."""
    import numpy as np
    import torch

    from paper_2411_09156_amd.gsr import gsr, knn
    log("[bench] surface regulariser: neighbour lists, then losses and gradients")
    n = sp.n
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nb = knn(sp, 16)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        nb = knn(sp, 16)
    e1.record()
    torch.cuda.synchronize()
    knn_ms = e0.elapsed_time(e1) / args.steps
    xi = torch.as_tensor(np.random.default_rng(31).standard_normal((3, n)).astype(np.float32), device="cuda")
    grads = {k: torch.zeros_like(getattr(sp, k)) for k in ("mean", "scale", "quat", "opacity", "beta")}
    w = 1.0 / n
    out = gsr(sp, rs, nb, xi, w_sdf=w, w_nor=w, grads=grads)
    for _ in range(args.warmup):
        gsr(sp, rs, nb, xi, w_sdf=w, w_nor=w, grads=grads)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        out = gsr(sp, rs, nb, xi, w_sdf=w, w_nor=w, grads=grads)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    losses = out["losses"].cpu().numpy().astype(np.float64) / n
    # algorithmic HBM bytes per splat: frames (48 B of parameters read, 64 B
    # written), the loss pass (own frame 64, xi 12, list 64, partials 16 x 48
    # written, per-sample results 16), the gather (inverse list 68, partials
    # 768, gradients 48 read + 48 written) and the loss sum (16)
    per_splat = 48 + 64 + (64 + 12 + 64 + 768 + 16) + (68 + 768 + 96) + 16
    ach = per_splat * n / (ms * 1e-3)
    log(f"[bench] gsr: knn {knn_ms:.3f} ms, losses + gradients {ms:.3f} ms, L_sdf {losses[0]:.4g} L_nor {losses[1]:.4g}")
    return {"splats": n, "neighbours": 16, "knn_ms": round(knn_ms, 4), "ms": round(ms, 4),
            "samples_per_s": round(n / (ms * 1e-3), 1), "l_sdf": round(float(losses[0]), 6),
            "l_nor": round(float(losses[1]), 6),
            "roofline": {"bound": "hbm", "kernel": "gsr (frames + loss + gather + sum)", "achieved": round(ach / 1e9, 1),
                         "peak": HBM_BYTES_PER_S / 1e9, "unit": "GB/s", "frac": round(ach / HBM_BYTES_PER_S, 4),
                         "traffic": None, "algorithmic_bytes_per_launch": per_splat * n}}


def surface_leg(args):
    """Level-set surface points (the mesh-extraction sampling step) on the
    workload --surface-workload (default: the sphere shells, where the density
    of the opaque shells crosses the 0.3 level at most covered pixels): the
    extended forward gives the depth and alpha maps, then --surface rays at
    pixels with alpha >= 0.5, grouped by tile, K = 32 samples each."""
    import numpy as np
    import torch

    import gesr_inputs as gi
    from paper_2411_09156_amd import Rasterizer, RasterSettings, Splats
    k = args.surface_workload
    scene = gi.make_workload(k)
    log(f"[bench] surface points on workload {k} ({scene.name})")
    rs = RasterSettings(sh_degree=scene.sh_degree, tile_w=16, tile_h=16, variant=0)
    sp = Splats.from_aos(scene.means, scene.scales, scene.quats, scene.opacities, scene.betas, scene.sh)
    rast = Rasterizer(scene.cameras, rs, store_tile_ids=False)
    K_S = 32
    fx = rast.forward(sp, sync=True, channels=True)
    alpha_h = fx["alpha"].cpu().numpy()
    cov = np.nonzero(alpha_h >= 0.5)[0]
    pick = np.random.default_rng([k, 79]).choice(cov, min(args.surface, cov.size), replace=False)
    # grouped by tile, so the rays a wave serves share their tile's list
    cams = scene.cameras
    widths = np.array([c.width for c in cams])
    pbase = np.cumsum([0] + [c.width * c.height for c in cams])
    tx_n = (widths + rs.tile_w - 1) // rs.tile_w
    tbase = np.cumsum([0] + [int(tx_n[j]) * ((c.height + rs.tile_h - 1) // rs.tile_h) for j, c in enumerate(cams)])
    vv = np.searchsorted(pbase, pick, side="right") - 1
    loc = pick - pbase[vv]
    tile = tbase[vv] + (loc // widths[vv]) // rs.tile_h * tx_n[vv] + (loc % widths[vv]) // rs.tile_w
    pick = pick[np.argsort(tile, kind="stable")]
    pix_t = torch.as_tensor(pick.astype(np.int32), device="cuda")

    def run_s():
        return rast.surface_points(sp, fx["proj"], fx["bins"], fx["depth"], fx["alpha"], pix_t, n_samples=K_S)
    sres = run_s()
    for _ in range(args.warmup):
        run_s()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        run_s()
    e1.record()
    torch.cuda.synchronize()
    s_ms = e0.elapsed_time(e1) / args.steps
    cand = int(sres["n_candidates"].to(torch.int64).sum().item())
    valid = float(sres["points"][:, 3].mean().item())
    s_ach = cand * K_S * SURFACE_SLOTS_PER_SAMPLE / (s_ms * 1e-3) / 1e12
    log(f"[bench] surface points: {pick.size} rays in {s_ms:.3f} ms, valid {valid:.3f}")
    return {"workload": scene.name, "rays": int(pick.size), "covered_pixels": int(cov.size),
            "samples_per_ray": K_S, "ms": round(s_ms, 4), "rays_per_s": round(pick.size / (s_ms * 1e-3), 1),
            "valid_fraction": round(valid, 4), "candidates_per_ray": round(cand / max(pick.size, 1), 1),
            "roofline": {"bound": "alu", "kernel": "surface_points", "achieved": round(s_ach, 3),
                         "peak": round(VALU_SLOTS_PER_S / 1e12, 3), "unit": "Tslot/s",
                         "frac": round(s_ach / (VALU_SLOTS_PER_S / 1e12), 4),
                         "algorithmic_slots_per_launch": cand * K_S * SURFACE_SLOTS_PER_SAMPLE}}


def cpu_info():
    """Host CPU model (as lscpu reports it, from /proc/cpuinfo), logical CPUs and
    the threads this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_threads": usable}


def cpu_baseline(scene, k, views, rs, channels=False):
    """The FP64 oracle (as it stands) on the same workload restricted to a
    subset of its views: project, bin, render, L1 gradient, backward (with the
    depth and alpha channels and seeded upstream gradients for them when
    `channels`); and the same on the first of those views with one thread."""
    import copy

    import numpy as np

    import gesr_inputs as gi
    import oracle
    st = oracle.Settings(sh_degree=scene.sh_degree, tile_w=rs.tile_w, tile_h=rs.tile_h)
    targets = gi.target_images(scene, k)

    def run(vs):
        sub = copy.copy(scene)
        sub.cameras = [scene.cameras[v] for v in vs]
        tgt = oracle.flat_images([targets[v] for v in vs])
        t0 = time.perf_counter()
        fo = oracle.forward(sub, st, channels=channels)
        dL = np.sign(fo["image"] - tgt) / tgt.size
        if channels:
            rng = np.random.default_rng([k, 78])
            oracle.backward(sub, st, fo, dL, dL_ddepth=rng.standard_normal(sub.n_pixels) / (3 * sub.n_pixels),
                            dL_dalpha=rng.standard_normal(sub.n_pixels) / (3 * sub.n_pixels))
        else:
            oracle.backward(sub, st, fo, dL)
        return sub.n_pixels, time.perf_counter() - t0

    threads = oracle.num_threads()
    log(f"[bench] cpu baseline: oracle on views {views} with {threads} threads")
    px, dt = run(views)
    oracle.set_threads(1)
    try:
        log(f"[bench] cpu baseline: oracle on view {views[0]} with one thread")
        px1, dt1 = run(views[:1])
    finally:
        oracle.set_threads(threads)
    suffix = " with the depth and alpha channels" if channels else ""
    out = {"value": round(px / dt / 1e6, 4), "unit": "Mpix/s", "cores": threads, "kind": "oracle",
           "seconds": round(dt, 2),
           "sample": f"views {views} of the workload ({px} px, all {scene.n} splats), FP64 fwd+bwd" + suffix,
           "single_thread": {"value": round(px1 / dt1 / 1e6, 5), "unit": "Mpix/s", "seconds": round(dt1, 2),
                             "sample": f"view {views[0]} ({px1} px, all {scene.n} splats), FP64 fwd+bwd" + suffix}}
    out.update(cpu_info())
    return out


if __name__ == "__main__":
    main()
