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
graph followed by the fused Adam step, with the Adam kernel's HBM roofline)
and a surface-regulariser leg (neighbour lists, losses and gradients).
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
# for the kernel source it was measured on (fingerprint below: the kernel and the
# binning that builds the tile lists it walks); otherwise null.
MEASURED_TRAFFIC = {"kernel": "render_bwd_tiles", "workload": "drt-batch-500k-8views",
                    "fingerprint": "bcb1c09c8efd434b", "bytes": 3031883827,
                    "settings": (16, 16, 0, 64)}  # tile_w, tile_h, variant, batch of the measured run


def kernel_fingerprint():
    """First 16 hex digits of the sha256 of the sources with comments and blank
    lines removed (a comment edit does not change what was measured)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("gesr_render.hip", "gesr_device.h", "gesr_bin.hip"):
        with open(os.path.join(ROOT, "paper_2411_09156_amd", "csrc", f)) as fh:
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
    p.add_argument("--surface", type=int, default=0,
                   help="also time level-set surface points for this many covered pixels (32 samples per ray)")
    p.add_argument("--no-train", action="store_true",
                   help="skip the training-step leg (fwd+bwd graph followed by the fused Adam step)")
    p.add_argument("--no-gsr", action="store_true",
                   help="skip the surface-regulariser leg (neighbour lists, losses and gradients)")
    p.add_argument("--entropy", type=float, default=0.0,
                   help="weight of the opacity-entropy term in the training-step leg")
    p.add_argument("--channels", action="store_true",
                   help="extended rasterizer: depth and alpha maps in the forward and seeded synthetic upstream "
                        "gradients for them in the backward (16x16 one-wave renderer; implies --no-autotune)")
    p.add_argument("--calibrate-copy", type=int, default=0,
                   help="also run a plain device copy of this many MiB (hardware counter calibration)")
    return p.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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

    def make_step(rast, sp, target, m_cap, events=None, chan=None):
        n = sp.n
        scale = 1.0 / float(target.numel())

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
            dL = rast.l1_grad(f["image"], target, scale)
            rec(4)
            ws = rast.render_bwd_tiles(proj, bins, n, f["final_T"], f["n_contrib"], dL,
                                       dL_ddepth=None if chan is None else chan[0],
                                       dL_dalpha=None if chan is None else chan[1])
            rec(5)
            g = rast.project_bwd(sp, proj, bins, ws)
            rec(6)
            return f, g, bins
        return step

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
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            res = step()
        run = graph.replay
    else:
        res = None
        run = step
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} batched steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    if res is not None:
        cnt = res[2]["counters"].cpu().numpy().view(np.uint32)
        assert cnt[1] == 0, "instance capacity overflowed inside the graph"
    value = P / (ms * 1e-3) / 1e6

    # ------------------------------------- per-stage times (eager, events)
    names = ["project", "bin", "render_fwd", "l1_grad", "render_bwd_tiles", "seg_reduce+project_bwd"]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    tstep = make_step(rast, sp, target, m_cap, evs, chan=chan)
    tstep()
    torch.cuda.synchronize()
    acc = np.zeros(6)
    for _ in range(args.steps):
        tstep()
        torch.cuda.synchronize()
        acc += [evs[i].elapsed_time(evs[i + 1]) for i in range(6)]
    stage_ms = dict(zip(names, (acc / args.steps).round(4).tolist()))
    eager_ms = float(acc.sum() / args.steps)

    # -------------------------------------------------- per-view baseline
    per_view = None
    if not args.no_per_view:
        log("[bench] per-view pipelines")
        rasts, steps = [], []
        off = offp = 0
        for v, cam in enumerate(scene.cameras):
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
            steps.append(make_step(r, sp, tv, mv, chan=cv))

        def per_view_step():
            total = None
            for s in steps:
                f, g, _ = s()
                if total is None:
                    total = {k2: v2.clone() for k2, v2 in g.items()}
                else:
                    for k2 in total:
                        total[k2].add_(g[k2])
            return total
        for _ in range(args.warmup):
            per_view_step()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            per_view_step()
        e1.record()
        torch.cuda.synchronize()
        pv_ms = e0.elapsed_time(e1) / args.steps
        pv_graph_ms = None
        if not args.no_graph:
            g2 = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                per_view_step()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            with torch.cuda.graph(g2):
                per_view_step()
            for _ in range(args.warmup):
                g2.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                g2.replay()
            e1.record()
            torch.cuda.synchronize()
            pv_graph_ms = e0.elapsed_time(e1) / args.steps
        per_view = {"eager_ms_per_step": round(pv_ms, 4), "eager_mpix_s": round(P / (pv_ms * 1e-3) / 1e6, 2),
                    "graph_ms_per_step": None if pv_graph_ms is None else round(pv_graph_ms, 4),
                    "graph_mpix_s": None if pv_graph_ms is None else round(P / (pv_graph_ms * 1e-3) / 1e6, 2),
                    "batched_speedup_vs_eager": round(pv_ms / ms, 3),
                    "batched_speedup_vs_graph": None if pv_graph_ms is None else round(pv_graph_ms / ms, 3)}

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
    surface = None
    if args.surface > 0:
        if (rs.tile_w, rs.tile_h, rs.variant) != (16, 16, 0):
            log("[bench] --surface needs the 16x16 one-wave renderer; skipped")
        else:
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
            tbase = np.cumsum([0] + [int(tx_n[j]) * ((c.height + rs.tile_h - 1) // rs.tile_h)
                                     for j, c in enumerate(cams)])
            vv = np.searchsorted(pbase, pick, side="right") - 1
            loc = pick - pbase[vv]
            tile = tbase[vv] + (loc // widths[vv]) // rs.tile_h * tx_n[vv] + (loc % widths[vv]) // rs.tile_w
            pick = pick[np.argsort(tile, kind="stable")]
            pix_t = torch.as_tensor(pick.astype(np.int32), device="cuda")
            run_s = lambda: rast.surface_points(sp, fx["proj"], fx["bins"], fx["depth"], fx["alpha"], pix_t,  # noqa
                                                n_samples=K_S)
            sres = run_s()
            for _ in range(args.warmup):
                run_s()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                run_s()
            e1.record()
            torch.cuda.synchronize()
            s_ms = e0.elapsed_time(e1) / args.steps
            cand = int(sres["n_candidates"].to(torch.int64).sum().item())
            valid = float(sres["points"][:, 3].mean().item())
            s_ach = cand * K_S * SURFACE_SLOTS_PER_SAMPLE / (s_ms * 1e-3) / 1e12
            surface = {"rays": int(pick.size), "samples_per_ray": K_S, "ms": round(s_ms, 4),
                       "rays_per_s": round(pick.size / (s_ms * 1e-3), 1), "valid_fraction": round(valid, 4),
                       "candidates_per_ray": round(cand / max(pick.size, 1), 1),
                       "roofline": {"bound": "alu", "kernel": "surface_points", "achieved": round(s_ach, 3),
                                    "peak": round(VALU_SLOTS_PER_S / 1e12, 3), "unit": "Tslot/s",
                                    "frac": round(s_ach / (VALU_SLOTS_PER_S / 1e12), 4),
                                    "algorithmic_slots_per_launch": cand * K_S * SURFACE_SLOTS_PER_SAMPLE}}
            log(f"[bench] surface points: {pick.size} rays in {s_ms:.3f} ms, valid {valid:.3f}")
            del fx

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
    # the interval includes the read-back of the kept count
    from paper_2411_09156_amd.optim import prune
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


def cpu_baseline(scene, k, views, rs, channels=False):
    """The FP64 oracle (as it stands) on the same workload restricted to a
    subset of its views: project, bin, render, L1 gradient, backward (with the
    depth and alpha channels and seeded upstream gradients for them when
    `channels`)."""
    import copy

    import numpy as np

    import gesr_inputs as gi
    import oracle
    sub = copy.copy(scene)
    sub.cameras = [scene.cameras[v] for v in views]
    st = oracle.Settings(sh_degree=scene.sh_degree, tile_w=rs.tile_w, tile_h=rs.tile_h)
    targets = gi.target_images(scene, k)
    tgt = oracle.flat_images([targets[v] for v in views])
    log(f"[bench] cpu baseline: oracle on views {views} ({sub.n_pixels} px) with {oracle.num_threads()} threads")
    t0 = time.perf_counter()
    fo = oracle.forward(sub, st, channels=channels)
    dL = np.sign(fo["image"] - tgt) / tgt.size
    if channels:
        rng = np.random.default_rng([k, 78])
        oracle.backward(sub, st, fo, dL, dL_ddepth=rng.standard_normal(sub.n_pixels) / (3 * sub.n_pixels),
                        dL_dalpha=rng.standard_normal(sub.n_pixels) / (3 * sub.n_pixels))
    else:
        oracle.backward(sub, st, fo, dL)
    dt = time.perf_counter() - t0
    return {"value": round(sub.n_pixels / dt / 1e6, 4), "unit": "Mpix/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"views {views} of the workload ({sub.n_pixels} px, all {scene.n} splats), FP64 fwd+bwd"
                      + (" with the depth and alpha channels" if channels else "")}


if __name__ == "__main__":
    main()
