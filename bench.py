"""Benchmark: 640x480 HOG face detection on one MI355X, batched vs plain.

A step is one pass of the whole detection path (pyramid, gradients,
histograms, features, window scores, threshold, NMS) over one 64-frame
clip of 640x480 frames with 5 filters, replayed from a hipGraph, inputs
already in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s + p99 frame latency, 640×480 HOG detect, batched vs plain on one GPU"
H, W_PX, NF, CLIP = 480, 640, 5, 64
FP32_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
HBM_PEAK_GBS = 8000.0
# Vector-ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# operation per lane per cycle (no packed FP32 in this build)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic vector operations per pyramid pixel of the histogram stage:
# resample 6 (three 2-tap lerps; none at a scale-1 level, so 6 x 0.69 = 4 on
# the 640x480 pyramid), central differences 2, magnitude 3, orientation 11
# (four boundary tests, their signs, the unfold), four weighted votes 8.
HIST_OPS_PER_PX = 28
# Per cell of the feature stage: 4 block sums 12, 4 normalisers 8, 27
# truncated products x 4 blocks 216 (multiply, min, add), 4 energy sums 72.
FEAT_OPS_PER_CELL = 308

KERNEL_SOURCES = {
    "hog_hist_kernel": ("hog_internal.h", "hog_device.h", "stage_hist.h", "k_hist.hip"),
    "hog_score_kernel": ("hog_internal.h", "hog_device.h", "stage_score.h", "k_score.hip"),
    "hog_sep_score_kernel": ("hog_internal.h", "hog_device.h", "stage_score.h", "k_score.hip"),
    "hog_feat_kernel": ("hog_internal.h", "hog_device.h", "stage_feat.h", "k_feat.hip"),
}


def kernel_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3
    counter summaries (FETCH_SIZE and WRITE_SIZE, calibrated by a plain
    copy), if the kernel's sources are still the ones profiled; else None."""
    import glob
    import hashlib
    if kernel not in KERNEL_SOURCES:
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2006_00816_amd", "csrc", f), "rb").read()
                   for f in KERNEL_SOURCES[kernel])
    sha = hashlib.sha256(src).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if line.startswith("traffic "):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("sha256_16") == sha:
                    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def pyramid_stats(h, w, nf):
    from paper_2006_00816_amd import hog355
    lv = hog355.pyramid(h, w, 1, nf)
    return {"pixels": sum(l["h"] * l["w"] for l in lv), "cells": sum(l["cy"] * l["cx"] for l in lv),
            "windows": sum(l["rows"] * l["cols"] for l in lv), "levels": len(lv)}


def kernel_times(hog355, run, names, steps):
    """Per kernel: HIP-event launch durations on the launch streams over
    `steps` eager steps: ms per launch, launches per step, ms per step."""
    import torch
    run()
    torch.cuda.synchronize()
    hog355.profile_reset()
    hog355.profile_enable(True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    res = {}
    for name in names:
        ms, cnt = hog355.profile_read(name)
        if cnt:
            res[name] = {"ms_per_launch": round(ms / cnt, 5), "launches_per_step": round(cnt / steps, 3),
                         "ms_per_step": round(ms / steps, 5)}
    hog355.profile_enable(False)
    hog355.profile_reset()
    return res


def rooflines(kt, ps, frames, score_flop_per_window, score_kernel):
    """Roofline entries of the stage kernels: algorithmic work per launch
    (per-frame work x frames per launch) over the measured launch time."""
    entries = []
    defs = [("hist", "hog_hist_kernel", "alu", HIST_OPS_PER_PX * ps["pixels"], VALU_PEAK_TOPS, "Tops/s"),
            ("feat", "hog_feat_kernel", "alu", FEAT_OPS_PER_CELL * ps["cells"], VALU_PEAK_TOPS, "Tops/s"),
            ("score", score_kernel, "mfma", score_flop_per_window * ps["windows"], FP32_PEAK_TFLOPS, "TFLOP/s")]
    for name, kernel, bound, per_frame, peak, unit in defs:
        if name not in kt:
            continue
        t = kt[name]
        fpl = frames / t["launches_per_step"]
        work = per_frame * fpl
        achieved = work / (t["ms_per_launch"] * 1e-3) / 1e12
        entries.append({"bound": bound, "kernel": kernel, "achieved": round(achieved, 3), "peak": round(peak, 2),
                        "unit": unit, "frac": round(achieved / peak, 4), "traffic": kernel_traffic(kernel),
                        "work_per_launch": work, "frames_per_launch": fpl, "avg_launch_ms": t["ms_per_launch"],
                        "ms_per_step": t["ms_per_step"]})
    return entries


def _oracle_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    frame, W, b = args
    from oracle import hog as oracle
    oracle.detect(frame, W, b)
    return True


def profiler_active(env=None) -> bool:
    """True when a rocprofiler tool library is preloaded (rocprofv3 sets
    LD_PRELOAD and ROCPROF* variables): every process started then
    initialises the GPU under the profiler, so no worker pool may start."""
    env = os.environ if env is None else env
    if "rocprof" in env.get("LD_PRELOAD", ""):
        return True
    return any(k.startswith(("ROCPROF", "ROCP_")) for k in env)


def cpu_baseline(frames, W, b, budget_frames):
    """The float64 oracle on host cores, one process per frame.  Not run
    under a profiler (returns None without starting a process)."""
    if profiler_active():
        return None
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16, budget_frames)
    sample = [(frames[i % len(frames)], W, b) for i in range(budget_frames)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_worker, sample[:cores])          # import / warm-up
        t0 = time.perf_counter()
        pool.map(_oracle_worker, sample)
        dt = time.perf_counter() - t0
    return {"value": len(sample) / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} frames of the 640x480 clip, float64 numpy oracle, "
                      f"one process per frame on {cores} host cores, {dt:.1f} s wall"}


def train_leg(steps):
    """Filter training on config-3 crops (4,096 positives, 16,384
    negatives): window scores, hinge loss + 1e-4 L2, filter backward with
    recomputed features, update.  Times whole steps."""
    import torch
    from paper_2006_00816_amd import hog355, synth
    crops, labels = synth.config3(seed=3)
    W0, b0 = synth.filters([3])
    cr = torch.from_numpy(crops).cuda()
    lb = torch.from_numpy(labels).cuda()
    W = torch.from_numpy(W0).cuda()
    b = torch.from_numpy(b0).cuda()
    n = int(cr.shape[0])
    win = hog355.windows_tensor(torch.arange(n, dtype=torch.int32), 0, 0, 0, 0)
    ws = hog355.Workspace()

    def step():
        s = hog355.window_scores(cr, W, b, win, ws=ws)
        loss, dscore, dW = hog355.hinge_loss(s, lb, W, 1e-4)
        dW, db, _ = hog355.filter_backward(cr, W, win, dscore, dW=dW, ws=ws)
        W.sub_(0.5 * dW)
        b.sub_(0.5 * db)
        return loss

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"workload": "config 3: 20,480 80x80 u8 crops, 1 filter f32, hinge + 1e-4 L2, full batch",
            "steps": steps, "ms_per_step": round(1e3 * dt, 4), "crops_per_s": round(n / dt, 1),
            "loss_after": round(float(loss.item()), 6)}


def pixel_grad_leg(n_frames, chunk):
    """Config 4: 1920x1080 frames on a pyramid from 2x, 5 filters: detect,
    top-10 windows and the backward of their summed scores to the pixels,
    in chunks of frames.  Times the whole pass over n_frames."""
    import torch
    from paper_2006_00816_amd import hog355, synth
    wl = synth.config4(seed=4, n=n_frames)
    fr = torch.from_numpy(wl.frames).cuda()
    W = torch.from_numpy(wl.W).cuda()
    b = torch.from_numpy(wl.b).cuda()
    ws_d, ws_g = hog355.Workspace(), hog355.Workspace()
    dets, nd = hog355.alloc_dets(chunk, 256)
    ones = torch.ones(chunk * 10, device="cuda")

    def run(lo, hi):
        f = fr[lo:hi]
        m = hi - lo
        # detections and top-10 windows from one forward pass
        win, _ = hog355.detect_topk_into(f, W, b, dets[:m], nd[:m], 10, upsample=2, ws=ws_d)
        _, _, dpix = hog355.filter_backward(f, W, win.reshape(-1, 5).contiguous(), ones[:m * 10], upsample=2,
                                            pixels=True, ws=ws_g)
        return dpix

    run(0, min(chunk, n_frames))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lo in range(0, n_frames, chunk):
        dpix = run(lo, min(lo + chunk, n_frames))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": f"config 4: {n_frames} 1920x1080 u8 frames, pyramid from 2x, 5 filters f32; detect and "
                        f"top-10 from one forward pass + backward of summed top-10 scores to pixels, chunks of {chunk}",
            "frames": n_frames, "frames_per_s": round(n_frames / dt, 2), "ms_per_frame": round(1e3 * dt / n_frames, 4),
            "dpix_abs_max_last_chunk": float(dpix.abs().max())}


def separable_leg(hog355, frames, rank, steps, warmup, ksteps, ps):
    """The clip with separable filters (row and column factors, `rank` pairs
    per channel, 5 filters): graph-replayed frames/s and the scoring
    kernel's launch time and roofline."""
    import torch
    from paper_2006_00816_amd import synth
    row, col, b = synth.separable_filters(range(101, 106), rank)
    bank = hog355.FilterBank(torch.from_numpy(b).cuda(), row=torch.from_numpy(row).cuda(),
                             col=torch.from_numpy(col).cuda())
    g = hog355.DetectGraph(frames, bank=bank)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    ws = hog355.Workspace()
    dets, nd = hog355.alloc_dets(CLIP, hog355.MAX_DETS)
    kt = kernel_times(hog355, lambda: hog355.detect_batch_bank_into(frames, bank, dets, nd, ws=ws),
                      ("hist", "feat", "score", "nms_edges", "nms"), ksteps) if ksteps else {}
    # algorithmic work of a separable filter: 10 + 10 multiply-adds per
    # window, channel (31), pair and filter
    lines = rooflines(kt, ps, CLIP, 2.0 * 620 * rank * NF, "hog_sep_score_kernel")
    return {"rank": rank, "fps": round(CLIP * steps / dt, 1), "ms_per_step": round(1e3 * dt / steps, 4),
            "kernels_per_step": kt, "score_roofline": [e for e in lines if e["kernel"] == "hog_sep_score_kernel"]}


def pipeline_leg(frames_np, W, b, batches):
    """The host pipeline (Sec. V-C): 64-frame batches of the clip submitted
    from host memory, detections back to a consumer thread that counts the
    boxes.  frames/s including both PCIe transfers, for frames in pageable
    memory copied straight from there, pageable memory through the
    pipeline's page-locked staging, and page-locked memory copied straight
    from there."""
    import torch
    from paper_2006_00816_amd import hog355
    n = frames_np.shape[0]
    pinned = torch.from_numpy(frames_np).pin_memory()
    out = []
    for name, staging, src in (("pageable, direct", False, frames_np), ("pageable, staged", True, frames_np),
                               ("page-locked, direct", False, pinned)):
        boxes = [0]
        p = hog355.Pipeline(W, b, H, W_PX, n, depth=3, cap=64, consumer_threads=2, staging=staging,
                            consumer=lambda first, d, nd: boxes.__setitem__(0, boxes[0] + int(nd.sum())))
        for i in range(2):
            p.submit(src, i * n)
        p.drain()
        boxes[0] = 0
        t0 = time.perf_counter()
        for i in range(batches):
            p.submit(src, i * n)
        p.drain()
        dt = time.perf_counter() - t0
        p.close()
        fps = batches * n / dt
        out.append({"source": name, "fps": round(fps, 1), "ms_per_batch": round(1e3 * dt / batches, 4),
                    "h2d_gbs": round(fps * H * W_PX / 1e9, 3), "boxes_per_frame": round(boxes[0] / (batches * n), 2)})
    return {"workload": f"{batches} batches of the 64-frame 640x480 clip from host memory, 3 stages, 2 consumer "
                        "threads, 64 detections per frame copied back", "legs": out}


def graph_fps(hog355, frames, Wt, bt, steps, warmup, **kw):
    """Graph-replayed frames/s of the clip under detection options kw."""
    import torch
    g = hog355.DetectGraph(frames, Wt, bt, **kw)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, nd = hog355.dets_to_numpy(g.dets, g.n_dets)
    g.close()
    return CLIP * steps / dt, 1e3 * dt / steps, float(np.mean(nd))


def options_leg(hog355, frames, Wt, bt, tuning, steps, warmup, ksteps):
    """The clip under the options that change which levels and windows run
    and how levels are built: the largest scale skipped (min_face 96, the
    paper's configuration for 640x480 frames with faces of at least 20 %),
    a search region around the face found in the first frame (its box grown
    by 32 px, levels +- 1), and the recursive pyramid.  Graph-replayed
    frames/s and per-kernel times of eager steps."""
    ws = hog355.Workspace()
    dets, nd = hog355.alloc_dets(CLIP, hog355.MAX_DETS)
    regions = first_frame_region(hog355, frames, Wt, bt)
    hog355.tuning_set(H, W_PX, 1 | hog355.CASCADE, CLIP, NF, tuning)
    legs = []
    for name, kw in (("min_face 96 (largest scale skipped)", {"min_face": 96}),
                     ("search region: first-frame face box + 32 px, levels +- 1", {"regions": regions}),
                     ("recursive pyramid", {"upsample": 1 | hog355.CASCADE})):
        fps, ms, kept = graph_fps(hog355, frames, Wt, bt, steps, warmup, **kw)
        run = lambda: hog355.detect_batch_into(frames, Wt, bt, dets, nd, ws=ws, **kw)
        kt = kernel_times(hog355, run, ("geom", "cascade", "hist", "feat", "score", "nms_edges", "nms"),
                          ksteps) if ksteps else {}
        legs.append({"option": name, "fps": round(fps, 1), "ms_per_step": round(ms, 4),
                     "kept_per_frame_mean": round(kept, 2), "kernels_per_step": kt})
    r = regions[0].tolist()
    return {"region": r, "tuning": tuning, "legs": legs}


def tracking_leg(hog355, frames, Wt, bt, n_frames):
    """One frame per call, as the closed-loop eyeblink case needs: plain,
    and with the search region of each frame derived on the device from the
    previous frame's detections (box + 32 px, levels +- 1).  Submit to
    completion latency."""
    import torch
    ws = hog355.Workspace()
    dets, nd = hog355.alloc_dets(1, hog355.MAX_DETS)
    regions = hog355.region_tensor([(0, 0, W_PX, H, 0, hog355.ALL_LEVELS)])
    out = {}
    for name, track in (("plain", False), ("tracked region", True)):
        lat = []
        for i in range(n_frames + 20):
            t1 = time.perf_counter()
            hog355.detect_batch_into(frames[i % CLIP:i % CLIP + 1], Wt, bt, dets, nd, ws=ws,
                                     regions=regions if track else None)
            if track:
                hog355.track_regions(dets, nd, H, W_PX, 32, 1, regions)
            torch.cuda.synchronize()
            if i >= 20:
                lat.append(1e3 * (time.perf_counter() - t1))
        lat = np.array(lat)
        out[name] = {"p50_ms": round(float(np.percentile(lat, 50)), 4),
                     "p99_ms": round(float(np.percentile(lat, 99)), 4), "frames": n_frames}
    return out


def copy_calibration(mib):
    """A plain device-to-device copy of known size, to scale the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of the detector's kernels."""
    import torch
    torch.cuda.set_device(0)
    n = mib << 20
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def first_frame_region(hog355, frames, Wt, bt, margin=32, span=1):
    """Search regions [CLIP][6] for the clip: the best detection of its first
    frame grown by `margin` px, levels +- span (hog_track_regions)."""
    import torch
    dets, nd = hog355.alloc_dets(1, hog355.MAX_DETS)
    hog355.detect_batch_into(frames[:1], Wt, bt, dets, nd)
    regions = torch.zeros((CLIP, 6), dtype=torch.int32, device="cuda")
    hog355.track_regions(dets, nd, H, W_PX, margin, span, regions[:1])
    regions[:] = regions[:1].clone()
    return regions


def option_kwargs(hog355, name, frames, Wt, bt):
    if name == "min_face":
        return {"min_face": 96}
    if name == "region":
        return {"regions": first_frame_region(hog355, frames, Wt, bt)}
    if name == "cascade":
        return {"upsample": 1 | hog355.CASCADE}
    return {}


def batched_leg(hog355, frames, Wt, bt, args, kw=None):
    """The clip replayed from a hipGraph under the schedule the autotuner
    picks (or the one named), with per-kernel HIP-event times of eager
    steps of that schedule."""
    import torch
    staged = {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "split": 1, "nms_rounds": 3,
              "score_rows": 0, "stagger": 0}
    fused = {**staged, "fused": 1}
    tune_ms = None
    if args.schedule == "auto":
        tuning, tune_ms = hog355.autotune(frames, Wt, bt, reps=5)
    else:
        tuning = staged if args.schedule == "staged" else fused
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, tuning)
    torch.cuda.synchronize()

    kw = kw or {}
    if "upsample" in kw:
        hog355.tuning_set(H, W_PX, kw["upsample"], CLIP, NF, tuning)
    g = hog355.DetectGraph(frames, Wt, bt, **kw)
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    lat = []
    for _ in range(min(args.steps, 200)):
        t1 = time.perf_counter()
        g.launch()
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t1))
    lat = np.array(lat)
    _, n_kept = hog355.dets_to_numpy(g.dets, g.n_dets)
    n_ref = g.n_dets.clone()
    g.close()

    # throughput with several clips in flight: one captured graph per input
    # buffer, launched in turn on as many streams, under the schedule timed
    # fastest in that mode
    inflight = None
    if args.schedule == "auto" and args.in_flight != 1 and not kw:
        cands = [{**staged, "split": sp, "nms_rounds": nr, "score_rows": rows}
                 for sp in (1, 2) for nr in (0, 1, 2, 3) for rows in (4, 16)]
        best = None
        for depth in ((2, 3, 4) if args.in_flight == 0 else (args.in_flight,)):
            fl = [frames] + [frames.clone() for _ in range(depth - 1)]
            t, ms = hog355.tune_clip_stream(fl, Wt, bt, cands)
            if best is None or ms < best[2]:
                best = (depth, t, ms, fl)
        depth, t_if, ms_if, fl = best
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, t_if)
        cs = hog355.ClipStream(fl, Wt, bt)
        for _ in range(args.warmup):
            cs.launch()
        cs.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cs.launch()
        cs.synchronize()
        torch.cuda.synchronize()
        dt_if = time.perf_counter() - t0
        same = all(bool(torch.equal(gg.n_dets, n_ref)) for gg in cs.graphs)
        cs.close()
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, tuning)
        inflight = {"clips": depth, "tuning": t_if, "tune_ms": ms_if, "dt": dt_if, "same_counts": same}

    # kernel durations with HIP events on the launch streams, eager steps:
    # of the timed schedule, and of the per-stage schedule with one group
    # (every launch covers all 64 frames, no launch overlaps another), from
    # which the rooflines are taken
    ws = hog355.Workspace()
    dets, nd = hog355.alloc_dets(CLIP, hog355.MAX_DETS)
    ksteps = min(args.steps, args.kernel_steps)
    names = ("geom", "cascade", "hist", "feat", "score", "fused", "nms_edges", "nms")
    run = lambda: hog355.detect_batch_into(frames, Wt, bt, dets, nd, ws=ws, **kw)
    kern = kernel_times(hog355, run, names, ksteps) if ksteps else {}
    u = kw.get("upsample", 1)
    if tuning == staged:
        kern_staged = kern
    else:
        hog355.tuning_set(H, W_PX, u, CLIP, NF, staged)
        kern_staged = kernel_times(hog355, run, names, ksteps) if ksteps else {}
        hog355.tuning_set(H, W_PX, u, CLIP, NF, tuning)
    return {"dt": dt, "lat": lat, "n_kept": n_kept, "tuning": tuning, "tune_ms": tune_ms, "kern": kern,
            "kern_staged": kern_staged, "staged": staged, "ksteps": ksteps, "inflight": inflight}


def f16x3_leg(hog355, frames, Wt, bt, bl, steps, warmup, ksteps, ps):
    """The clip with window scores from split fp16 operands
    (HOG_ARITH_F16X3, an opt-in arithmetic; the headline uses FP32): one
    captured graph under the autotuned schedule, the clips in flight under
    the in-flight schedule, the scoring kernel's HIP-event time on the
    per-stage schedule, and the largest difference of its scores from the
    FP32 scorer's over one frame."""
    import torch
    A = hog355.ARITH_F16X3
    res = {"arith": "f16x3: each product from three fp16 matrix products of split operands "
                    "(hi + 2^-11 lo), FP32 sums"}
    g = hog355.DetectGraph(frames, Wt, bt, arith=A)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, nk = hog355.dets_to_numpy(g.dets, g.n_dets)
    g.close()
    res["fps_one_clip_in_flight"] = round(CLIP * steps / dt, 1)
    res["ms_per_clip_one_in_flight"] = round(1e3 * dt / steps, 4)
    inf = bl["inflight"]
    if inf:
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, inf["tuning"])
        fl = [frames] + [frames.clone() for _ in range(inf["clips"] - 1)]
        cs = hog355.ClipStream(fl, Wt, bt, arith=A)
        for _ in range(warmup):
            cs.launch()
        cs.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            cs.launch()
        cs.synchronize()
        torch.cuda.synchronize()
        dt_if = time.perf_counter() - t0
        cs.close()
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, bl["tuning"])
        res["fps"] = round(CLIP * steps / dt_if, 1)
        res["ms_per_clip"] = round(1e3 * dt_if / steps, 4)
        res["clips_in_flight"] = inf["clips"]
        res["in_flight_tuning"] = inf["tuning"]
    if ksteps:
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, bl["staged"])
        ws = hog355.Workspace()
        dets, nd = hog355.alloc_dets(CLIP, hog355.MAX_DETS)
        kt = kernel_times(hog355, lambda: hog355.detect_batch_into(frames, Wt, bt, dets, nd, ws=ws, arith=A),
                          ("feat", "score"), ksteps)
        hog355.tuning_set(H, W_PX, 1, CLIP, NF, bl["tuning"])
        res["kernels_per_step_staged"] = kt
        if "score" in kt:
            ms = kt["score"]["ms_per_launch"]
            tf = 2.0 * 3100 * NF * ps["windows"] * CLIP / (ms * 1e-3) / 1e12
            res["score_tflops_algorithmic"] = round(tf, 2)
            res["score_frac_of_fp32_matrix_peak"] = round(tf / FP32_PEAK_TFLOPS, 4)
    s0 = hog355.scores(frames[0], Wt, bt)
    s1 = hog355.scores(frames[0], Wt, bt, arith=A)
    torch.cuda.synchronize()
    res["max_abs_score_diff_vs_f32_frame0"] = float(max(float((a[1] - c[1]).abs().max()) for a, c in zip(s0, s1)))
    res["kept_per_frame_mean"] = float(np.mean(nk))
    return res


def plain_leg(hog355, frames, Wt, bt, n_frames, autotune=True):
    """One frame per call, submit to completion, on the clip's frames, under
    the schedule the autotuner picks for one frame (NMS rounds, scoring
    rows)."""
    import torch
    tuning = None
    if autotune:
        tuning, _ = hog355.autotune(frames[:1], Wt, bt, reps=20)
    ws = hog355.Workspace()
    one = frames[0]
    for _ in range(20):
        hog355.detect(one, Wt, bt, ws=ws)
    torch.cuda.synchronize()
    pdets, pnd = hog355.alloc_dets(1, hog355.MAX_DETS)
    plain_lat = []
    t0 = time.perf_counter()
    for i in range(n_frames):
        t1 = time.perf_counter()
        hog355.detect_batch_into(frames[i % CLIP:i % CLIP + 1], Wt, bt, pdets, pnd, ws=ws)
        torch.cuda.synchronize()
        plain_lat.append(1e3 * (time.perf_counter() - t1))
    plain_dt = time.perf_counter() - t0
    plain_lat = np.array(plain_lat)
    # the same frames through a captured one-frame graph (a fixed-size
    # stream): each frame is copied into the graph's bound buffer before its
    # replay, outside the timed interval
    buf = frames[0:1].clone()
    g = hog355.DetectGraph(buf, Wt, bt)
    glat, same = [], True
    for i in range(n_frames + 20):
        buf.copy_(frames[i % CLIP:i % CLIP + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.launch()
        torch.cuda.synchronize()
        if i >= 20:
            glat.append(1e3 * (time.perf_counter() - t1))
        if i == 20:
            hog355.detect_batch_into(buf, Wt, bt, pdets, pnd, ws=ws)
            torch.cuda.synchronize()
            same = bool(torch.equal(g.n_dets, pnd))
    g.close()
    glat = np.array(glat)
    return {"fps": round(n_frames / max(plain_dt, 1e-9), 1),
            "p50_ms": round(float(np.percentile(plain_lat, 50)), 4),
            "p99_ms": round(float(np.percentile(plain_lat, 99)), 4),
            "latency": "one frame per call, submit to completion", "tuning": tuning,
            "graph": {"p50_ms": round(float(np.percentile(glat, 50)), 4),
                      "p99_ms": round(float(np.percentile(glat, 99)), 4),
                      "latency": "one replay of a captured one-frame graph, submit to completion (the frame "
                                 "copied into the graph's buffer before each replay, not timed)",
                      "count_equals_call": same}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--plain-frames", type=int, default=640)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=32)
    ap.add_argument("--kernel-steps", type=int, default=100, help="eager steps timed per kernel (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="seconds of served Poisson stream per rate (0: skip)")
    ap.add_argument("--train-steps", type=int, default=10, help="config-3 training steps timed (0: skip)")
    ap.add_argument("--pixel-grad-frames", type=int, default=256,
                    help="config-4 frames for the pixel-gradient leg (0: skip)")
    ap.add_argument("--schedule", choices=("auto", "staged", "fused"), default="auto",
                    help="auto: run the library's autotuner on the clip first")
    ap.add_argument("--in-flight", type=int, default=0,
                    help="clips in flight for the throughput loop (auto schedule only): 0 picks 2, 3 or 4, 1 is one "
                         "captured graph replayed on one stream")
    ap.add_argument("--separable-rank", type=int, default=1,
                    help="also time the clip with separable filters of this rank (0: skip)")
    ap.add_argument("--option", choices=("none", "min_face", "region", "cascade"), default="none",
                    help="run the batched clip itself under one detection option (for profiling it alone): "
                         "min_face 96, a first-frame face region, or the recursive pyramid")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the level-skipping, search-region, recursive-pyramid and tracking legs")
    ap.add_argument("--pipeline-batches", type=int, default=20,
                    help="64-frame batches through the host pipeline per source (0: skip)")
    ap.add_argument("--no-f16x3", action="store_true",
                    help="skip the leg with split-fp16 window scoring (HOG_ARITH_F16X3)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched clip (autotune, graph replay, kernel timing), e.g. to profile the "
                         "other legs alone; the line then has no value")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run device-to-device copies of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the detector shards by frame with no collective on the "
              "hot path, and multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return

    from paper_2006_00816_amd import synth

    wl = synth.config1(seed=1, n=CLIP)
    # the CPU baseline runs first, before this process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl.frames, wl.W, wl.b, args.cpu_frames)
    if cpu is None and not args.no_cpu_baseline:
        print("bench.py: a profiler is preloaded; the CPU-baseline worker pool is not started", file=sys.stderr)

    import torch
    from paper_2006_00816_amd import hog355

    torch.cuda.set_device(0)
    frames = torch.from_numpy(wl.frames).cuda()
    Wt = torch.from_numpy(wl.W).cuda()
    bt = torch.from_numpy(wl.b).cuda()
    torch.cuda.synchronize()

    ps = pyramid_stats(H, W_PX, NF)
    win = ps["windows"]
    flop_per_frame = 2.0 * 3100 * NF * win
    out = {
        "metric": METRIC,
        "value": None,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64-frame 640x480 u8 clip (config 1), 5 filters 10x10x31 f32, batched hipGraph",
                   "frames_per_step": CLIP, "h": H, "w": W_PX, "filters": NF, "levels": ps["levels"],
                   "windows_per_frame": win, "thresh": 0.0, "iou": 0.5},
    }
    if args.option != "none":
        out["config"]["option"] = args.option
    if not args.no_batched:
        bl = batched_leg(hog355, frames, Wt, bt, args, option_kwargs(hog355, args.option, frames, Wt, bt))
        fps_one = CLIP * args.steps / bl["dt"]
        inf = bl["inflight"]
        dt_main = inf["dt"] if inf else bl["dt"]
        fps = CLIP * args.steps / dt_main
        out["config"]["clips_in_flight"] = inf["clips"] if inf else 1
        lines = rooflines(bl["kern_staged"], ps, CLIP, 2.0 * 3100 * NF, "hog_score_kernel")
        # the dominant kernel: most GPU time per step among the stage kernels
        roofline = max(lines, key=lambda e: e["ms_per_step"]) if lines else None
        # the whole path against the FP32 and HBM rooflines: algorithmic
        # scoring FLOP, and the bytes a frame must cross (frame in,
        # detections out)
        det_bytes = 40.0 * float(np.mean(bl["n_kept"]))
        path = {"fp32_tflops": round(flop_per_frame * fps / 1e12, 3),
                "fp32_frac": round(flop_per_frame * fps / 1e12 / FP32_PEAK_TFLOPS, 4),
                "hbm_gbs": round((H * W_PX + det_bytes) * fps / 1e9, 2),
                "hbm_frac": round((H * W_PX + det_bytes) * fps / 1e9 / HBM_PEAK_GBS, 5)}
        out.update({
            "value": round(fps, 1),
            "ms_per_step": round(1e3 * dt_main / args.steps, 4),
            "batched": {"fps": round(fps, 1), "clips_in_flight": inf["clips"] if inf else 1,
                        "fps_one_clip_in_flight": round(fps_one, 1),
                        "p50_ms": round(float(np.percentile(bl["lat"], 50)), 4),
                        "p99_ms": round(float(np.percentile(bl["lat"], 99)), 4),
                        "latency": "one clip in flight, submit to completion (every frame of the clip)"},
            "schedule": {"tuning": bl["tuning"], "autotune_best_ms": bl["tune_ms"],
                         "in_flight": ({"clips": inf["clips"], "tuning": inf["tuning"],
                                        "tune_ms_per_clip": round(inf["tune_ms"], 4),
                                        "results_equal_one_in_flight": inf["same_counts"]} if inf else None)},
            "kernels_per_step": bl["kern"],
            "kernels_per_step_staged": {"tuning": bl["staged"], "kernels": bl["kern_staged"],
                                        "note": "per-stage schedule, one group: each launch covers all 64 "
                                                "frames and runs alone; the rooflines are taken from these"},
            "kept_per_frame_mean": float(np.mean(bl["n_kept"])),
            "roofline": roofline,
            "roofline_kernels": lines,
            "roofline_path": path,
        })
    if not args.no_batched and not args.no_f16x3 and args.option == "none":
        out["score_f16x3"] = f16x3_leg(hog355, frames, Wt, bt, bl, args.steps, args.warmup,
                                       min(args.steps, args.kernel_steps), ps)
    if args.plain_frames > 0:
        out["plain"] = plain_leg(hog355, frames, Wt, bt, args.plain_frames, autotune=args.schedule == "auto")
    if not args.no_options and not args.no_batched:
        out["options"] = options_leg(hog355, frames, Wt, bt, bl["tuning"], min(args.steps, 200), args.warmup,
                                     min(args.steps, args.kernel_steps))
        out["tracking"] = tracking_leg(hog355, frames, Wt, bt, max(args.plain_frames, 200))
    out["paper_context"] = {"ms_per_frame": 0.333, "hardware": "NVIDIA Titan X (Pascal), 16 images per launch",
                            "end_to_end_ms_per_frame": 0.533}
    ksteps = min(args.steps, args.kernel_steps)
    if args.separable_rank > 0:
        out["separable"] = separable_leg(hog355, frames, args.separable_rank, args.steps, args.warmup, ksteps, ps)
    if args.serve_seconds > 0:
        # served stream: Poisson arrivals, 40/40/20 % 320x240 / 640x480 / 1280x720
        from paper_2006_00816_amd import serve
        pools, Ws, bs = serve.pinned_pools(per_res=64)
        out["served"] = [serve.served_stream(rate, args.serve_seconds, Ws, bs, pools)[0]
                         for rate in (500.0, 2000.0, 8000.0)]
    if args.pipeline_batches > 0:
        out["pipeline"] = pipeline_leg(wl.frames, Wt, bt, args.pipeline_batches)
    if args.train_steps > 0:
        out["train"] = train_leg(args.train_steps)
    if args.pixel_grad_frames > 0:
        out["pixel_grad"] = pixel_grad_leg(args.pixel_grad_frames, 32)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
