"""Level skipping and search regions on the GPU against the oracle.

Sec. V-A ("image sequence with constant size") skips the pyramid scales on
which no face of the minimum size can appear; Sec. VII proposes limiting
the scales and locations searched per frame from the previous frame.  The
oracle applies the same level rule (face_levels) and region test
(window_in_region) to its windows; the GPU detections must equal the
oracle's NMS over the GPU's own candidates under that mask, bit for bit,
and the oracle's end-to-end decisions outside near ties.
"""
import numpy as np
import pytest
import torch

import nms_exclusion
from oracle import hog as oracle
from paper_2006_00816_amd import synth
from test_gpu_parity import BOX, H, NEAR, cand_key, cu, det_key, gpu_candidates  # noqa: F401

pytestmark = pytest.mark.gpu


def _same(a, b):
    return len(a) == len(b) and all(np.array_equal(a[f].view(np.int32), b[f].view(np.int32)) for f in a.dtype.names)


def masked(cands, frame_shape, u, min_face=0, region=None):
    """The candidates a detection with this mask may consider."""
    levels = oracle.pyramid(*frame_shape, u)
    keep_k = set(l.k for l in oracle.face_levels(levels, min_face))
    ok = np.array([c["k"] in keep_k for c in cands], bool)
    if region is not None and len(cands):
        for l in levels:
            sel = cands["k"] == l.k
            if np.any(sel):
                ok[sel] &= oracle.window_in_region(l, cands["r"][sel], cands["c"][sel], region)
    return cands[ok]


def check_frame(Hm, frame, Wn, bn, u, dets, n, min_face=0, region=None, label="", arith=None):
    cg = masked(gpu_candidates(Hm, frame, Wn, bn, u, arith=arith), frame.shape, u, min_face, region)
    kept = oracle.nms(cg, 0.5)
    assert n == len(kept) == len(dets), (label, n, len(kept), len(dets))
    assert det_key(dets) == cand_key(kept), label
    assert np.array_equal(dets["score"], kept["score"].astype(np.float32)), label
    for f in BOX:
        assert np.array_equal(dets[f], kept[f]), (label, f)
    # end to end against the oracle's own scores, near ties excluded
    co = oracle.candidates(frame, Wn, bn, 0.0, u, min_face=min_face, region=region)
    near = set(k for k, s in zip(cand_key(co), co["score"]) if abs(s) < NEAR)
    gnear = set(k for k, s in zip(cand_key(cg), cg["score"]) if abs(s) < NEAR)
    assert set(cand_key(co)) - near - gnear == set(cand_key(cg)) - near - gnear, label
    st = nms_exclusion.check_kept(frame, Wn, bn, u, dets, 0.0, 0.5, NEAR, cand_gpu=cg, min_face=min_face,
                                  region=region)
    assert st["unknown"] <= max(32, 3 * st["windows"] // 100), (label, st)
    return st


def test_min_face_skips_the_largest_scale(H):
    """640x480 frames with faces of at least 20 % of the image (96 px):
    level 0 is not analysed (Sec. V-A worked example)."""
    wl = synth.config1(seed=31, n=2)
    fr = cu(wl.frames)
    dets, nd = H.detect_batch(fr, cu(wl.W), cu(wl.b), min_face=96)
    for i in range(2):
        print(f"min_face 96 frame {i}: {nd[i]} kept", flush=True)
        assert nd[i] > 0 and np.all(dets[i]["level"] >= 1) and np.all(dets[i]["frame"] == i)
        check_frame(H, wl.frames[i], wl.W, wl.b, 1, dets[i], int(nd[i]), min_face=96, label=f"mf96 {i}")


@pytest.mark.parametrize("min_face,u", [(81, 1), (200, 1), (41, 2), (5000, 1)])
def test_min_face_other_bounds(H, min_face, u):
    gen = synth.ClipGenerator(32, 240, 320, face_h=100.0)
    frame = gen.frame()
    Wn, bn = synth.filters(range(101, 106))
    dets, nd = H.detect_batch(cu(frame[None]), cu(Wn), cu(bn), upsample=u, min_face=min_face)
    kept_levels = [l.k for l in oracle.face_levels(oracle.pyramid(240, 320, u), min_face)]
    print(f"min_face {min_face} u={u}: levels {kept_levels}, {nd[0]} kept", flush=True)
    if not kept_levels:
        assert nd[0] == 0 and len(dets[0]) == 0
        return
    assert np.all(np.isin(dets[0]["level"], kept_levels))
    check_frame(H, frame, Wn, bn, u, dets[0], int(nd[0]), min_face=min_face, label=f"mf{min_face}")


def _face_region(frame_shape, seed):
    rng = np.random.default_rng(seed)
    h, w = frame_shape
    x0, y0 = int(rng.integers(0, w // 3)), int(rng.integers(0, h // 3))
    return (x0, y0, x0 + int(rng.integers(w // 3, 2 * w // 3)), y0 + int(rng.integers(h // 3, 2 * h // 3)), 0,
            oracle.HUGE_LEVEL)


REGIONS = {
    "box": lambda s: _face_region(s, 1),
    "levels": lambda s: (0, 0, s[1], s[0], 2, 4),
    "box_levels": lambda s: (50, 30, s[1] - 40, s[0] - 20, 1, 3),
    "corner": lambda s: (0, 0, 100, 96, 0, oracle.HUGE_LEVEL),
    "empty": lambda s: (200, 200, 150, 300, 0, oracle.HUGE_LEVEL),
    "outside": lambda s: (-1000, -1000, 5000, 5000, -3, oracle.HUGE_LEVEL),
}


@pytest.mark.parametrize("n,nf", [(2, 5), (1, 5), (3, 7), (2, 1)])
def test_region_parity(H, n, nf):
    """Every frame of a batch with its own region: one region per kind
    (box, level range, both, corner, empty, wider than the frame), over
    small and large batches (score rows split in halves at n = 1) and one
    or two filter groups (keys stored or merged by atomic max)."""
    wl = synth.config1(seed=33 + n, n=n)
    Wn, bn = synth.filters(range(200, 200 + nf))
    kinds = list(REGIONS)
    for rep in range(0, len(kinds), n):
        names = [kinds[(rep + i) % len(kinds)] for i in range(n)]
        regs = [REGIONS[k](wl.frames[0].shape) for k in names]
        rt = H.region_tensor(regs)
        dets, nd = H.detect_batch(cu(wl.frames), cu(Wn), cu(bn), regions=rt)
        for i in range(n):
            print(f"region {names[i]} {regs[i]} n={n} nf={nf}: {nd[i]} kept", flush=True)
            if names[i] == "empty":
                assert nd[i] == 0
            check_frame(H, wl.frames[i], Wn, bn, 1, dets[i], int(nd[i]), region=regs[i],
                        label=f"{names[i]} n={n} nf={nf}")


def test_region_whole_frame_and_batch_invariance(H):
    """The whole-frame region gives the detections of no region, and a
    frame's result with a region is the same alone and in a batch, bit for
    bit."""
    wl = synth.config1(seed=41, n=3)
    W, b = cu(wl.W), cu(wl.b)
    fr = cu(wl.frames)
    plain, pn = H.detect_batch(fr, W, b)
    whole = H.region_tensor([(0, 0, 640, 480, 0, H.ALL_LEVELS)] * 3)
    got, gn = H.detect_batch(fr, W, b, regions=whole)
    assert np.array_equal(pn, gn) and all(_same(plain[i], got[i]) for i in range(3))
    regs = [REGIONS["box"]((480, 640)), REGIONS["box_levels"]((480, 640)), REGIONS["levels"]((480, 640))]
    batch, bnd = H.detect_batch(fr, W, b, regions=H.region_tensor(regs))
    for i in range(3):
        one, on = H.detect_batch(fr[i:i + 1], W, b, regions=H.region_tensor(regs[i:i + 1]))
        d = one[0].copy()
        d["frame"] = i
        assert on[0] == bnd[i] and _same(d, batch[i]), i


def test_region_split_schedule(H):
    """Regions under a split schedule (frame groups on forked streams): the
    same detections as the default schedule."""
    wl = synth.config1(seed=42, n=4)
    W, b = cu(wl.W), cu(wl.b)
    fr = cu(wl.frames)
    regs = H.region_tensor([REGIONS[k]((480, 640)) for k in ("box", "levels", "corner", "box_levels")])
    a, an = H.detect_batch(fr, W, b, regions=regs)
    H.lib().hog_init()
    H.tuning_set(480, 640, 1, 4, 5, {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2,
                                     "split": 2, "nms_rounds": 4, "score_rows": 16})
    try:
        c, cn = H.detect_batch(fr, W, b, regions=regs)
    finally:
        H.tuning_set(480, 640, 1, 4, 5, None)
    assert np.array_equal(an, cn) and all(_same(a[i], c[i]) for i in range(4))


def test_track_regions_kernel(H):
    """hog_track_regions against the oracle's track_region, frame by frame,
    including frames without detections and a frame with an error count."""
    rng = np.random.default_rng(5)
    n, cap, h, w = 6, 8, 480, 640
    d = np.zeros((n, cap, 10), np.int32)
    counts = np.array([3, 0, 1, 8, -7, 2], np.int32)
    for i in range(n):
        for j in range(cap):
            x0, y0 = int(rng.integers(-5, w - 50)), int(rng.integers(-5, h - 50))
            s = int(rng.integers(80, 300))
            d[i, j] = [i, 0, int(rng.integers(0, 10)), 0, 0, x0, y0, x0 + s, y0 + s, 0]
    dt, nt = cu(d), cu(counts)
    regs = torch.zeros((n, 6), dtype=torch.int32, device="cuda")
    for margin, span in ((16, 1), (0, 0), (40, 3)):
        H.track_regions(dt, nt, h, w, margin, span, regs)
        got = regs.cpu().numpy()
        dets, _ = H.dets_to_numpy(dt, nt.clamp(min=0))
        for i in range(n):
            kept = np.zeros(max(int(counts[i]), 0), oracle.CAND_DTYPE)
            if len(kept):
                dd = dets[i]
                kept["x0"], kept["y0"], kept["x1"], kept["y1"], kept["k"] = (dd["x0"], dd["y0"], dd["x1"], dd["y1"],
                                                                            dd["level"])
            assert tuple(got[i]) == oracle.track_region(kept, h, w, margin, span), (i, margin, span)


def test_tracking_sequence_and_graph(H):
    """A detect -> track -> detect loop over clip frames, one frame per call,
    with the regions kept on the device: each frame's region is the oracle's
    track_region of the previous frame's GPU detections, and each frame's
    detections match the oracle under that region.  The same loop replayed
    from a captured graph (frame and region buffers refreshed in place)
    gives the same detections bit for bit."""
    wl = synth.config1(seed=43, n=6)
    W, b = cu(wl.W), cu(wl.b)
    margin, span = 24, 1
    regs = H.region_tensor([(0, 0, 640, 480, 0, H.ALL_LEVELS)])
    dets, nd = H.alloc_dets(1, H.MAX_DETS)
    prev = None
    eager = []
    for t in range(len(wl.frames)):
        want_reg = (0, 0, 640, 480, 0, oracle.HUGE_LEVEL) if prev is None else prev
        assert tuple(regs.cpu().numpy()[0]) == want_reg, t
        H.detect_batch_into(cu(wl.frames[t:t + 1]), W, b, dets, nd, regions=regs)
        d, n = H.dets_to_numpy(dets, nd)
        eager.append(d[0].copy())
        print(f"track frame {t}: region {want_reg}, {n[0]} kept", flush=True)
        if t < 3:
            check_frame(H, wl.frames[t], wl.W, wl.b, 1, d[0], int(n[0]), region=want_reg, label=f"track {t}")
        kept = np.zeros(len(d[0]), oracle.CAND_DTYPE)
        kept["x0"], kept["y0"], kept["x1"], kept["y1"], kept["k"] = (d[0]["x0"], d[0]["y0"], d[0]["x1"], d[0]["y1"],
                                                                    d[0]["level"])
        prev = oracle.track_region(kept, 480, 640, margin, span)
        H.track_regions(dets, nd, 480, 640, margin, span, regs)
    # the same loop from a graph: detect captured once, track enqueued after
    # each replay on the graph's stream
    frame_buf = cu(wl.frames[0:1]).clone()
    regs.copy_(H.region_tensor([(0, 0, 640, 480, 0, H.ALL_LEVELS)]))
    g = H.DetectGraph(frame_buf, W, b, cap=H.MAX_DETS, regions=regs)
    try:
        for t in range(len(wl.frames)):
            frame_buf.copy_(cu(wl.frames[t:t + 1]))
            torch.cuda.synchronize()
            g.launch()
            H.track_regions(g.dets, g.n_dets, 480, 640, margin, span, regs)
            torch.cuda.synchronize()
            d, n = H.dets_to_numpy(g.dets, g.n_dets)
            assert _same(d[0], eager[t]), t
    finally:
        g.close()
