"""Window scores from split fp16 operands (HOG_ARITH_F16X3) against the
float64 oracle, at the same tolerances as the FP32 scorer (1e-5 relative +
2e-5 absolute), and detection with it: the GPU NMS equals the oracle's NMS
over the split-fp16 candidates, and the end-to-end kept set is the
oracle's apart from near-threshold windows and near ties."""
import numpy as np
import pytest
import torch

from oracle import hog as oracle
from paper_2006_00816_amd import synth
from test_gpu_batch import _same
from test_gpu_parity import (BOX, H, assert_end_to_end, case_frame, cand_key, close, cu,  # noqa: F401
                             det_key)

pytestmark = pytest.mark.gpu


def _cands(H, frame, Wn, bn, u, thresh=0.0):
    """Candidates from the split-fp16 dense scores, with their float32
    scores."""
    rows = []
    levels = oracle.pyramid(*frame.shape, u)
    for glv, gS in H.scores(cu(frame), cu(Wn), cu(bn), u, arith=H.ARITH_F16X3):
        s = gS.cpu().numpy()
        f, r, c = np.nonzero(s > np.float32(thresh))
        lv = levels[glv["k"]]
        a = np.empty(len(f), oracle.CAND_DTYPE)
        x0, y0, x1, y1 = oracle.window_box(lv, r, c)
        a["score"], a["f"], a["k"], a["r"], a["c"] = s[f, r, c].astype(np.float64), f, lv.k, r, c
        a["x0"], a["y0"], a["x1"], a["y1"] = x0, y0, x1, y1
        rows.append(a)
    return np.concatenate(rows) if rows else np.empty(0, oracle.CAND_DTYPE)


def _assert_nms(H, frame, Wn, bn, u, dets, n):
    cg = _cands(H, frame, Wn, bn, u)
    kept = oracle.nms(cg, 0.5)
    assert n == len(kept), (n, len(kept))
    m = min(len(dets), len(kept))
    assert len(dets) == m
    assert det_key(dets) == cand_key(kept[:m])
    assert np.array_equal(dets["score"], kept["score"][:m].astype(np.float32))
    for f in BOX:
        assert np.array_equal(dets[f], kept[f][:m]), f
    return cg


@pytest.mark.parametrize("name,nf", [("c0", 1), ("c1", 5), ("ragged", 5), ("tall", 3), ("u2", 7),
                                     ("exact80", 5), ("c0", 12), ("c1", 4), ("c1", 2)])
def test_scores_f16x3_parity(H, name, nf):
    frame, u = case_frame(name)
    Wn, bn = synth.filters(range(300, 300 + nf))
    print(f"f16x3 scores {name} nf={nf}", flush=True)
    got = H.scores(cu(frame), cu(Wn), cu(bn), u, arith=H.ARITH_F16X3)
    want = []
    oracle.candidates(frame, Wn, bn, 0.0, u, levels_out=want)
    assert len(got) == len(want)
    for (glv, gS), (olv, oS) in zip(got, want):
        ok, err, nbad = close(gS.cpu().numpy(), oS)
        assert ok, (name, nf, olv.k, err, nbad)


@pytest.mark.parametrize("scale", [2.0 ** 12, 2.0 ** -14])
def test_scores_f16x3_weight_range(H, scale):
    """Weights scaled by 2^12 (up to about 2^11, far from the fp16 limit of
    2^15) and by 2^-14 (fp16 subnormals in the high parts): the scores stay
    within the tolerance scaled alike."""
    frame, u = case_frame("c1")
    Wn, bn = synth.filters(range(310, 315))
    Ws = (Wn.astype(np.float64) * scale).astype(np.float32)
    bs = (bn.astype(np.float64) * scale).astype(np.float32)
    print(f"f16x3 weight scale {scale}", flush=True)
    got = H.scores(cu(frame), cu(Ws), cu(bs), u, arith=H.ARITH_F16X3)
    want = []
    oracle.candidates(frame, Ws, bs, 0.0, u, levels_out=want)
    for (glv, gS), (olv, oS) in zip(got, want):
        g = gS.cpu().numpy().astype(np.float64) / scale
        ok, err, nbad = close(g, oS / scale)
        assert ok, (scale, olv.k, err, nbad)


@pytest.mark.parametrize("name,nf", [("c0", 1), ("c1", 5), ("ragged", 5), ("tall", 2), ("u2", 5),
                                     ("exact80", 5), ("c1", 7)])
def test_detect_f16x3_parity(H, name, nf):
    # the cases of the FP32 detection parity test
    frame, u = case_frame(name)
    Wn, bn = synth.filters(range(100, 100 + nf))
    print(f"f16x3 detect {name} nf={nf}", flush=True)
    dets, nd = H.detect_batch(cu(frame[None]), cu(Wn), cu(bn), 0.0, 0.5, u, arith=H.ARITH_F16X3)
    cg = _assert_nms(H, frame, Wn, bn, u, dets[0], int(nd[0]))
    st = assert_end_to_end(frame, Wn, bn, u, cg, dets[0], int(nd[0]), f"f16x3 detect {name} nf={nf}")
    print(st, flush=True)


def test_clip_64_f16x3_batch_graph_and_sampled_frames(H):
    """The 64-frame 640x480 clip with split-fp16 scoring: the batch gives
    each frame the detections of that frame alone (frame index aside), a
    replayed graph gives the batch's, and two sampled frames pass the NMS
    and end-to-end checks against the oracle."""
    wl = synth.config1(seed=1, n=64)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    print("f16x3 64-frame clip", flush=True)
    ref, nref = H.detect_batch(fr, W, b, arith=H.ARITH_F16X3)
    g = H.DetectGraph(fr, W, b, arith=H.ARITH_F16X3)
    try:
        for _ in range(2):
            g.launch()
            torch.cuda.synchronize()
            got, n = H.dets_to_numpy(g.dets, g.n_dets)
            assert np.array_equal(n, nref)
            for i in range(64):
                assert _same(got[i], ref[i]), i
    finally:
        g.close()
    for i in (0, 37):
        one, n1 = H.detect_batch(fr[i:i + 1], W, b, arith=H.ARITH_F16X3)
        a, c = one[0].copy(), ref[i].copy()
        c["frame"] = 0
        assert int(n1[0]) == int(nref[i]) and _same(a, c), i
        cg = _assert_nms(H, wl.frames[i], wl.W, wl.b, 1, ref[i], int(nref[i]))
        assert_end_to_end(wl.frames[i], wl.W, wl.b, 1, cg, ref[i], int(nref[i]), f"f16x3 clip frame {i}")


@pytest.mark.parametrize("split,rounds,rows", [(2, 3, 16), (1, 0, 4), (4, 8, 16)])
def test_f16x3_schedules_equal(H, split, rounds, rows):
    """Split-fp16 scoring under other per-stage schedules (frame groups on
    forked streams, NMS rounds, scoring rows per item): the same detections
    in every field as the single-group schedule; a request for the fused
    schedule runs the per-stage one."""
    wl = synth.config1(seed=27, n=12)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    base = {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "stagger": 0, "split": 1,
            "nms_rounds": 3, "score_rows": 16}
    print(f"f16x3 split={split} rounds={rounds} rows={rows}", flush=True)
    out = []
    for t in (base, {**base, "split": split, "nms_rounds": rounds, "score_rows": rows}, {**base, "fused": 1}):
        H.tuning_set(480, 640, 1, 12, 5, t)
        try:
            out.append(H.detect_batch(fr, W, b, arith=H.ARITH_F16X3))
        finally:
            H.tuning_set(480, 640, 1, 12, 5, None)
    (ref, nref) = out[0]
    for got, n in out[1:]:
        assert np.array_equal(n, nref)
        for i in range(12):
            assert _same(got[i], ref[i]), i


def test_f16x3_clips_in_flight(H):
    """Three clips in flight with split-fp16 scoring: every graph gives the
    detections of detect_batch on its own buffer."""
    clips = [synth.config1(seed=50 + k, n=4) for k in range(3)]
    W, b = cu(clips[0].W), cu(clips[0].b)
    frames = [cu(c.frames) for c in clips]
    refs = [H.detect_batch(f, W, b, arith=H.ARITH_F16X3) for f in frames]
    print("f16x3: 3 clips in flight", flush=True)
    cs = H.ClipStream(frames, W, b, arith=H.ARITH_F16X3)
    try:
        for _ in range(7):
            cs.launch()
        cs.synchronize()
        torch.cuda.synchronize()
        for g, (ref, nref) in zip(cs.graphs, refs):
            got, n = H.dets_to_numpy(g.dets, g.n_dets)
            assert np.array_equal(n, nref)
            for i in range(len(ref)):
                assert _same(got[i], ref[i]), i
    finally:
        cs.close()


@pytest.mark.parametrize("n,nf", [(2, 5), (3, 7)])
def test_f16x3_regions_and_min_face(H, n, nf):
    """Split-fp16 scoring with per-frame search regions (rows and tiles
    narrowed per window row) and with the largest scale skipped: the GPU
    NMS equals the oracle's over the split-fp16 candidates under the same
    mask, and the end-to-end decisions are the oracle's outside near ties."""
    from test_gpu_region import REGIONS, check_frame
    wl = synth.config1(seed=60 + n, n=n)
    Wn, bn = synth.filters(range(210, 210 + nf))
    names = ["box", "box_levels", "corner"][:n]
    regs = [REGIONS[k](wl.frames[0].shape) for k in names]
    dets, nd = H.detect_batch(cu(wl.frames), cu(Wn), cu(bn), regions=H.region_tensor(regs), arith=H.ARITH_F16X3)
    for i in range(n):
        print(f"f16x3 region {names[i]} n={n} nf={nf}: {nd[i]} kept", flush=True)
        check_frame(H, wl.frames[i], Wn, bn, 1, dets[i], int(nd[i]), region=regs[i], label=f"f16x3 {names[i]}",
                    arith=H.ARITH_F16X3)
    dets, nd = H.detect_batch(cu(wl.frames), cu(Wn), cu(bn), min_face=96, arith=H.ARITH_F16X3)
    for i in range(n):
        assert np.all(dets[i]["level"] >= 1)
        check_frame(H, wl.frames[i], Wn, bn, 1, dets[i], int(nd[i]), min_face=96, label=f"f16x3 mf96 {i}",
                    arith=H.ARITH_F16X3)
