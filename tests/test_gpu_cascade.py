"""The recursive pyramid (HOG_PYRAMID_CASCADE; Sec. V-A, image-scaling
kernel: each scaled image is computed from the one a scale higher) on the
GPU against the oracle's cascade_levels: every level image bit for bit,
orientation bins bit for bit, histograms, features and scores within the
float32 tolerance, and detections as the oracle's NMS over the GPU's
candidates (bit for bit) and end to end outside near ties."""
import numpy as np
import pytest

import nms_exclusion
from oracle import hog as oracle
from paper_2006_00816_amd import synth
from test_gpu_parity import BOX, NEAR, H, cand_key, case_frame, close, cu, det_key  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = ["c0", "c1", "ragged", "u2", "exact80"]


@pytest.mark.parametrize("name", CASES)
def test_cascade_levels_bins_hist(H, name):
    frame, u = case_frame(name)
    fr = cu(frame)
    want = oracle.cascade_levels(frame, u)
    got = H.pyramid(*frame.shape, u | H.CASCADE)
    print(f"cascade {name}: {frame.shape} u={u}, {len(want)} levels", flush=True)
    assert [(l["h"], l["w"]) for l in got] == [(lv.h, lv.w) for lv, _ in want]
    for lv, L in want:
        px, bins, hist = H.level_maps(fr, lv.k, u | H.CASCADE)
        assert np.array_equal(px.cpu().numpy().astype(np.float64), L), (name, lv.k)
        gx, gy = oracle.gradients(L)
        ob = np.where((gx != 0) | (gy != 0), oracle.orientation_bins(gx, gy), 0)
        assert np.array_equal(bins.cpu().numpy(), ob.astype(np.uint8)), (name, lv.k)
        ok, err, nbad = close(hist.cpu().numpy(), oracle.cell_histograms(L))
        assert ok, (name, lv.k, err, nbad)


@pytest.mark.parametrize("name,nf", [("c0", 1), ("c1", 5), ("ragged", 5), ("u2", 7)])
def test_cascade_features_and_scores(H, name, nf):
    frame, u = case_frame(name)
    gotF = H.features(cu(frame), u | H.CASCADE)
    for (glv, gF), (lv, L) in zip(gotF, oracle.cascade_levels(frame, u)):
        ok, err, nbad = close(gF.cpu().numpy(), oracle.features_from_hist(oracle.cell_histograms(L)))
        assert ok, (name, lv.k, err, nbad)
    Wn, bn = synth.filters(range(300, 300 + nf))
    got = H.scores(cu(frame), cu(Wn), cu(bn), u | H.CASCADE)
    want = []
    oracle.candidates(frame, Wn, bn, 0.0, u, levels_out=want, cascade=True)
    assert len(got) == len(want)
    for (glv, gS), (olv, oS) in zip(got, want):
        ok, err, nbad = close(gS.cpu().numpy(), oS)
        assert ok, (name, nf, olv.k, err, nbad)


def _gpu_cands(H, frame, Wn, bn, u):
    levels = oracle.pyramid_cascade(*frame.shape, u)
    rows = []
    for glv, gS in H.scores(cu(frame), cu(Wn), cu(bn), u | H.CASCADE):
        s = gS.cpu().numpy()
        f, r, c = np.nonzero(s > np.float32(0.0))
        lv = levels[glv["k"]]
        a = np.empty(len(f), oracle.CAND_DTYPE)
        a["score"], a["f"], a["k"], a["r"], a["c"] = s[f, r, c].astype(np.float64), f, lv.k, r, c
        a["x0"], a["y0"], a["x1"], a["y1"] = oracle.window_box(lv, r, c)
        rows.append(a)
    return np.concatenate(rows) if rows else np.empty(0, oracle.CAND_DTYPE)


@pytest.mark.parametrize("name,nf,min_face", [("c0", 1, 0), ("c1", 5, 0), ("u2", 5, 0), ("c1", 5, 130)])
def test_cascade_detect(H, name, nf, min_face):
    """Detections on the recursive pyramid, also with skipped levels (whose
    images the later levels are still computed from)."""
    frame, u = case_frame(name)
    Wn, bn = synth.filters(range(100, 100 + nf))
    dets, nd = H.detect_batch(cu(frame[None]), cu(Wn), cu(bn), upsample=u | H.CASCADE, min_face=min_face)
    dets, n = dets[0], int(nd[0])
    print(f"cascade detect {name} nf={nf} min_face={min_face}: {n} kept", flush=True)
    keep_k = set(l.k for l in oracle.face_levels(oracle.pyramid_cascade(*frame.shape, u), min_face))
    cg = _gpu_cands(H, frame, Wn, bn, u)
    cg = cg[np.isin(cg["k"], list(keep_k))]
    kept = oracle.nms(cg, 0.5)
    assert n == len(kept) == len(dets)
    assert det_key(dets) == cand_key(kept)
    assert np.array_equal(dets["score"], kept["score"].astype(np.float32))
    for f in BOX:
        assert np.array_equal(dets[f], kept[f]), f
    co = oracle.candidates(frame, Wn, bn, 0.0, u, min_face=min_face, cascade=True)
    near = set(k for k, s in zip(cand_key(co), co["score"]) if abs(s) < NEAR)
    gnear = set(k for k, s in zip(cand_key(cg), cg["score"]) if abs(s) < NEAR)
    assert set(cand_key(co)) - near - gnear == set(cand_key(cg)) - near - gnear


def test_cascade_batch_equals_single_and_rejects_backward(H):
    wl = synth.config1(seed=61, n=3)
    W, b = cu(wl.W), cu(wl.b)
    fr = cu(wl.frames)
    batch, bn = H.detect_batch(fr, W, b, upsample=1 | H.CASCADE)
    for i in range(3):
        one, on = H.detect_batch(fr[i:i + 1], W, b, upsample=1 | H.CASCADE)
        d = one[0].copy()
        d["frame"] = i
        assert on[0] == bn[i]
        assert all(np.array_equal(d[f].view(np.int32), batch[i][f].view(np.int32)) for f in d.dtype.names)
    win = H.windows_tensor([0], 0, 0, 0, 0)
    with pytest.raises(H.HogError, match="not implemented"):
        H.filter_backward(fr[:1], W, win, cu(np.ones(1, np.float32)), upsample=1 | H.CASCADE)
