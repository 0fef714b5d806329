"""Parity of the HIP path (through the C ABI) with the float64 oracle.

Bars: pyramid levels, orientation bins, candidate windows and NMS output
bit-exact; histograms, features and scores within 1e-5 relative + 2e-5
absolute.  Windows whose oracle score lies within 1e-4 of the threshold,
or of a tie with an overlapping candidate, are excluded from the
end-to-end detection comparison.
"""
import json
import os

import numpy as np
import pytest
import torch

import nms_exclusion
from oracle import hog as oracle
from paper_2006_00816_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 2e-5
NEAR = 1e-4


@pytest.fixture(scope="module")
def H():
    from paper_2006_00816_amd import hog355
    hog355.lib()
    return hog355


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _face_frame(seed, h, w, face):
    rng = np.random.default_rng(seed)
    img = synth.background(rng, h, w)
    synth.paint_face(img, h / 2, w / 2, face, 205.0)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def case_frame(name):
    if name == "c0":
        return synth.config0(0).frames[0], 1
    if name == "c1":
        return synth.ClipGenerator(1).frame(), 1
    if name == "ragged":
        return _face_frame(7, 97, 131, 70), 1
    if name == "tall":
        return _face_frame(8, 263, 85, 60), 1
    if name == "u2":
        return _face_frame(9, 100, 124, 60), 2
    if name == "exact80":
        return _face_frame(10, 80, 80, 60), 1
    raise KeyError(name)


CASES = ["c0", "c1", "ragged", "tall", "u2", "exact80"]


def close(got, want):
    got = np.asarray(got, np.float64)
    err = np.abs(got - want)
    bad = err > ATOL + RTOL * np.abs(want)
    return (not bad.any()), float(err.max()) if err.size else 0.0, int(bad.sum())


# ------------------------------------------------------------ orientation
def _near_boundary(rng, n):
    out = []
    for deg in (10, 30, 50, 70):
        for quad in range(4):
            a = np.deg2rad(deg + 90 * quad)
            N = rng.integers(1 << 18, 1 << 23, n)
            gx = np.rint(N * np.cos(a)).astype(np.int64) + rng.integers(-1, 2, n)
            gy = np.rint(N * np.sin(a)).astype(np.int64) + rng.integers(-1, 2, n)
            out.append((gx, gy))
            # mirrored angles (180 - a)
            out.append((-gx, gy))
    gx = np.concatenate([o[0] for o in out])
    gy = np.concatenate([o[1] for o in out])
    return gx, gy


def test_orientation_bins_bit_exact(H):
    v = np.arange(-255, 256, dtype=np.int64) << 16
    gx, gy = np.meshgrid(v, v, indexing="ij")
    rng = np.random.default_rng(77)
    rx = rng.integers(-(1 << 24) + 1, 1 << 24, 1_000_000)
    ry = rng.integers(-(1 << 24) + 1, 1 << 24, 1_000_000)
    bx, by = _near_boundary(rng, 20000)
    small = np.arange(-40, 41, dtype=np.int64)
    sx, sy = np.meshgrid(small, small, indexing="ij")
    GX = np.concatenate([gx.ravel(), rx, bx, sx.ravel()]).astype(np.int32)
    GY = np.concatenate([gy.ravel(), ry, by, sy.ravel()]).astype(np.int32)
    print(f"orientation: {GX.size} gradients", flush=True)
    got = H.orient_bins(cu(GX), cu(GY)).cpu().numpy()
    want = oracle.orientation_bins(GX.astype(np.float64) * 2.0 ** -16, GY.astype(np.float64) * 2.0 ** -16)
    assert np.array_equal(got, want.astype(np.uint8)), int((got != want).sum())


# ------------------------------------------------------------- per level
@pytest.mark.parametrize("name", CASES)
def test_levels_bins_hist_bit_exact(H, name):
    frame, u = case_frame(name)
    fr = cu(frame)
    levels = oracle.pyramid(*frame.shape, u)
    print(f"{name}: {frame.shape} u={u}, {len(levels)} levels", flush=True)
    assert [(l["h"], l["w"]) for l in H.pyramid(*frame.shape, u)] == [(l.h, l.w) for l in levels]
    for lv in levels:
        px, bins, hist = H.level_maps(fr, lv.k, u)
        L = oracle.resample(frame, lv)
        assert np.array_equal(px.cpu().numpy().astype(np.float64), L), (name, lv.k)
        gx, gy = oracle.gradients(L)
        ob = np.where((gx != 0) | (gy != 0), oracle.orientation_bins(gx, gy), 0)
        assert np.array_equal(bins.cpu().numpy(), ob.astype(np.uint8)), (name, lv.k)
        ok, err, nbad = close(hist.cpu().numpy(), oracle.cell_histograms(L))
        assert ok, (name, lv.k, err, nbad)


@pytest.mark.parametrize("name", CASES)
def test_features_parity(H, name):
    frame, u = case_frame(name)
    got = H.features(cu(frame), u)
    want = oracle.pyramid_features(frame, u)
    assert len(got) == len(want)
    for (glv, gF), (olv, oF) in zip(got, want):
        ok, err, nbad = close(gF.cpu().numpy(), oF)
        assert ok, (name, olv.k, err, nbad)


@pytest.mark.parametrize("name,nf", [("c0", 1), ("c1", 5), ("ragged", 5), ("tall", 3), ("u2", 7),
                                     ("exact80", 5), ("c0", 12)])
def test_scores_parity(H, name, nf):
    frame, u = case_frame(name)
    Wn, bn = synth.filters(range(300, 300 + nf))
    got = H.scores(cu(frame), cu(Wn), cu(bn), u)
    want = []
    oracle.candidates(frame, Wn, bn, 0.0, u, levels_out=want)
    assert len(got) == len(want)
    for (glv, gS), (olv, oS) in zip(got, want):
        ok, err, nbad = close(gS.cpu().numpy(), oS)
        assert ok, (name, nf, olv.k, err, nbad)


# -------------------------------------------------------------- detection
def gpu_candidates(H, frame, Wn, bn, u, thresh=0.0, arith=None):
    """Candidates from the GPU dense scores, with the GPU's float32 scores
    (arith: the scoring arithmetic, as hog_scores_arith; None: hog_scores)."""
    rows = []
    levels = oracle.pyramid(*frame.shape, u)
    for (glv, gS) in H.scores(cu(frame), cu(Wn), cu(bn), u, arith=arith):
        s = gS.cpu().numpy()
        f, r, c = np.nonzero(s > np.float32(thresh))
        lv = levels[glv["k"]]
        a = np.empty(len(f), oracle.CAND_DTYPE)
        x0, y0, x1, y1 = oracle.window_box(lv, r, c)
        a["score"], a["f"], a["k"], a["r"], a["c"] = s[f, r, c].astype(np.float64), f, lv.k, r, c
        a["x0"], a["y0"], a["x1"], a["y1"] = x0, y0, x1, y1
        rows.append(a)
    return np.concatenate(rows) if rows else np.empty(0, oracle.CAND_DTYPE)


def det_key(d):
    return list(zip(d["filter"].tolist(), d["level"].tolist(), d["row"].tolist(), d["col"].tolist()))


def cand_key(c):
    return list(zip(c["f"].tolist(), c["k"].tolist(), c["r"].tolist(), c["c"].tolist()))


BOX = ("x0", "y0", "x1", "y1")


def assert_nms_function(H, frame, Wn, bn, u, dets, n, iou=0.5, thresh=0.0):
    """GPU NMS equals the oracle's NMS applied to the GPU's candidates, in
    every field: window, box and score bits."""
    cg = gpu_candidates(H, frame, Wn, bn, u, thresh)
    kept = oracle.nms(cg, float(np.float32(iou)))
    assert n == len(kept), (n, len(kept))
    m = min(len(dets), len(kept))
    assert len(dets) == m
    assert det_key(dets) == cand_key(kept[:m])
    assert np.array_equal(dets["score"], kept["score"][:m].astype(np.float32))
    for f in BOX:
        assert np.array_equal(dets[f], kept[f][:m]), f
    return cg


def _log_exclusion(stats):
    path = os.environ.get("HOG_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(stats) + "\n")


def assert_end_to_end(frame, Wn, bn, u, cg, dets, n=None, label=""):
    """The GPU's candidate set equals the oracle's apart from windows within
    NEAR of the threshold, and every kept/dropped decision that near-
    threshold windows and near ties cannot change is the oracle's (per
    window: see nms_exclusion)."""
    co = oracle.candidates(frame, Wn, bn, 0.0, u)
    near = set(k for k, s in zip(cand_key(co), co["score"]) if abs(s) < NEAR)
    gnear = set(k for k, s in zip(cand_key(cg), cg["score"]) if abs(s) < NEAR)
    so = set(cand_key(co)) - near - gnear
    sg = set(cand_key(cg)) - near - gnear
    assert so == sg, (len(so ^ sg))
    if n is not None:
        assert n == len(dets), "the comparison needs every kept detection"
    stats = nms_exclusion.check_kept(frame, Wn, bn, u, dets, 0.0, 0.5, NEAR, cand_gpu=cg)
    stats["case"] = label
    _log_exclusion(stats)
    # the exclusion must stay a small fraction of the windows (on the 64
    # frames of the 640x480 clip it is 0.3 % on average, 1.8 % at most)
    assert stats["unknown"] <= max(32, 3 * stats["windows"] // 100), stats
    return stats


@pytest.mark.parametrize("name,nf", [("c0", 1), ("c1", 5), ("ragged", 5), ("tall", 2), ("u2", 5),
                                     ("exact80", 5), ("c1", 7)])
def test_detect_parity(H, name, nf):
    frame, u = case_frame(name)
    Wn, bn = synth.filters(range(100, 100 + nf))
    print(f"detect {name} nf={nf}", flush=True)
    dets, n = H.detect(cu(frame), cu(Wn), cu(bn), 0.0, 0.5, u)
    cg = assert_nms_function(H, frame, Wn, bn, u, dets, n)
    st = assert_end_to_end(frame, Wn, bn, u, cg, dets, n, f"detect {name} nf={nf}")
    print(st, flush=True)


def test_detect_small_frames_have_no_levels(H):
    Wn, bn = synth.filters([1])
    for shape in ((79, 200), (200, 79), (40, 40)):
        fr = cu(np.full(shape, 100, np.uint8))
        dets, n = H.detect(fr, cu(Wn), cu(bn))
        assert n == 0 and len(dets) == 0


def test_detect_cap_overflow_reports_true_count(H):
    frame, u = case_frame("c1")
    Wn, bn = synth.filters(range(101, 106))
    full, n = H.detect(cu(frame), cu(Wn), cu(bn))
    part, n2 = H.detect(cu(frame), cu(Wn), cu(bn), cap=5)
    assert n2 == n > 5 and len(part) == 5
    assert np.array_equal(part, full[:5])


def test_constant_frame_scores_equal_bias(H):
    Wn, bn = synth.filters(range(5))
    bn = np.array([0.5, -0.5, 0.25, 0.0, 1.0], np.float32)
    got = H.scores(cu(np.full((200, 240), 90, np.uint8)), cu(Wn), cu(bn))
    for lv, S in got:
        assert np.array_equal(S.cpu().numpy(), np.broadcast_to(bn[:, None, None], S.shape))


def test_detect_large_frame_nms_states_in_global_memory(H):
    """4096x4096: more window positions than the NMS keeps in LDS, so the
    decision states live in global memory.  The filter bias is lowered so
    that the oracle's NMS over the GPU candidates stays quick."""
    rng = np.random.default_rng(21)
    frame = np.clip(np.rint(synth.background(rng, 4096, 4096)), 0, 255).astype(np.uint8)
    Wn, bn = synth.filters(range(500, 505), bias=-2.2)
    levels = H.pyramid(4096, 4096, 1, 5)
    assert sum(l["rows"] * l["cols"] for l in levels) > 16 * 29696
    dets, n = H.detect(cu(frame), cu(Wn), cu(bn))
    print(f"4096x4096: {n} kept", flush=True)
    assert n > 0
    assert_nms_function(H, frame, Wn, bn, 1, dets, n)


@pytest.mark.parametrize("iou,thresh", [(0.6, 0.0), (0.75, 0.5), (0.95, -0.25), (0.5, 1.0)])
def test_detect_iou_and_threshold(H, iou, thresh):
    """NMS thresholds above 1/2 (the exact test I * den > num * U on the
    binary fraction of the float32 iou) and other score thresholds: the GPU
    result equals the oracle's NMS over the GPU's candidates."""
    frame, u = case_frame("c1")
    Wn, bn = synth.filters(range(101, 106))
    print(f"detect iou={iou} thresh={thresh}", flush=True)
    dets, n = H.detect(cu(frame), cu(Wn), cu(bn), thresh, iou, u)
    assert_nms_function(H, frame, Wn, bn, u, dets, n, iou, thresh)
