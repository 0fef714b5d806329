"""Per-window exclusion for end-to-end detection parity.

The GPU computes scores in float32 and the oracle in float64, so two
things can legitimately differ: whether a window whose score lies within
NEAR of the threshold is a candidate at all, and the rank order of two
overlapping candidates whose scores lie within NEAR of each other.  Greedy
NMS (Sec. IV-A, non-maximum suppression: detections of one face reduced to
the best-scoring one) propagates such a difference only along conflicts:
a candidate's decision depends on the decisions of the better-ranked
candidates whose boxes overlap it with IoU above the NMS threshold.

``decisions`` runs the greedy pass over the oracle's windows in
three-valued logic.  A window is
  KEPT     if every better-ranked conflicting window is surely DROPPED and
           its own candidacy and rank are unambiguous;
  DROPPED  if some better-ranked conflicting window is surely KEPT (then
           it is suppressed whether or not it is a candidate, and whatever
           its rank among near ties);
  UNKNOWN  otherwise.
Only UNKNOWN windows may differ between the GPU and the oracle; every
window with a sure decision must match.
"""
from __future__ import annotations

import numpy as np

from oracle import hog as oracle

KEPT, DROPPED, UNKNOWN = 1, 2, 0


def _conflict_lists(c, iou):
    """For each window i (rank order), the indices j of all windows whose
    boxes overlap it with IoU > iou, tested exactly on integer areas."""
    num, den = float(iou).as_integer_ratio()
    x0, y0, x1, y1 = (c[f].astype(np.int64) for f in ("x0", "y0", "x1", "y1"))
    area = (x1 - x0) * (y1 - y0)
    out = []
    for i in range(len(c)):
        iw = np.maximum(0, np.minimum(x1, x1[i]) - np.maximum(x0, x0[i]))
        ih = np.maximum(0, np.minimum(y1, y1[i]) - np.maximum(y0, y0[i]))
        inter = iw * ih
        union = area + area[i] - inter
        hit = inter * den > num * union
        hit[i] = False
        out.append(np.nonzero(hit)[0])
    return out


def decisions(windows, thresh, iou, near):
    """Three-valued greedy NMS over `windows` (oracle CAND_DTYPE records of
    every window scoring above thresh - near).  Returns the windows in rank
    order and their decisions."""
    c, st, _ = decisions_with_conflicts(windows, thresh, iou, near)
    return c, st


def decisions_with_conflicts(windows, thresh, iou, near):
    """decisions(), also returning the conflict lists (rank order)."""
    c = windows[oracle.rank_order(windows)]
    conf = _conflict_lists(c, iou)
    return c, _decide(c, conf, thresh, near), conf


def _decide(c, conf, thresh, near):
    s = c["score"]
    maybe = np.abs(s - thresh) < near
    tie = np.zeros(len(c), bool)
    for i, js in enumerate(conf):
        if len(js) and np.any(np.abs(s[js] - s[i]) < near):
            tie[i] = True
    st = np.full(len(c), UNKNOWN, np.int8)
    for i, js in enumerate(conf):
        better = js[js < i]
        sb = st[better]
        if np.any(sb == KEPT):
            st[i] = DROPPED
        elif maybe[i] or tie[i]:
            st[i] = UNKNOWN
        elif np.all(sb == DROPPED):
            st[i] = KEPT
    return st


def check_ranking(c, conf, cand_gpu, near):
    """Among the GPU's candidates (structured array with the GPU's float32
    scores), every pair of conflicting windows is ranked as the oracle
    ranks them (c: oracle windows in rank order, conf: their conflict
    lists), unless the two oracle scores are within `near`.  Returns the
    number of conflicting pairs checked."""
    key = {k: i for i, k in enumerate(zip(c["f"].tolist(), c["k"].tolist(), c["r"].tolist(), c["c"].tolist()))}
    n = len(c)
    gs = np.full(n, np.nan)
    gidx = np.full(n, -1, np.int64)
    g = cand_gpu[oracle.rank_order(cand_gpu)]
    for pos, kk in enumerate(zip(g["f"].tolist(), g["k"].tolist(), g["r"].tolist(), g["c"].tolist())):
        i = key[kk]
        gs[i] = g["score"][pos]
        gidx[i] = pos                      # the GPU's rank
    s = c["score"]
    pairs = 0
    for i, js in enumerate(conf):
        if gidx[i] < 0:
            continue
        js = js[(js < i) & (gidx[js] >= 0)]          # oracle ranks j before i
        pairs += len(js)
        flipped = js[gidx[js] > gidx[i]]
        bad = flipped[np.abs(s[flipped] - s[i]) >= near]
        assert len(bad) == 0, (f"GPU ranks window {i} above conflicting window {int(bad[0])} although "
                               f"their oracle scores differ by {float(s[bad[0]] - s[i]):.3g}")
    return pairs


def check_kept(frame, W, b, upsample, dets, thresh=0.0, iou=0.5, near=1e-4, cand_gpu=None, min_face=0, region=None):
    """End-to-end check of a frame's GPU detections against the oracle:
    every window whose decision is sure must be kept or dropped on the GPU
    exactly as by the oracle; with the GPU's candidates, also their rank
    order (check_ranking).  min_face and region restrict the windows as in
    the detection.  Returns statistics of the comparison."""
    allw = oracle.candidates(frame, W, b, thresh - near, upsample, min_face=min_face, region=region)
    c, st, conf = decisions_with_conflicts(allw, thresh, iou, near)
    key = list(zip(c["f"].tolist(), c["k"].tolist(), c["r"].tolist(), c["c"].tolist()))
    index = {k: i for i, k in enumerate(key)}
    got = list(zip(dets["filter"].tolist(), dets["level"].tolist(), dets["row"].tolist(), dets["col"].tolist()))
    outside = [g for g in got if g not in index]
    assert not outside, f"GPU kept windows scoring below thresh - near in the oracle: {outside[:5]}"
    kept_gpu = np.zeros(len(c), bool)
    kept_gpu[[index[g] for g in got]] = True
    sure = st != UNKNOWN
    want = st == KEPT
    bad = np.nonzero(sure & (kept_gpu != want))[0]
    stats = {"windows": int(len(c)), "unknown": int((~sure).sum()), "kept_sure": int(want.sum()),
             "kept_unknown_gpu": int((kept_gpu & ~sure).sum()), "differ_sure": int(len(bad))}
    if cand_gpu is not None:
        stats["ranked_pairs"] = check_ranking(c, conf, cand_gpu, near)
    assert len(bad) == 0, (f"sure decisions differ at {len(bad)} windows, e.g. "
                           f"{[(key[i], float(c['score'][i]), int(st[i])) for i in bad[:5]]}; {stats}")
    return stats
