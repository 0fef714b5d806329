"""Separable (row / column) filters through the C ABI against the float64
oracle applied to the combined filter W[dr][dc][ch] = sum_i col_i[dr][ch]
row_i[dc][ch] (the paper's row-then-column classifier, Sec. V-A):
scores within 1e-5 relative + 2e-5 absolute, candidate windows bit-exact,
NMS as a function bit-exact, end-to-end kept windows equal up to the
per-window exclusion; batches and graph replays equal single frames."""
import numpy as np
import pytest
import torch

from oracle import hog as oracle
from paper_2006_00816_amd import synth
from test_gpu_batch import _assert_frames_numbered, _renumbered, _same
from test_gpu_parity import (H, assert_end_to_end, assert_nms_function, case_frame, close, cu,  # noqa: F401
                             gpu_candidates)

pytestmark = pytest.mark.gpu


def _bank(H, row, col, b):
    return H.FilterBank(cu(b), row=cu(row), col=cu(col))


@pytest.mark.parametrize("name,nf,rank", [("c0", 1, 1), ("c1", 5, 1), ("c1", 5, 2), ("ragged", 5, 3),
                                          ("tall", 3, 4), ("u2", 7, 1), ("exact80", 5, 2), ("c0", 12, 1)])
def test_separable_scores_parity(H, name, nf, rank):
    frame, u = case_frame(name)
    row, col, b = synth.separable_filters(range(700, 700 + nf), rank)
    print(f"separable scores {name} nf={nf} rank={rank}", flush=True)
    got = H.scores_bank(cu(frame), _bank(H, row, col, b), u)
    Wfull = oracle.separable_filters(row, col)
    want = []
    oracle.candidates(frame, Wfull, b, 0.0, u, levels_out=want)
    assert len(got) == len(want)
    for (glv, gS), (olv, oS) in zip(got, want):
        ok, err, nbad = close(gS.cpu().numpy(), oS)
        assert ok, (name, nf, rank, olv.k, err, nbad)


def _sep_candidates(H, frame, bank, u):
    """GPU candidates of a filter bank from its dense scores (as
    gpu_candidates does for full filters)."""
    rows = []
    levels = oracle.pyramid(*frame.shape, u)
    for glv, gS in H.scores_bank(cu(frame), bank, u):
        s = gS.cpu().numpy()
        f, r, c = np.nonzero(s > np.float32(0.0))
        lv = levels[glv["k"]]
        a = np.empty(len(f), oracle.CAND_DTYPE)
        x0, y0, x1, y1 = oracle.window_box(lv, r, c)
        a["score"], a["f"], a["k"], a["r"], a["c"] = s[f, r, c].astype(np.float64), f, lv.k, r, c
        a["x0"], a["y0"], a["x1"], a["y1"] = x0, y0, x1, y1
        rows.append(a)
    return np.concatenate(rows) if rows else np.empty(0, oracle.CAND_DTYPE)


@pytest.mark.parametrize("name,nf,rank", [("c0", 1, 1), ("c1", 5, 1), ("c1", 5, 2), ("ragged", 5, 1),
                                          ("u2", 5, 2)])
def test_separable_detect_parity(H, name, nf, rank):
    frame, u = case_frame(name)
    row, col, b = synth.separable_filters(range(720, 720 + nf), rank)
    bank = _bank(H, row, col, b)
    print(f"separable detect {name} nf={nf} rank={rank}", flush=True)
    (dets,), (n,) = H.detect_batch_bank(cu(frame[None]), bank, upsample=u)
    n = int(n)
    cg = _sep_candidates(H, frame, bank, u)
    kept = oracle.nms(cg)
    assert n == len(kept) == len(dets)
    assert list(zip(dets["filter"].tolist(), dets["level"].tolist(), dets["row"].tolist(), dets["col"].tolist())) == \
        list(zip(kept["f"].tolist(), kept["k"].tolist(), kept["r"].tolist(), kept["c"].tolist()))
    assert np.array_equal(dets["score"], kept["score"].astype(np.float32))
    for f in ("x0", "y0", "x1", "y1"):
        assert np.array_equal(dets[f], kept[f])
    st = assert_end_to_end(frame, oracle.separable_filters(row, col), b, u, cg, dets, n,
                           f"separable {name} nf={nf} rank={rank}")
    print(st, flush=True)


def test_separable_clip_batch_graph_and_small_batch(H):
    """The 64-frame clip with rank-1 filters: eager batch, graph replays and
    frames alone give the same detections in every field; sampled frames
    against the oracle."""
    wl = synth.config1(seed=1, n=64)
    row, col, b = synth.separable_filters(range(101, 106), 1)
    bank = _bank(H, row, col, b)
    fr = cu(wl.frames)
    ref, nr = H.detect_batch_bank(fr, bank)
    _assert_frames_numbered(ref)
    g = H.DetectGraph(fr, bank=bank)
    for rep in range(2):
        g.launch()
        torch.cuda.synchronize()
        got, ng = H.dets_to_numpy(g.dets, g.n_dets)
        assert np.array_equal(ng, nr)
        for i in range(64):
            assert _same(got[i], ref[i]), (rep, i)
    g.close()
    for i in (0, 40):
        (single,), (ns,) = H.detect_batch_bank(fr[i:i + 1], bank)
        assert int(ns) == nr[i] and _same(_renumbered(single, i), ref[i])
        cg = _sep_candidates(H, wl.frames[i], bank, 1)
        kept = oracle.nms(cg)
        assert len(kept) == nr[i]
        assert_end_to_end(wl.frames[i], oracle.separable_filters(row, col), b, 1, cg, ref[i], int(nr[i]),
                          f"separable clip frame {i}")


def test_separable_rank_one_of_full_filter_equals_full(H):
    """A full filter that is exactly separable (W = col x row per channel)
    scores the same through both banks, to float32 rounding."""
    frame, u = case_frame("c1")
    row, col, b = synth.separable_filters(range(740, 745), 1)
    W = oracle.separable_filters(row, col).astype(np.float32)
    full = H.scores(cu(frame), cu(W), cu(b), u)
    sep = H.scores_bank(cu(frame), _bank(H, row, col, b), u)
    for (lv, a), (_, s) in zip(full, sep):
        ok, err, nbad = close(s.cpu().numpy(), a.cpu().numpy().astype(np.float64))
        assert ok, (lv["k"], err, nbad)
