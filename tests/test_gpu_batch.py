"""Batched and graph-replayed detection: every frame's result is the same
alone, in a batch and in a replayed graph; the 64-frame 640x480 clip in
the benchmark's launch configuration is checked against the oracle on
sampled frames."""
import numpy as np
import pytest
import torch

from paper_2006_00816_amd import synth
from test_gpu_parity import H, assert_end_to_end, assert_nms_function, cu  # noqa: F401

pytestmark = pytest.mark.gpu


def _same(a, b):
    """Equal detections, bit for bit, in every field (frame index
    included)."""
    if len(a) != len(b):
        return False
    return all(np.array_equal(a[f].view(np.int32), b[f].view(np.int32)) for f in a.dtype.names)


def _renumbered(d, i):
    """A copy of detections d with the frame field set to i."""
    d = d.copy()
    d["frame"] = i
    return d


def _assert_frames_numbered(dets):
    """Frame i of a batch reports frame index i in every detection."""
    for i, d in enumerate(dets):
        assert np.all(d["frame"] == i), (i, np.unique(d["frame"]))


def test_batch_equals_single(H):
    wl = synth.config1(seed=11, n=6)
    fr = cu(wl.frames)
    W, b = cu(wl.W), cu(wl.b)
    batch, nb = H.detect_batch(fr, W, b)
    _assert_frames_numbered(batch)
    for i in range(len(wl.frames)):
        single, n = H.detect(fr[i], W, b)
        assert nb[i] == n
        assert np.all(single["frame"] == 0)
        assert _same(batch[i], _renumbered(single, i)), i


def test_batch_mixed_filter_groups(H):
    # 7 filters: two filter groups merge their keys with atomic max
    wl = synth.config1(seed=12, n=3)
    W, b = synth.filters(range(400, 407))
    fr = cu(wl.frames)
    batch, nb = H.detect_batch(fr, cu(W), cu(b))
    _assert_frames_numbered(batch)
    for i in range(3):
        single, n = H.detect(fr[i], cu(W), cu(b))
        assert nb[i] == n and _same(batch[i], _renumbered(single, i))


def test_graph_replay_matches_eager(H):
    wl = synth.config1(seed=13, n=8)
    fr = cu(wl.frames)
    W, b = cu(wl.W), cu(wl.b)
    eager, ne = H.detect_batch(fr, W, b)
    g = H.DetectGraph(fr, W, b)
    other = cu(synth.config0(5).frames[0])
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        got, ng = H.dets_to_numpy(g.dets, g.n_dets)
        assert np.array_equal(ng, ne), rep
        for i in range(8):
            assert _same(got[i], eager[i]), (rep, i)
        # unrelated eager work between replays
        H.scores(other, W, b)
        torch.cuda.synchronize()
    # new frames in the same buffer
    wl2 = synth.config1(seed=14, n=8)
    fr.copy_(cu(wl2.frames))
    eager2, ne2 = H.detect_batch(fr, W, b)
    g.launch()
    torch.cuda.synchronize()
    got, ng = H.dets_to_numpy(g.dets, g.n_dets)
    assert np.array_equal(ng, ne2)
    for i in range(8):
        assert _same(got[i], eager2[i])
    g.close()


def test_clip_64x640x480_graph_sampled_against_oracle(H):
    wl = synth.config1(seed=1, n=64)
    fr = cu(wl.frames)
    W, b = cu(wl.W), cu(wl.b)
    g = H.DetectGraph(fr, W, b)
    g.launch()
    torch.cuda.synchronize()
    got, ng = H.dets_to_numpy(g.dets, g.n_dets)
    _assert_frames_numbered(got)
    for i in (0, 31, 63):
        print(f"clip frame {i}: {ng[i]} kept", flush=True)
        cg = assert_nms_function(H, wl.frames[i], wl.W, wl.b, 1, _renumbered(got[i], 0), int(ng[i]))
        assert_end_to_end(wl.frames[i], wl.W, wl.b, 1, cg, got[i], int(ng[i]), f"clip frame {i}")
    g.close()


def test_padded_batch_against_oracle(H):
    """Frames whose rows are padded (pitch > w) in a buffer whose frames are
    padded too (frame stride > pitch * h), the padding filled with 255:
    detections equal those of the packed frames in every field, and frames
    0 and 4 equal the oracle's."""
    wl = synth.config1(seed=15, n=5)
    n, h, w = wl.frames.shape
    big = torch.full((n, h + 3, w + 24), 255, dtype=torch.uint8, device="cuda")
    big[:, :h, :w] = cu(wl.frames)
    view = big[:, :h, :w]
    assert view.stride() == ((h + 3) * (w + 24), w + 24, 1)
    W, b = cu(wl.W), cu(wl.b)
    got, ng = H.detect_batch(view, W, b)
    ref, nr = H.detect_batch(cu(wl.frames), W, b)
    assert np.array_equal(ng, nr)
    _assert_frames_numbered(got)
    for i in range(n):
        assert _same(got[i], ref[i]), i
    for i in (0, 4):
        single, ns = H.detect(view[i], W, b)
        assert _same(_renumbered(single, i), got[i])
        cg = assert_nms_function(H, wl.frames[i], wl.W, wl.b, 1, _renumbered(got[i], 0), int(ng[i]))
        assert_end_to_end(wl.frames[i], wl.W, wl.b, 1, cg, got[i], int(ng[i]), f"padded frame {i}")


def test_fused_schedule_against_oracle(H):
    """The persistent fused schedule's detections against the oracle on
    sampled frames of an 8-frame 640x480 clip (not only against the
    per-stage schedule)."""
    wl = synth.config1(seed=16, n=8)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    H.tuning_set(480, 640, 1, 8, 5, {"fused": 1, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2,
                                     "split": 1, "nms_rounds": 3, "score_rows": 0})
    try:
        got, ng = H.detect_batch(fr, W, b)
    finally:
        H.tuning_set(480, 640, 1, 8, 5, None)
    _assert_frames_numbered(got)
    for i in (0, 7):
        print(f"fused frame {i}: {ng[i]} kept", flush=True)
        cg = assert_nms_function(H, wl.frames[i], wl.W, wl.b, 1, _renumbered(got[i], 0), int(ng[i]))
        assert_end_to_end(wl.frames[i], wl.W, wl.b, 1, cg, got[i], int(ng[i]), f"fused frame {i}")
