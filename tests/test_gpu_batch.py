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


def _same(a, b, frame=None):
    """Equal detections, bit for bit, apart from the frame index, which a
    batch numbers by position."""
    if len(a) != len(b):
        return False
    if frame is not None and not (np.all(a["frame"] == frame) and np.all(b["frame"] == 0)):
        return False
    fields = [f for f in a.dtype.names if f != "frame"]
    return all(np.array_equal(a[f].view(np.int32), b[f].view(np.int32)) for f in fields)


def test_batch_equals_single(H):
    wl = synth.config1(seed=11, n=6)
    fr = cu(wl.frames)
    W, b = cu(wl.W), cu(wl.b)
    batch, nb = H.detect_batch(fr, W, b)
    for i in range(len(wl.frames)):
        single, n = H.detect(fr[i], W, b)
        assert nb[i] == n
        assert _same(batch[i], single, i), i


def test_batch_mixed_filter_groups(H):
    # 7 filters: two filter groups merge their keys with atomic max
    wl = synth.config1(seed=12, n=3)
    W, b = synth.filters(range(400, 407))
    fr = cu(wl.frames)
    batch, nb = H.detect_batch(fr, cu(W), cu(b))
    for i in range(3):
        single, n = H.detect(fr[i], cu(W), cu(b))
        assert nb[i] == n and _same(batch[i], single, i)


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
    for i in (0, 31, 63):
        print(f"clip frame {i}: {ng[i]} kept", flush=True)
        cg = assert_nms_function(H, wl.frames[i], wl.W, wl.b, 1, got[i], int(ng[i]))
        assert_end_to_end(wl.frames[i], wl.W, wl.b, 1, cg, got[i])
    g.close()
