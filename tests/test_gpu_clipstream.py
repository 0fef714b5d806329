"""Several clips in flight (ClipStream): every captured graph, launched in
turn on its own stream, gives the detections of hog_detect_batch on its
own input buffer, replay after replay; the in-flight tuner keeps one of
its candidates."""
import numpy as np
import pytest
import torch

from paper_2006_00816_amd import synth
from test_gpu_batch import _same
from test_gpu_parity import H, cu  # noqa: F401

pytestmark = pytest.mark.gpu


def _check_graph(H, g, ref, nref):
    torch.cuda.synchronize()
    got, n = H.dets_to_numpy(g.dets, g.n_dets)
    assert np.array_equal(n, nref), (n, nref)
    for i in range(len(ref)):
        assert _same(got[i], ref[i]), i


@pytest.mark.parametrize("depth", [2, 3, 4])
def test_clips_in_flight_equal_detect_batch(H, depth):
    # different clips in the buffers, so that a graph reading another's
    # buffer or workspace would show
    clips = [synth.config1(seed=30 + k, n=4) for k in range(depth)]
    W, b = cu(clips[0].W), cu(clips[0].b)
    frames = [cu(c.frames) for c in clips]
    refs = [H.detect_batch(f, W, b) for f in frames]
    print(f"clips in flight: {depth}, 4 frames of 640x480 each", flush=True)
    cs = H.ClipStream(frames, W, b)
    try:
        for _ in range(3 * depth + 1):
            cs.launch()
        cs.synchronize()
        for g, f, (ref, nref) in zip(cs.graphs, frames, refs):
            _check_graph(H, g, ref, nref)
    finally:
        cs.close()


def test_refilled_buffer_between_launches(H):
    # a graph's input refreshed on its own stream before its next launch
    a = synth.config1(seed=41, n=3)
    c = synth.config1(seed=42, n=3)
    W, b = cu(a.W), cu(a.b)
    fa, fc = cu(a.frames), cu(c.frames)
    bufs = [fa.clone(), fa.clone()]
    cs = H.ClipStream(bufs, W, b)
    try:
        g0 = cs.launch()
        cs.launch()
        with torch.cuda.stream(cs.stream_of(g0)):
            bufs[0].copy_(fc)
        g = cs.launch()
        assert g is g0
        cs.synchronize()
        _check_graph(H, g0, *H.detect_batch(fc, W, b))
        _check_graph(H, cs.graphs[1], *H.detect_batch(fa, W, b))
    finally:
        cs.close()


def test_tune_clip_stream_keeps_a_candidate(H):
    wl = synth.config1(seed=43, n=2)
    W, b = cu(wl.W), cu(wl.b)
    fr = cu(wl.frames)
    base = {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "stagger": 0, "score_rows": 0}
    cands = [{**base, "split": 1, "nms_rounds": nr} for nr in (2, 5)]
    best, ms = H.tune_clip_stream([fr, fr.clone()], W, b, cands, warmup=2, reps=4)
    try:
        assert best in cands and ms > 0
        ref, nref = H.detect_batch(fr, W, b)
        cs = H.ClipStream([fr, fr.clone()], W, b)
        try:
            cs.launch()
            cs.launch()
            cs.synchronize()
            for g in cs.graphs:
                _check_graph(H, g, ref, nref)
        finally:
            cs.close()
    finally:
        n, h, w = (int(v) for v in fr.shape)
        H.tuning_set(h, w, 1, n, int(W.shape[0]), None)


@pytest.mark.parametrize("rounds", [0, 3])
def test_clip_64_in_flight_schedules(H, rounds):
    """The 64-frame 640x480 clip, three clips in flight under the schedules
    the benchmark's in-flight tuner chooses among (one group, 16-row
    scoring items, 0 or 3 parallel NMS rounds): every graph's detections
    equal those of the default schedule, bit for bit."""
    wl = synth.config1(seed=1, n=64)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    ref, nref = H.detect_batch(fr, W, b)
    t = {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "stagger": 0, "split": 1,
         "nms_rounds": rounds, "score_rows": 16}
    print(f"64-frame clip, 3 in flight, nms_rounds={rounds}", flush=True)
    H.tuning_set(480, 640, 1, 64, 5, t)
    try:
        cs = H.ClipStream([fr, fr.clone(), fr.clone()], W, b)
        try:
            for _ in range(7):
                cs.launch()
            cs.synchronize()
            for g in cs.graphs:
                _check_graph(H, g, ref, nref)
        finally:
            cs.close()
    finally:
        H.tuning_set(480, 640, 1, 64, 5, None)
