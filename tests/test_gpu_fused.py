"""Schedules of hog_detect_batch give the same detections, bit for bit:
the fused persistent kernel (histograms, features and scores of every
frame and level from one work list) for several work-list settings, batch
sizes that do not fill the queues evenly, several filter groups, 2x
upsampling and graph replay; the per-stage kernels with the frames split
into groups on forked streams; and the autotuner's pick."""
import numpy as np
import pytest
import torch

from paper_2006_00816_amd import synth
from test_gpu_batch import _assert_frames_numbered, _same
from test_gpu_parity import H, cu  # noqa: F401

pytestmark = pytest.mark.gpu

STAGED = {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "split": 1, "nms_rounds": 3, "score_rows": 0}


def _run(H, fr, W, b, tuning, upsample=1):
    n, h, w = (int(v) for v in fr.shape)
    nf = int(W.shape[0])
    H.tuning_set(h, w, upsample, n, nf, tuning)
    try:
        return H.detect_batch(fr, W, b, upsample=upsample)
    finally:
        H.tuning_set(h, w, upsample, n, nf, None)


def _assert_same(a, b, n):
    """Same counts and detections in every field; frame i of each batch
    numbered i."""
    (da, na), (db, nb) = a, b
    assert np.array_equal(na, nb), (na, nb)
    _assert_frames_numbered(da)
    _assert_frames_numbered(db)
    for i in range(n):
        assert _same(da[i], db[i]), i


@pytest.mark.parametrize("queues,wg,lag_f,lag_s", [(8, 32, 1, 2), (1, 256, 1, 2), (8, 4, 2, 3), (3, 5, 1, 3),
                                                   (1, 1, 1, 2)])
def test_fused_equals_staged_clip(H, queues, wg, lag_f, lag_s):
    wl = synth.config1(seed=21, n=13)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    print(f"fused q={queues} wg={wg} lags=({lag_f},{lag_s}) n=13", flush=True)
    ref = _run(H, fr, W, b, STAGED)
    got = _run(H, fr, W, b, {"fused": 1, "queues": queues, "wg_per_queue": wg, "lag_f": lag_f, "lag_s": lag_s, "split": 1, "nms_rounds": 3, "score_rows": 0})
    _assert_same(got, ref, 13)
    assert sum(ref[1]) > 0


@pytest.mark.parametrize("nf,shape,upsample,n", [(1, (240, 320), 1, 2), (7, (480, 640), 1, 9),
                                                 (12, (131, 97), 1, 4), (5, (120, 100), 2, 3),
                                                 (4, (85, 263), 1, 1)])
def test_fused_equals_staged_shapes(H, nf, shape, upsample, n):
    h, w = shape
    frames = []
    for i in range(n):
        rng = np.random.default_rng(500 + i)
        U = synth.background(rng, h, w)
        synth.paint_face(U, h / 2 + 3 * i, w / 2, 0.5 * min(h, w), 200.0)
        frames.append(np.clip(np.rint(U), 0, 255).astype(np.uint8))
    fr = cu(np.stack(frames))
    W, b = synth.filters(range(600, 600 + nf))
    W, b = cu(W), cu(b)
    print(f"fused nf={nf} {h}x{w} u={upsample} n={n}", flush=True)
    ref = _run(H, fr, W, b, STAGED, upsample)
    got = _run(H, fr, W, b, {"fused": 1, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "split": 1, "nms_rounds": 3, "score_rows": 0}, upsample)
    _assert_same(got, ref, n)


@pytest.mark.parametrize("split,n,rounds,rows", [(2, 13, 3, 16), (3, 13, 0, 4), (4, 5, 8, 16), (4, 3, 16, 4),
                                                (1, 6, 0, 4), (1, 6, 16, 16), (1, 1, 3, 4)])
def test_split_rounds_rows_equal_staged(H, split, n, rounds, rows):
    wl = synth.config1(seed=24, n=n)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    print(f"split={split} n={n} nms_rounds={rounds} score_rows={rows}", flush=True)
    ref = _run(H, fr, W, b, {**STAGED, "score_rows": 16})
    got = _run(H, fr, W, b, {**STAGED, "split": split, "nms_rounds": rounds, "score_rows": rows})
    _assert_same(got, ref, n)


@pytest.mark.parametrize("split,stagger", [(2, 0), (4, 0), (2, 1), (4, 1), (2, 2), (3, 2)])
def test_split_clip_64_frames_numbered(H, split, stagger):
    """The 64-frame 640x480 clip under split schedules (frame groups on
    forked streams, starting together or staggered after the previous
    group's histograms or scores; eager and graph-replayed): every field of
    every detection equals the single-group schedule's, frame index
    included."""
    wl = synth.config1(seed=1, n=64)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    print(f"split={split} stagger={stagger} n=64", flush=True)
    ref = _run(H, fr, W, b, STAGED)
    got = _run(H, fr, W, b, {**STAGED, "split": split, "stagger": stagger})
    _assert_same(got, ref, 64)
    H.tuning_set(480, 640, 1, 64, 5, {**STAGED, "split": split, "stagger": stagger})
    try:
        g = H.DetectGraph(fr, W, b)
        g.launch()
        torch.cuda.synchronize()
        _assert_same(H.dets_to_numpy(g.dets, g.n_dets), ref, 64)
        g.close()
    finally:
        H.tuning_set(480, 640, 1, 64, 5, None)


def test_split_graph_replay(H):
    wl = synth.config1(seed=25, n=16)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    ref = _run(H, fr, W, b, STAGED)
    H.tuning_set(480, 640, 1, 16, 5, {**STAGED, "split": 2})
    try:
        g = H.DetectGraph(fr, W, b)
        other = cu(synth.config0(5).frames[0])
        for rep in range(3):
            g.launch()
            torch.cuda.synchronize()
            _assert_same(H.dets_to_numpy(g.dets, g.n_dets), ref, 16)
            H.scores(other, W, b)
            torch.cuda.synchronize()
        g.close()
    finally:
        H.tuning_set(480, 640, 1, 16, 5, None)


def test_fused_graph_replay(H):
    wl = synth.config1(seed=22, n=16)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    ref = _run(H, fr, W, b, STAGED)
    H.tuning_set(480, 640, 1, 16, 5, {"fused": 1, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2, "split": 1, "nms_rounds": 3, "score_rows": 0})
    try:
        g = H.DetectGraph(fr, W, b)
        other = cu(synth.config0(5).frames[0])
        for rep in range(3):
            g.launch()
            torch.cuda.synchronize()
            got = H.dets_to_numpy(g.dets, g.n_dets)
            _assert_same(got, ref, 16)
            H.scores(other, W, b)
            torch.cuda.synchronize()
        g.close()
    finally:
        H.tuning_set(480, 640, 1, 16, 5, None)


def test_autotune_keeps_detections(H):
    wl = synth.config1(seed=23, n=8)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    ref = _run(H, fr, W, b, STAGED)
    best, ms = H.autotune(fr, W, b, reps=2)
    print(f"autotune: {best} {ms:.3f} ms", flush=True)
    assert ms > 0 and best["fused"] in (0, 1)
    t, found = H.tuning_get(480, 640, 1, 8, 5)
    assert found and t == best
    got = H.detect_batch(fr, W, b)
    _assert_same(got, ref, 8)
    H.tuning_set(480, 640, 1, 8, 5, None)


def test_split_on_thread_without_helper_streams(H):
    """A host thread that never ran hog_init has no helper streams: the
    split schedule then runs its frame groups in order on the caller's
    stream, with the same detections."""
    import threading
    wl = synth.config1(seed=26, n=6)
    fr, W, b = cu(wl.frames), cu(wl.W), cu(wl.b)
    ref = _run(H, fr, W, b, STAGED)
    H.tuning_set(480, 640, 1, 6, 5, {**STAGED, "split": 3})
    out = {}

    def work():
        try:
            out["got"] = H.detect_batch(fr, W, b)
            torch.cuda.synchronize()
        except Exception as e:   # reported below
            out["err"] = e

    try:
        t = threading.Thread(target=work)
        t.start()
        t.join(120)
    finally:
        H.tuning_set(480, 640, 1, 6, 5, None)
    assert "err" not in out, out.get("err")
    _assert_same(out["got"], ref, 6)
