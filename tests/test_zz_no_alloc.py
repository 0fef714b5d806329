"""hog_detect_batch_static (the library's fixed scratch array as workspace,
no allocation) against hog_detect_batch with a caller workspace: the same
detections, bit for bit in every field, on two calls in a row, the second
with a smaller input than the first, under the default schedule and a
split schedule on forked streams."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2006_00816_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2006_00816_amd import hog355
    hog355.lib()
    return hog355


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same(a, b):
    if len(a) != len(b):
        return False
    return all(np.array_equal(a[f].view(np.int32), b[f].view(np.int32)) for f in a.dtype.names)


def _both(H, fr, W, b, cap=1024):
    n = int(fr.shape[0])
    d0, n0 = H.alloc_dets(n, cap)
    d1, n1 = H.alloc_dets(n, cap)
    # poison the static outputs so that a call that writes nothing fails
    d1.fill_(-7)
    n1.fill_(-7)
    H.detect_batch_into(fr, W, b, d0, n0)
    H.detect_batch_static_into(fr, W, b, d1, n1)
    torch.cuda.synchronize()
    a, ca = H.dets_to_numpy(d0, n0)
    s, cs = H.dets_to_numpy(d1, n1)
    return a, ca, s, cs


def _check(H, fr, W, b):
    a, ca, s, cs = _both(H, fr, W, b)
    assert np.array_equal(ca, cs), (ca, cs)
    for i in range(len(a)):
        assert np.all(s[i]["frame"] == i)
        assert _same(a[i], s[i]), i
    return int(np.sum(cs))


def test_static_matches_workspace_two_calls(H):
    # first call: 8 frames of 640x480, 5 filters (44.5 MiB of the 64 MiB)
    wl = synth.config1(seed=21, n=8)
    W, b = _cu(wl.W), _cu(wl.b)
    fr = _cu(wl.frames)
    assert H.workspace_bytes(480, 640, 1, 8, 5) <= H.STATIC_SCRATCH_BYTES
    kept = _check(H, fr, W, b)
    assert kept > 0
    # second call, smaller: 3 frames of 320x240 with one filter of another
    # seed, so that stale state of the first call would show
    gen = synth.ClipGenerator(22, 240, 320, face_h=80.0)
    fr2 = _cu(gen.frames(3))
    W2, b2 = synth.filters([123])
    kept2 = _check(H, fr2, _cu(W2), _cu(b2))
    assert kept2 > 0


def test_static_split_schedule(H):
    # the same under a split schedule (frame groups on forked streams) with
    # two filter groups (7 filters, keys merged by atomic max)
    wl = synth.config1(seed=23, n=4)
    W, b = synth.filters(range(300, 307))
    fr = _cu(wl.frames)
    H.lib().hog_init()
    H.tuning_set(480, 640, 1, 4, 7, {"fused": 0, "queues": 8, "wg_per_queue": 32, "lag_f": 1, "lag_s": 2,
                                     "split": 2, "nms_rounds": 4, "score_rows": 0})
    try:
        _check(H, fr, _cu(W), _cu(b))
        _check(H, fr[:2].contiguous(), _cu(W), _cu(b))
    finally:
        H.tuning_set(480, 640, 1, 4, 7, None)


def test_static_rejects_oversized(H):
    # 64 frames of 640x480 need 355 MiB: rejected before anything is enqueued
    wl = synth.config1(seed=24, n=1)
    fr = _cu(np.repeat(wl.frames, 64, axis=0))
    W, b = _cu(wl.W), _cu(wl.b)
    d, nd = H.alloc_dets(64, 16)
    nd.fill_(-3)
    with pytest.raises(H.HogError, match="fixed scratch"):
        H.detect_batch_static_into(fr, W, b, d, nd)
    torch.cuda.synchronize()
    assert torch.all(nd == -3)
