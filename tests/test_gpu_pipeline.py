"""Host pipeline (Sec. V-C, pipelining; Sec. V-A, data transfers): frames
submitted from host memory come back to the consumer with the detections
hog_detect_batch gives for the same frames, bit for bit, whatever the
staging mode, the number of stages and consumer threads, and the size of
the last batch."""
import threading

import numpy as np
import pytest
import torch

from paper_2006_00816_amd import synth
from test_gpu_parity import H, cu  # noqa: F401

pytestmark = pytest.mark.gpu


def _same(a, b):
    return len(a) == len(b) and all(np.array_equal(a[f].view(np.int32), b[f].view(np.int32)) for f in a.dtype.names)


@pytest.mark.parametrize("staging,depth,threads,pinned", [(1, 3, 1, False), (0, 2, 2, False), (1, 1, 1, False),
                                                          (0, 3, 3, True)])
def test_pipeline_equals_detect_batch(H, staging, depth, threads, pinned):
    wl = synth.config1(seed=51, n=10)
    W, b = cu(wl.W), cu(wl.b)
    ref, ref_n = H.detect_batch(cu(wl.frames), W, b, cap=64)
    got = {}
    lock = threading.Lock()

    def consumer(first, dets, nd):
        with lock:
            for i in range(len(nd)):
                got[first + i] = (dets[i][:min(int(nd[i]), 64)].copy(), int(nd[i]))

    src = torch.from_numpy(wl.frames).pin_memory() if pinned else wl.frames
    p = H.Pipeline(W, b, 480, 640, batch=4, depth=depth, cap=64, consumer_threads=threads, staging=bool(staging),
                   consumer=consumer)
    try:
        for s in range(0, 10, 4):
            p.submit(src[s:s + 4], s)          # the last batch holds 2 frames
        p.drain()
    finally:
        p.close()
    assert sorted(got) == list(range(10))
    for i in range(10):
        d, n = got[i]
        assert n == ref_n[i], i
        e = ref[i].copy()
        e["frame"] = i % 4                     # the frame field is the index in its batch
        assert _same(d, e), i


def test_pipeline_reuses_stages_many_batches(H):
    """More batches than stages: every stage is reused and every frame's
    result still matches a direct call."""
    wl = synth.config1(seed=52, n=3)
    W, b = cu(wl.W), cu(wl.b)
    ref, ref_n = H.detect_batch(cu(wl.frames), W, b, cap=32)
    counts = []
    p = H.Pipeline(W, b, 480, 640, batch=3, depth=2, cap=32, consumer_threads=2,
                   consumer=lambda first, d, nd: counts.append((first, nd.tolist())))
    try:
        for i in range(12):
            p.submit(wl.frames, 3 * i)
        p.drain()
    finally:
        p.close()
    assert sorted(c[0] for c in counts) == [3 * i for i in range(12)]
    assert all(c[1] == ref_n.tolist() for c in counts)
