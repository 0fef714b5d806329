"""Served stream: every request's detections are the same as for that
frame alone, and every request is served."""
import numpy as np
import pytest
import torch

from test_gpu_parity import H  # noqa: F401

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone(H):
    from paper_2006_00816_amd import serve
    pools, W, b = serve.pinned_pools(per_res=8)
    stats, done, frames = serve.served_stream(3000.0, 0.4, W, b, pools, max_batch=8, slots=3)
    print(stats, flush=True)
    assert stats["frames"] == len(done) > 500
    assert stats["mean_batch"] > 1.0          # requests were batched together
    for r in done[::7]:
        alone, n = H.detect(r.frame.cuda(), W, b, cap=256)
        assert r.n_dets == n
        assert len(r.dets) == len(alone)
        assert np.all(r.dets["frame"] == r.batch_index) and np.all(alone["frame"] == 0)
        for f in ("filter", "level", "row", "col", "x0", "y0", "x1", "y1"):
            assert np.array_equal(r.dets[f], alone[f]), (r.rid, f)
        assert np.array_equal(r.dets["score"].view(np.int32), alone["score"].view(np.int32))
    lat = np.array([r.done - r.arrival for r in done])
    assert np.all(lat > 0)
