"""hog_detect_topk: detections and top-k windows from one forward pass are
bit for bit those of hog_detect_batch and hog_topk_windows called apart."""
import numpy as np
import pytest

from paper_2006_00816_amd import synth
from test_gpu_parity import H, cu  # noqa: F401

pytestmark = pytest.mark.gpu


def _same(a, b):
    return len(a) == len(b) and all(np.array_equal(a[f].view(np.int32), b[f].view(np.int32)) for f in a.dtype.names)


@pytest.mark.parametrize("n,nf,u,shape", [(3, 5, 1, (480, 640)), (2, 7, 1, (240, 320)), (1, 5, 2, (150, 170))])
def test_detect_topk_equals_separate_calls(H, n, nf, u, shape):
    gen = synth.ClipGenerator(71 + n, *shape, face_h=min(160.0, shape[0] / 2))
    fr = cu(gen.frames(n))
    W, b = synth.filters(range(600, 600 + nf))
    W, b = cu(W), cu(b)
    d0, n0 = H.alloc_dets(n, 256)
    d1, n1 = H.alloc_dets(n, 256)
    H.detect_batch_into(fr, W, b, d0, n0, upsample=u)
    w0, s0 = H.topk_windows(fr, W, b, 10, upsample=u)
    w1, s1 = H.detect_topk_into(fr, W, b, d1, n1, 10, upsample=u)
    a, ca = H.dets_to_numpy(d0, n0)
    c, cc = H.dets_to_numpy(d1, n1)
    assert np.array_equal(ca, cc)
    assert all(_same(a[i], c[i]) for i in range(n))
    assert np.array_equal(w0.cpu().numpy().reshape(n, 10, 5), w1.cpu().numpy())
    assert np.array_equal(s0.cpu().numpy().view(np.int32).reshape(n, 10), s1.cpu().numpy().view(np.int32))
