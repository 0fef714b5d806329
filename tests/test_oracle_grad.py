"""P12/P13: the oracle's analytic gradients against float64 central finite
differences of its own forward pass (a different computation: the
forward never evaluates a derivative)."""
import numpy as np
import pytest

from oracle import hog
from paper_2006_00816_amd import synth


def test_filter_gradient_matches_central_differences():
    crops, labels = synth.config3(seed=3, n_pos=16, n_neg=16)
    F = np.stack([hog.level_features(c, hog.Level(0, 1, 1, 80, 80)) for c in crops])
    assert F.shape == (32, 10, 10, 31)
    rng = np.random.default_rng(3)
    W = rng.normal(0, 0.1, (10, 10, 31))
    b = -0.5
    lam = 1e-4

    def loss(Wv, bv):
        S = bv + np.tensordot(F, Wv, axes=3)
        return hog.hinge_loss(S, labels, Wv, lam)

    S = b + np.tensordot(F, W, axes=3)
    dS = hog.hinge_dscore(S, labels)
    dW, db = hog.filter_grad(F, dS)
    dW = dW + 2 * lam * W
    h = 1e-6
    num = np.empty_like(W)
    for idx in np.ndindex(W.shape):
        Wp = W.copy()
        Wp[idx] += h
        Wm = W.copy()
        Wm[idx] -= h
        num[idx] = (loss(Wp, b) - loss(Wm, b)) / (2 * h)
    assert np.allclose(dW, num, rtol=1e-6, atol=1e-8)
    nb = (loss(W, b + h) - loss(W, b - h)) / (2 * h)
    assert abs(db - nb) <= 1e-8
    assert np.abs(dW).max() > 1e-3       # a non-trivial gradient


def _state(U, W, b, windows, u):
    """Discrete state the analytic gradient holds fixed: bins and clip
    decisions of every level holding a window, and the top-k set."""
    H, Wd = U.shape
    out = []
    for lv in hog.pyramid(H, Wd, u):
        if not np.any(windows["k"] == lv.k):
            continue
        st = hog.level_forward(U, lv)
        hn = st["hist"][..., None, :] * st["n"][..., :, None]
        uu = (st["hist"][..., :9] + st["hist"][..., 9:])[..., None, :] * st["n"][..., :, None]
        out.append((st["bins"], hn < hog.CLIP, uu < hog.CLIP))
    return out


def _same_state(a, b):
    return all(all(np.array_equal(x, y) for x, y in zip(p, q)) for p, q in zip(a, b))


@pytest.mark.parametrize("seed,u,h,w", [(61, 1, 104, 120), (62, 2, 60, 68)])
def test_pixel_gradient_matches_central_differences(seed, u, h, w):
    rng = np.random.default_rng(seed)
    U = synth.background(rng, h, w)
    synth.paint_face(U, h / 2, w / 2, 0.6 * min(h, w), 200.0)
    U = U + rng.uniform(-0.3, 0.3, U.shape)      # break exact gradient ties
    W, b = synth.filters([201, 202])
    dU, win = hog.topk_pixel_grad(U, W, b, 10, u)
    assert len(win) == 10
    s0 = _state(U, W, b, win, u)
    cand = np.argwhere(np.abs(dU) > 1e-4)
    assert len(cand) > 64
    pick = cand[rng.choice(len(cand), 64, replace=False)]
    hstep = 1e-6
    checked = 0
    for y, x in pick:
        Up = U.copy()
        Up[y, x] += hstep
        Um = U.copy()
        Um[y, x] -= hstep
        wp = hog.top_windows(Up, W, b, 10, u)
        wm = hog.top_windows(Um, W, b, 10, u)
        same_top = all(np.array_equal(wp[k], win[k]) and np.array_equal(wm[k], win[k])
                       for k in ("f", "k", "r", "c"))
        if not (same_top and _same_state(_state(Up, W, b, win, u), s0)
                and _same_state(_state(Um, W, b, win, u), s0)):
            continue
        fd = (hog.topk_objective(Up, W, b, win, u) - hog.topk_objective(Um, W, b, win, u)) / (2 * hstep)
        assert abs(fd - dU[y, x]) <= 1e-6 * abs(dU[y, x]) + 1e-8, (y, x, fd, dU[y, x])
        checked += 1
    assert checked >= 48
