"""P10: the vectorised float64 oracle against a pure-Python loop statement
of the same method (exact-rational taps, atan2 orientation, tent-weight
votes, explicit loops), on small frames."""
import numpy as np
import pytest

from oracle import brute, hog


@pytest.mark.parametrize("seed,h,w,u", [(21, 96, 104, 1), (22, 88, 99, 1), (23, 50, 60, 2)])
def test_pyramid_levels_match_brute(seed, h, w, u):
    rng = np.random.default_rng(seed)
    U = rng.integers(0, 256, (h, w)).astype(np.uint8)
    got = hog.pyramid(h, w, u)
    want = brute.pyramid_sizes(h, w, u)
    assert [(l.h, l.w) for l in got] == [(hk, wk) for _, _, hk, wk in want]
    Ul = U.tolist()
    for lv, (_, s, hk, wk) in zip(got, want):
        assert np.array_equal(hog.resample(U, lv), np.array(brute.level_image(Ul, s, hk, wk)))


@pytest.mark.parametrize("seed", [31, 32])
def test_hist_and_features_match_brute(seed):
    rng = np.random.default_rng(seed)
    U = rng.integers(0, 256, (58, 67)).astype(np.float64)
    L = hog.resample(U, hog.Level(0, 1, 1, 58, 67))
    hist = hog.cell_histograms(L)
    hb = np.array(brute.level_hist(L.tolist()))
    assert np.allclose(hist, hb, rtol=1e-12, atol=1e-9)
    F = hog.features_from_hist(hist)
    Fb = np.array(brute.features(hb.tolist()))
    assert np.allclose(F, Fb, rtol=1e-12, atol=1e-12)


def test_scores_match_brute():
    rng = np.random.default_rng(41)
    F = rng.uniform(0, 0.4, (12, 14, 31))
    W = rng.normal(0, 0.1, (2, 10, 10, 31))
    b = [-0.5, 0.3]
    S = hog.window_scores(F, W, b)
    Sb = np.array(brute.scores(F.tolist(), W.tolist(), b))
    assert np.allclose(S, Sb, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed,u", [(51, 1), (52, 2)])
def test_detect_matches_brute(seed, u):
    """End to end on a tiny frame: candidates, boxes and NMS.  The filter
    is scaled so that a good share of windows pass the threshold."""
    rng = np.random.default_rng(seed)
    if u == 1:
        U = rng.integers(0, 256, (104, 112)).astype(np.uint8)
    else:
        U = rng.integers(0, 256, (56, 60)).astype(np.uint8)
    W = rng.normal(0, 0.1, (2, 10, 10, 31))
    b = np.array([0.2, -0.1])
    got = hog.detect(U, W, b, 0.0, 0.5, u)
    want = brute.detect(U.tolist(), W.tolist(), b.tolist(), 0.0, 0.5, u)
    assert len(got) == len(want) > 0
    for g, wv in zip(got, want):
        assert (int(g["f"]), int(g["k"]), int(g["r"]), int(g["c"])) == wv[1:5]
        assert (int(g["x0"]), int(g["y0"]), int(g["x1"]), int(g["y1"])) == wv[5]
        assert abs(g["score"] - wv[0]) <= 1e-12
