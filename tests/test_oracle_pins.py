"""Pins of the float64 oracle against what the paper and mathematics fix.

None of these re-types the oracle's own formulas: each one checks a
closed form, an invariant, a special case or an independent formulation.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import hog

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------ constants
def test_paper_constants():
    g = _gold("paper_constants.json")
    assert hog.CELL == g["cell_px"]["value"]
    assert hog.NBINS == g["signed_bins"]["value"]
    assert hog.NFEAT == g["features"]["value"] == sum(g["features"]["parts"])
    assert hog.WIN == g["window_cells"]["value"]
    assert hog.WIN * hog.CELL == g["window_px"]["value"]
    assert hog.WIN * hog.WIN * hog.NFEAT == g["window_weights"]["value"]
    assert (hog.SCALE_NUM, hog.SCALE_DEN) == (g["scale_step"]["num"], g["scale_step"]["den"])
    assert hog.MIN_SIDE == g["min_side_px"]["value"]
    t = g["classifier_tile"]
    assert t["block_cols"] + hog.WIN - 1 == t["needed_cols"]


def test_orientation_table_exact_and_mirrored():
    c, s = hog.orientation_table()
    for o in range(9):
        a = o * math.pi / 9
        assert abs(c[o] - math.cos(a)) <= 2 * np.spacing(1.0)
        assert abs(s[o] - math.sin(a)) <= 2 * np.spacing(1.0)
    for o in range(1, 5):
        assert c[9 - o] == -c[o] and s[9 - o] == s[o]
    assert c[0] == 1.0 and s[0] == 0.0 and c[3] == 0.5


# ------------------------------------------------------------- pyramid
def test_pyramid_sizes_golden():
    g = _gold("pyramid_levels.json")
    for key in ("240x320_u1", "480x640_u1", "80x80_u1"):
        h, w = map(int, key.split("_")[0].split("x"))
        assert [[lv.h, lv.w] for lv in hog.pyramid(h, w)] == g[key]
    lv = hog.pyramid(480, 640)
    assert [l.rows * l.cols for l in lv] == g["480x640_u1_windows_per_level"]
    big = hog.pyramid(1080, 1920, 2)
    assert len(big) == g["1080x1920_u2_n_levels"]
    assert [big[0].h, big[0].w] == g["1080x1920_u2_first"]
    assert [big[-1].h, big[-1].w] == g["1080x1920_u2_last"]


@pytest.mark.parametrize("h,w,u", [(240, 320, 1), (480, 640, 1), (97, 331, 1), (100, 120, 2), (1080, 1920, 2)])
def test_pyramid_stop_rule(h, w, u):
    lv = hog.pyramid(h, w, u)
    assert min(lv[-1].h, lv[-1].w) >= 80
    s_next = u * (5 / 6) ** (lv[-1].k + 1)
    assert min(math.floor(h * s_next + 1e-9), math.floor(w * s_next + 1e-9)) < 80
    for l in lv:
        assert abs(l.h - h * l.p / l.q) < 1 and abs(l.w - w * l.p / l.q) < 1


def test_pyramid_too_small():
    assert hog.pyramid(79, 500) == []
    assert len(hog.pyramid(80, 80)) == 1


def test_resample_identity_and_constant():
    rng = np.random.default_rng(5)
    U = rng.integers(0, 256, (120, 150)).astype(np.uint8)
    lv = hog.pyramid(120, 150)
    assert np.array_equal(hog.resample(U, lv[0]), U.astype(np.float64))
    C = np.full((120, 150), 77, np.uint8)
    for l in lv:
        assert np.all(hog.resample(C, l) == 77.0)
    for l in hog.pyramid(120, 150, 2):
        assert np.all(hog.resample(C, l) == 77.0)


@pytest.mark.parametrize("u", [1, 2])
def test_resample_reproduces_linear_ramp(u):
    """Bilinear sampling reproduces a linear function at the pixel-centre
    aligned source coordinate (i + 1/2)/s - 1/2, up to the 1/256 weight
    quantisation (at most 1/512 px), away from the clamped border."""
    H, W = 200, 260
    U = np.tile(np.arange(W, dtype=np.float64), (H, 1))
    for l in hog.pyramid(H, W, u):
        L = hog.resample(U, l)
        xs = (np.arange(l.w) + 0.5) * l.q / l.p - 0.5
        inner = (xs >= 0) & (xs <= W - 1)
        err = np.abs(L[l.h // 2, inner] - xs[inner])
        assert err.max() <= 1 / 512 + 1e-12


def test_resample_values_exact_dyadic():
    rng = np.random.default_rng(6)
    U = rng.integers(0, 256, (130, 170)).astype(np.uint8)
    for l in hog.pyramid(130, 170, 2):
        L = hog.resample(U, l)
        q = L * 65536.0
        assert np.array_equal(q, np.round(q)) and L.max() <= 255 and L.min() >= 0


def test_resample_adjoint():
    rng = np.random.default_rng(7)
    H, W = 150, 190
    x = rng.standard_normal((H, W))
    for u in (1, 2):
        for l in hog.pyramid(H, W, u):
            y = rng.standard_normal((l.h, l.w))
            lhs = np.sum(hog.resample(x, l) * y)
            rhs = np.sum(x * hog.resample_transpose(y, l, H, W))
            assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


# ------------------------------------------------------- P1 constant
def test_constant_image_all_zero():
    U = np.full((160, 200), 123, np.uint8)
    W = np.random.default_rng(0).normal(0, 0.1, (2, 10, 10, 31))
    b = np.array([-0.5, 0.25])
    for lv, F in hog.pyramid_features(U):
        L = hog.resample(U, lv)
        gx, gy = hog.gradients(L)
        assert not gx.any() and not gy.any()
        assert not hog.cell_histograms(L).any()
        assert not F.any()
        S = hog.window_scores(F, W, b)
        assert np.all(S == b[:, None, None])


# ----------------------------------------------------- P2 ramp bins
def _bin_by_angle(gx, gy):
    if gx == 0:
        return 4 if gy > 0 else 13
    deg = math.degrees(math.atan2(gy, gx)) % 360
    return int((deg + 10) // 20) % 18


def _ramp(a, b, H=96, W=96):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return 128 + a * (x - W / 2) + b * (y - H / 2)


@pytest.mark.parametrize("a,b", [(a, b) for a in range(-3, 4) for b in range(-3, 4) if (a, b) != (0, 0)])
def test_ramp_bin_is_nearest_direction(a, b):
    U = _ramp(a, b)
    gx, gy = hog.gradients(U)
    assert np.all(gx[1:-1, 1:-1] == 2 * a) and np.all(gy[1:-1, 1:-1] == 2 * b)
    bins = hog.orientation_bins(gx[1:-1, 1:-1], gy[1:-1, 1:-1])
    assert np.all(bins == _bin_by_angle(2 * a, 2 * b))


def test_named_edge_directions():
    # (gx, gy) -> bin, y pointing down, angle measured from +x towards +y
    cases = {(1, 0): 0, (2, 1): 1, (1, 1): 2, (1, 2): 3, (0, 1): 4, (-1, 2): 6,
             (-1, 1): 7, (-1, 0): 9, (-1, -1): 11, (0, -1): 13, (1, -2): 15, (1, -1): 16}
    for (gx, gy), want in cases.items():
        got = hog.orientation_bins(np.array([float(gx)]), np.array([float(gy)]))[0]
        assert got == want, (gx, gy, got, want)


# -------------------------------------------- P3 closed-form features
@pytest.mark.parametrize("a,b", [(1, 0), (2, 1), (1, 1), (-1, 2), (0, -1), (3, -2)])
def test_ramp_closed_form_features(a, b):
    U = _ramp(a, b)
    lv = hog.pyramid(96, 96)[0]
    L = hog.resample(U, lv)
    hist = hog.cell_histograms(L)
    F = hog.features_from_hist(hist)
    mag = 2 * math.hypot(a, b)
    bn = _bin_by_angle(2 * a, 2 * b)
    cy = 12
    for i in range(1, cy - 1):
        for j in range(1, cy - 1):
            want = np.zeros(18)
            want[bn] = 64 * mag
            assert np.allclose(hist[i, j], want, rtol=1e-13, atol=1e-12)
    want = np.zeros(31)
    want[bn] = 0.4
    want[18 + bn % 9] = 0.4
    want[27:] = 0.2 / math.sqrt(18)
    for i in range(2, cy - 2):
        for j in range(2, cy - 2):
            assert np.allclose(F[i, j], want, rtol=0, atol=1e-12)


# ------------------------------------ unclipped normalisation, by hand
def test_unclipped_normaliser_hand_pattern():
    """A 3x3-cell histogram in which no normalised value reaches the 0.2
    clip, so the 1e-4 term and the grouping of the energies into four 2x2
    blocks set the centre cell's features.  Centre cell (1, 1): all 18
    bins = v, so its energy is 9 (2v)^2 = 36 v^2.  Top-left cell (0, 0):
    one bin = t, energy t^2.  Every other cell is empty.  The centre's
    blocks are (-1,-1) = {(0,0), (0,1), (1,0), (1,1)}, which holds both
    energies, and (-1,+1), (+1,-1), (+1,+1), which hold only its own:
      n_0 = (36 v^2 + t^2 + 1e-4)^-1/2,  n_1 = n_2 = n_3 = (36 v^2 + 1e-4)^-1/2.
    With v = 1e-3 and t = 5e-3: n_0 = 1/sqrt(1.61e-4) = 78.8110...,
    n_k = 1/sqrt(1.36e-4) = 85.7492..., so v n_k ~ 0.08 and 2 v n_k ~ 0.17,
    all below 0.2, and
      signed   F[b]      = (v n_0 + 3 v n_1) / 2                = 0.168029...
      unsigned F[18 + o] = (2 v n_0 + 6 v n_1) / 2              = 0.336058...
      energy   F[27]     = 18 v n_0 / sqrt(18) = sqrt(18) v n_0 = 0.334366...
               F[28..30] = sqrt(18) v n_1                       = 0.363803...
    (eps outside the square root, or a missing eps, or blocks of a
    different shape give other numbers)."""
    v, t = 1e-3, 5e-3
    hist = np.zeros((3, 3, 18))
    hist[1, 1, :] = v
    hist[0, 0, 5] = t
    F = hog.features_from_hist(hist)[1, 1]
    n0 = 1 / math.sqrt(36 * v * v + t * t + 1e-4)
    n1 = 1 / math.sqrt(36 * v * v + 1e-4)
    assert abs(n0 - 78.81104062391006) < 1e-9 and abs(n1 - 85.74929257125441) < 1e-9
    assert np.allclose(F[:18], 0.5 * (v * n0 + 3 * v * n1), rtol=0, atol=1e-15)
    assert np.allclose(F[18:27], 0.5 * (2 * v * n0 + 6 * v * n1), rtol=0, atol=1e-15)
    assert abs(F[27] - math.sqrt(18) * v * n0) < 1e-15
    assert np.allclose(F[28:], math.sqrt(18) * v * n1, rtol=0, atol=1e-15)
    assert abs(F[0] - 0.16802946) < 1e-8 and abs(F[27] - 0.33436693) < 1e-8 and abs(F[28] - 0.36380344) < 1e-8


def test_unclipped_low_contrast_ramp_features():
    """A horizontal ramp of slope 1e-5 grey levels per pixel: gx = 2e-5 and
    gy = 0 everywhere inside, so every interior cell holds h = 64 * 2e-5 =
    1.28e-3 in bin 0 (the tent weights of a cell sum to 64) and energy h^2;
    an interior cell's four blocks each hold 4 h^2.  Then
    h n = h / sqrt(4 h^2 + 1e-4) = 0.1240012... < 0.2, unclipped, and
      F[0] = F[18] = 4 h n / 2 = 2 h n,   F[27 + k] = h n / sqrt(18),
    every other feature 0.  Through the whole image path: resample,
    gradients, orientation, bilinear votes, energies, blocks, features."""
    H, W = 96, 120
    U = 128.0 + 1e-5 * np.tile(np.arange(W, dtype=np.float64), (H, 1))
    lv = hog.pyramid(H, W)[0]
    F = hog.level_features(U, lv)
    h = 64 * 2e-5
    hn = h / math.sqrt(4 * h * h + 1e-4)
    assert abs(hn - 0.12400121) < 1e-8
    want = np.zeros(31)
    want[0] = want[18] = 2 * hn
    want[27:] = hn / math.sqrt(18)
    for i in range(2, lv.cy - 2):
        for j in range(2, lv.cx - 2):
            assert np.allclose(F[i, j], want, rtol=1e-9, atol=1e-14), (i, j)


# ----------------------------------------------- hinge loss, by hand
def test_hinge_loss_hand_case():
    """Scores 2, 0.5, -0.3, -2, 1 with labels +1, +1, -1, -1, +1: the
    margins 1 - y s are -1, 0.5, 0.7, -1, 0, so the hinge terms are
    0, 0.5, 0.7, 0, 0 and their mean is 1.2 / 5 = 0.24.  A filter of 3100
    weights 0.01 has ||W||^2 = 0.31, times 1e-4 = 3.1e-5: loss 0.240031.
    The score gradient is -y_i / 5 where y_i s_i < 1 (the second and third
    score), and 0 elsewhere, also at the kink y s = 1 (the fifth)."""
    S = np.array([2.0, 0.5, -0.3, -2.0, 1.0])
    y = np.array([1.0, 1.0, -1.0, -1.0, 1.0])
    W = np.full((1, 10, 10, 31), 0.01)
    assert abs(hog.hinge_loss(S, y, W, 1e-4) - 0.240031) < 1e-15
    assert np.array_equal(hog.hinge_dscore(S, y), np.array([0.0, -0.2, 0.2, 0.0, 0.0]))


# ------------------------------------ top windows below the threshold
def test_top_windows_include_sub_threshold_windows():
    """On a constant frame every feature is 0, so every window of filter f
    scores b_f.  With b = (0.3, -0.5), filter 0's windows are the only
    candidates (score > 0); the top k for k beyond their count continue
    with filter 1's windows, all below the threshold, in (level, row,
    column) order.  The 120x160 pyramid has levels of 6x11, 3x7 and 1x4
    window anchors: 91 windows per filter."""
    U = np.full((120, 160), 77, np.uint8)
    W = np.random.default_rng(3).normal(0, 0.1, (2, 10, 10, 31))
    b = np.array([0.3, -0.5])
    assert [(l.rows, l.cols) for l in hog.pyramid(120, 160)] == [(6, 11), (3, 7), (1, 4)]
    cand = hog.candidates(U, W, b)
    assert len(cand) == 91 and np.all(cand["f"] == 0)
    top = hog.top_windows(U, W, b, k=96)
    order = [(0, k, r, c) for k, (R, C) in enumerate([(6, 11), (3, 7), (1, 4)])
             for r in range(R) for c in range(C)]
    order += [(1, 0, 0, c) for c in range(5)]
    assert list(zip(top["f"].tolist(), top["k"].tolist(), top["r"].tolist(), top["c"].tolist())) == order
    assert np.all(top["score"][:91] == 0.3) and np.all(top["score"][91:] == -0.5)


# ------------------------------------------------------ P4 cell mass
def _tent_matrix(n_cells, n_pix):
    c = (np.arange(n_pix) + 0.5) / 8 - 0.5
    return np.maximum(0.0, 1.0 - np.abs(c[None, :] - np.arange(n_cells)[:, None]))


def test_cell_mass_equals_tent_weighted_magnitude():
    rng = np.random.default_rng(11)
    U = rng.integers(0, 256, (150, 175)).astype(np.uint8)
    for lv in hog.pyramid(150, 175):
        L = hog.resample(U, lv)
        gx, gy = hog.gradients(L)
        mag = np.sqrt(gx * gx + gy * gy)[:8 * lv.cy, :8 * lv.cx]
        want = _tent_matrix(lv.cy, 8 * lv.cy) @ mag @ _tent_matrix(lv.cx, 8 * lv.cx).T
        got = hog.cell_histograms(L).sum(-1)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-9)


# ------------------------------------------------------- P5 symmetries
SIGNED_H = np.array([(9 - b) % 18 for b in range(18)])
UNSIGNED_H = np.array([(9 - o) % 9 for o in range(9)])
SIGNED_V = np.array([(18 - b) % 18 for b in range(18)])


def _perm_h():
    p = np.empty(31, np.int64)
    p[:18] = SIGNED_H
    p[18:27] = 18 + UNSIGNED_H
    p[27:] = 27 + np.array([1, 0, 3, 2])
    return p


def _perm_v():
    p = np.empty(31, np.int64)
    p[:18] = SIGNED_V
    p[18:27] = 18 + UNSIGNED_H
    p[27:] = 27 + np.array([2, 3, 0, 1])
    return p


def _level0(U):
    lv = hog.pyramid(*U.shape)[0]
    L = hog.resample(U, lv)
    hist = hog.cell_histograms(L)
    return lv, hist, hog.features_from_hist(hist)


def test_horizontal_flip_permutes_bins_and_features():
    rng = np.random.default_rng(12)
    U = rng.uniform(0, 255, (104, 120))        # continuous values: no exact ties
    _, h1, F1 = _level0(U)
    _, h2, F2 = _level0(U[:, ::-1])
    p = _perm_h()
    # F2[i][cx-1-j][p[ch]] == F1[i][j][ch]
    assert np.allclose(h2[:, ::-1][..., SIGNED_H], h1, rtol=1e-12, atol=1e-10)
    assert np.allclose(F2[:, ::-1][..., p], F1, rtol=1e-12, atol=1e-12)
    W = rng.normal(0, 0.1, (1, 10, 10, 31))
    Wf = np.empty_like(W)
    Wf[0][:, :, p] = W[0][:, ::-1, :]          # W'[dr][dc'][p[ch]] = W[dr][9-dc'][ch]
    S1 = hog.window_scores(F1, W, [0.1])
    S2 = hog.window_scores(F2, Wf, [0.1])
    assert np.allclose(S2[:, :, ::-1], S1, rtol=1e-12, atol=1e-12)


def test_vertical_flip_and_contrast_inversion():
    rng = np.random.default_rng(13)
    U = rng.uniform(0, 255, (96, 112))
    _, h1, F1 = _level0(U)
    _, h2, F2 = _level0(U[::-1, :])
    assert np.allclose(h2[::-1][..., SIGNED_V], h1, rtol=1e-12, atol=1e-10)
    assert np.allclose(F2[::-1][..., _perm_v()], F1, rtol=1e-12, atol=1e-12)
    _, h3, F3 = _level0(255.0 - U)
    inv = np.array([(b + 9) % 18 for b in range(18)])
    assert np.allclose(h3[..., inv], h1, rtol=1e-12, atol=1e-10)
    assert np.allclose(F3[..., 18:], F1[..., 18:], rtol=1e-12, atol=1e-12)
    assert np.allclose(F3[..., :18][..., inv], F1[..., :18], rtol=1e-12, atol=1e-12)


# ------------------------------------------------ P6 scale invariance
def test_contrast_scale_and_offset_invariance():
    rng = np.random.default_rng(14)
    U = rng.integers(20, 200, (112, 128)).astype(np.float64)
    _, _, F = _level0(U)
    _, _, F2 = _level0(2.0 * U)
    _, _, F3 = _level0(U + 37.0)
    assert np.allclose(F2, F, rtol=0, atol=1e-8)
    assert np.array_equal(F3, F)


# ----------------------------------------------------- P9 one-hot
def test_one_hot_filter_reads_feature():
    rng = np.random.default_rng(15)
    F = rng.uniform(0, 0.4, (14, 17, 31))
    for dr, dc, ch in [(0, 0, 0), (9, 9, 30), (3, 7, 12), (5, 0, 27)]:
        W = np.zeros((1, 10, 10, 31))
        W[0, dr, dc, ch] = 1.0
        S = hog.window_scores(F, W, [-0.5])
        assert np.array_equal(S[0], F[dr:dr + 5, dc:dc + 8, ch] - 0.5)
    W1, W2 = rng.normal(0, 1, (2, 1, 10, 10, 31))
    lin = hog.window_scores(F, W1 + W2, [0.0])
    assert np.allclose(lin, hog.window_scores(F, W1, [0.0]) + hog.window_scores(F, W2, [0.0]),
                       rtol=1e-12, atol=1e-12)


# ------------------------------------------------------ boxes / NMS
def test_window_box_level0_and_scaled():
    lv = hog.pyramid(480, 640)
    assert hog.window_box(lv[0], 3, 5) == (40, 24, 120, 104)
    x0, y0, x1, y1 = hog.window_box(lv[1], 0, 0)     # s = 5/6: 80 px -> 96 px
    assert (x0, y0, x1, y1) == (0, 0, 96, 96)
    x0, _, x1, _ = hog.window_box(lv[2], 0, 1)       # 8*36/25 = 11.52 -> 12; 88*36/25 = 126.72 -> 127
    assert (x0, x1) == (12, 127)


def _cands(boxes, scores, f=None):
    c = np.zeros(len(boxes), hog.CAND_DTYPE)
    for i, (bx, s) in enumerate(zip(boxes, scores)):
        c[i]["score"] = s
        c[i]["c"] = i
        c[i]["f"] = 0 if f is None else f[i]
        c[i]["x0"], c[i]["y0"], c[i]["x1"], c[i]["y1"] = bx
    return c


def test_nms_hand_cases():
    # same-level neighbours 1 and 2 cells apart: IoU 0.8182 and 0.6667 -> suppressed;
    # 4 cells apart: 48*80 / (2*6400 - 3840) = 0.4286 -> kept
    a, b1, b2, b4 = (0, 0, 80, 80), (8, 0, 88, 80), (16, 0, 96, 80), (32, 0, 112, 80)
    assert len(hog.nms(_cands([a, b1], [2.0, 1.0]))) == 1
    assert len(hog.nms(_cands([a, b2], [2.0, 1.0]))) == 1
    assert len(hog.nms(_cands([a, b4], [2.0, 1.0]))) == 2
    # exact IoU = 1/2 is not suppressed (strict >): I = 20*40 = 800,
    # U = 1200 + 1200 - 800 = 1600
    k = hog.nms(_cands([(0, 0, 30, 40), (10, 0, 40, 40)], [1.0, 0.5]))
    assert len(k) == 2
    # suppression chain: A > B > C, A suppresses B, B would suppress C but B is gone
    A, B, C = (0, 0, 80, 80), (16, 0, 96, 80), (32, 0, 112, 80)
    kept = hog.nms(_cands([A, B, C], [3.0, 2.0, 1.0]))
    assert sorted(kept["c"].tolist()) == [0, 2]


def test_nms_properties_random():
    rng = np.random.default_rng(16)
    n = 400
    x0 = rng.integers(0, 300, n)
    y0 = rng.integers(0, 200, n)
    sz = rng.integers(60, 140, n)
    boxes = list(zip(x0, y0, x0 + sz, y0 + sz))
    scores = rng.normal(size=n)
    c = _cands(boxes, scores)
    kept = hog.nms(c)

    def iou2(p, q):
        iw = max(0, min(p["x1"], q["x1"]) - max(p["x0"], q["x0"]))
        ih = max(0, min(p["y1"], q["y1"]) - max(p["y0"], q["y0"]))
        inter = iw * ih
        union = (p["x1"] - p["x0"]) * (p["y1"] - p["y0"]) + (q["x1"] - q["x0"]) * (q["y1"] - q["y0"]) - inter
        return 2 * inter > union

    for i in range(len(kept)):
        for j in range(i + 1, len(kept)):
            assert not iou2(kept[i], kept[j])
    kept_ids = set(kept["c"].tolist())
    for cand in c:
        if cand["c"] in kept_ids:
            continue
        assert any(iou2(cand, k) and (k["score"] > cand["score"]) for k in kept)
    assert np.array_equal(hog.nms(kept), kept)
    perm = rng.permutation(n)
    assert np.array_equal(hog.nms(c[perm]), kept)
    assert np.all(np.diff(kept["score"]) <= 0)


# ------------------------------------- separable (row / column) filters
def test_separable_one_hot_factors_read_one_feature():
    """Row factor e_(dc0, ch0) and column factor e_(dr0, ch0): the filter is
    one-hot at (dr0, dc0, ch0), so the score reads F[r + dr0][c + dc0][ch0]
    (a transposed or swapped factor reads another cell)."""
    rng = np.random.default_rng(41)
    F = rng.random((14, 17, 31))
    for dr0, dc0, ch0 in ((0, 0, 0), (3, 7, 12), (9, 2, 30), (5, 9, 27)):
        row = np.zeros((1, 1, 10, 31))
        col = np.zeros((1, 1, 10, 31))
        row[0, 0, dc0, ch0] = 1.0
        col[0, 0, dr0, ch0] = 1.0
        S = hog.window_scores(F, hog.separable_filters(row, col), np.array([0.25]))
        assert np.array_equal(S[0], F[dr0:dr0 + 5, dc0:dc0 + 8, ch0] + 0.25)


def test_separable_full_rank_svd_reproduces_filter():
    """numpy's SVD of each channel's 10x10 weight matrix W[:, :, ch] =
    U diag(s) V^T gives rank-10 factors col_i = s_i U[:, i] (over dr) and
    row_i = V^T[i, :] (over dc); their sum is the filter again."""
    rng = np.random.default_rng(42)
    W = rng.normal(0, 0.1, (3, 10, 10, 31))
    row = np.zeros((3, 10, 10, 31))
    col = np.zeros((3, 10, 10, 31))
    for f in range(3):
        for ch in range(31):
            U, sv, Vt = np.linalg.svd(W[f, :, :, ch])
            for i in range(10):
                col[f, i, :, ch] = sv[i] * U[:, i]
                row[f, i, :, ch] = Vt[i, :]
    assert np.allclose(hog.separable_filters(row, col), W, rtol=0, atol=1e-14)


def test_separable_two_pass_equals_filter_scores():
    """The paper's two passes written out as loops on a tiny feature map
    (row filter into a scratch image per channel, then the column filter,
    then the sum over channels) equal the scores of the combined filter."""
    rng = np.random.default_rng(43)
    F = rng.random((12, 13, 31))
    row = rng.normal(0, 0.1, (2, 2, 10, 31))
    col = rng.normal(0, 0.1, (2, 2, 10, 31))
    b = np.array([0.1, -0.2])
    S = hog.window_scores(F, hog.separable_filters(row, col), b)
    R, C = 3, 4
    for f in range(2):
        for r in range(R):
            for c in range(C):
                tot = b[f]
                for i in range(2):
                    for ch in range(31):
                        scratch = [sum(row[f, i, dc, ch] * F[y, c + dc, ch] for dc in range(10))
                                   for y in range(r, r + 10)]
                        tot += sum(col[f, i, dr, ch] * scratch[dr] for dr in range(10))
                assert abs(S[f, r, c] - tot) < 1e-12


# ------------------------------------- analysed levels and search regions
def test_level_skipping_worked_example():
    """Sec. V-A: 640x480 frames with faces of at least 20 % of the image
    skip the largest scale.  The minimum face (20 % of each side) and its
    size one 5/6 step down are the paper's numbers; the levels kept by
    face_levels at that minimum are every level but the first."""
    g = _gold("level_skipping.json")
    w, h = g["frame_wh"]["value"]
    frac = g["min_face_fraction"]["value"]
    fw, fh = round(frac * w), round(frac * h)
    assert [fw, fh] == g["min_face_wh_level0"]["value"]
    assert [round(fw * 5 / 6), round(fh * 5 / 6)] == g["min_face_wh_level1"]["value"]
    levels = hog.pyramid(h, w)
    kept = [lv.k for lv in hog.face_levels(levels, min(fw, fh))]
    skipped = sorted(set(lv.k for lv in levels) - set(kept))
    assert skipped == g["skipped_levels"]["value"]
    # the smallest face spans exactly one window at the first kept level
    assert round(min(fw, fh) * levels[kept[0]].p / levels[kept[0]].q) == hog.WIN * hog.CELL


def test_level_skipping_keeps_analysed_work_flat():
    """Sec. VI (scalability): with the face at least 20 % of the frame
    height, the skipped scales grow with the frame, and the analysed
    pyramid of 1280x960 and 2560x1920 frames stays near the 640x480 one
    (the paper reports feature and classifier time independent
    of the frame size).  The first kept level lands within one 5/6 step
    of the scale at which the smallest face is window-sized, so the
    analysed pyramids stay within a factor (6/5)^2 of each other; without
    skipping they grow about 4x per step."""
    sizes = [(480, 640), (960, 1280), (1920, 2560)]
    px = []
    full = []
    for h, w in sizes:
        lv = hog.pyramid(h, w)
        px.append(sum(l.h * l.w for l in hog.face_levels(lv, h // 5)))
        full.append(sum(l.h * l.w for l in lv))
    assert max(px) < 1.44 * min(px), px
    assert full[1] > 3.5 * full[0] and full[2] > 3.5 * full[1]


def test_level_skipping_boundary_is_exact():
    """A level is kept exactly when its window spans min_face frame px or
    more: 80 * (6/5)^k >= min_face.  At 640x480: 80 keeps level 0, 81
    skips it; 96 keeps level 1 (96 px window), 97 skips it too."""
    lv = hog.pyramid(480, 640)
    assert [l.k for l in hog.face_levels(lv, 0)] == list(range(10))
    assert hog.face_levels(lv, 80)[0].k == 0
    assert hog.face_levels(lv, 81)[0].k == 1
    assert hog.face_levels(lv, 96)[0].k == 1
    assert hog.face_levels(lv, 97)[0].k == 2
    # at 2x upsampling the first level's window spans 40 frame px
    lv2 = hog.pyramid(240, 320, 2)
    assert hog.face_levels(lv2, 40)[0].k == 0 and hog.face_levels(lv2, 41)[0].k == 1


def _cands_clip(seed=5):
    from paper_2006_00816_amd import synth
    wl = synth.config1(seed=seed, n=1)
    return wl.frames[0], wl.W, wl.b


def test_region_whole_frame_is_no_region():
    U, W, b = _cands_clip()
    U = U[::2, ::2].copy()   # 240x320 keeps the float64 oracle quick
    a = hog.candidates(U, W, b)
    c = hog.candidates(U, W, b, region=(0, 0, 320, 240, 0, hog.HUGE_LEVEL))
    assert len(a) > 100 and np.array_equal(a, c)
    assert len(hog.candidates(U, W, b, region=(0, 0, 0, 0, 0, hog.HUGE_LEVEL))) == 0
    assert len(hog.candidates(U, W, b, region=(0, 0, 320, 240, 99, 99))) == 0


def test_region_hand_cases():
    """Level-0 window (0, 0) of a 240x320 frame covers frame pixels
    [0, 80) x [0, 80); every box of a later level is at least 96 px wide,
    and the level-0 window (0, 1) starts at x = 8.  So the region
    [0, 80) x [0, 80) searches exactly window (0, 0) of level 0, and
    [0, 88) x [0, 80) adds window (0, 1)."""
    lv = hog.pyramid(240, 320)
    assert hog.window_box(lv[0], 0, 0) == (0, 0, 80, 80)
    assert hog.window_box(lv[0], 0, 1) == (8, 0, 88, 80)
    assert all(int(hog.window_box(l, 0, 0)[2]) >= 96 for l in lv[1:])
    m = [hog.window_in_region(l, *np.meshgrid(np.arange(l.rows), np.arange(l.cols), indexing="ij"),
                              (0, 0, 80, 80, 0, 99)) for l in lv]
    assert m[0][0, 0] and m[0].sum() == 1 and all(x.sum() == 0 for x in m[1:])
    m = hog.window_in_region(lv[0], *np.meshgrid(np.arange(lv[0].rows), np.arange(lv[0].cols), indexing="ij"),
                             (0, 0, 88, 80, 0, 0))
    assert sorted(zip(*np.nonzero(m))) == [(0, 0), (0, 1)]


def test_region_monotone_and_inside():
    """A region inside another searches a subset of its windows; every
    candidate's box lies inside its region and level range."""
    U, W, b = _cands_clip(6)
    U = U[::2, ::2].copy()
    big = (40, 20, 300, 230, 0, 4)
    small = (90, 50, 250, 200, 1, 3)
    A = hog.candidates(U, W, b, region=big)
    B = hog.candidates(U, W, b, region=small)
    key = lambda a: set(zip(a["f"], a["k"], a["r"], a["c"]))
    assert 0 < len(B) < len(A) and key(B) <= key(A)
    for a, reg in ((A, big), (B, small)):
        assert np.all(a["x0"] >= reg[0]) and np.all(a["y0"] >= reg[1])
        assert np.all(a["x1"] <= reg[2]) and np.all(a["y1"] <= reg[3])
        assert np.all(a["k"] >= reg[4]) and np.all(a["k"] <= reg[5])


def test_min_face_equals_dropping_levels():
    """Skipping levels removes exactly the candidates of the skipped
    levels and keeps the others bit for bit."""
    U, W, b = _cands_clip(7)
    U = U[::2, ::2].copy()
    a = hog.candidates(U, W, b)
    c = hog.candidates(U, W, b, min_face=61)     # 240x320: 80 (6/5)^k >= 61 keeps all; 81 drops level 0
    assert np.array_equal(a, c)
    d = hog.candidates(U, W, b, min_face=81)
    assert np.array_equal(d, a[a["k"] >= 1])


def test_track_region_hand_cases():
    kept = np.zeros(2, hog.CAND_DTYPE)
    kept["x0"], kept["y0"], kept["x1"], kept["y1"], kept["k"] = (100, 300), (50, 10), (196, 396), (146, 106), (2, 0)
    assert hog.track_region(kept, 480, 640, 16, 1) == (84, 34, 212, 162, 1, 3)
    kept["x0"][0], kept["y0"][0], kept["x1"][0], kept["y1"][0], kept["k"][0] = 5, 3, 635, 470, 0
    assert hog.track_region(kept, 480, 640, 16, 2) == (0, 0, 640, 480, 0, 2)
    assert hog.track_region(kept[:0], 480, 640, 16, 2) == (0, 0, 640, 480, 0, hog.HUGE_LEVEL)


# -------------------------------------------------- recursive pyramid (R20)
def test_cascade_sizes_hand_derived():
    """Recursive floor(5x/6) sizes of a 640x480 frame, worked by hand:
    533 = floor(3200/6), 444 = floor(2665/6), ... down to 122x91 (the next,
    101x75, is below the window).  They differ from the direct sizes by a
    pixel from level 4 on (230 against 231)."""
    want = [(480, 640), (400, 533), (333, 444), (277, 370), (230, 308), (191, 256), (159, 213), (132, 177),
            (110, 147), (91, 122)]
    assert [(l.h, l.w) for l in hog.pyramid_cascade(480, 640)] == want
    direct = [(l.h, l.w) for l in hog.pyramid(480, 640)]
    assert direct[:4] == want[:4] and direct[4] == (231, 308)
    assert [(l.h, l.w) for l in hog.pyramid_cascade(240, 320, 2)] == want
    assert [l.k for l in hog.pyramid_cascade(79, 500)] == []


def test_cascade_taps_exact_fractions():
    """A 5/6 step puts output sample i at (12 i + 1)/10 of the input: the
    fractional parts cycle through 1/10, 3/10, 5/10, 7/10, 9/10, whose
    nearest multiples of 1/256 are 26, 77, 128, 179 and 230."""
    i0, i1, a = hog.cascade_taps(10, 12)
    assert list(a) == [26, 77, 128, 179, 230] * 2
    assert list(i0) == [0, 1, 2, 3, 4, 6, 7, 8, 9, 10] and list(i1) == [1, 2, 3, 4, 5, 7, 8, 9, 10, 11]


def test_cascade_constant_and_ramp():
    """A constant frame stays constant at every level; a horizontal ramp
    U = 2x + 20 is reproduced at level 1 within the rounding to grey levels
    (1/2) plus the weight rounding (1/512 of a 2-unit step)."""
    for lv, L in hog.cascade_levels(np.full((200, 260), 77, np.uint8)):
        assert np.all(L == 77), lv.k
    U = np.tile(2 * np.arange(110) + 20, (180, 1)).astype(np.uint8)
    (l0, L0), (l1, L1) = hog.cascade_levels(U)[:2]
    assert np.array_equal(L0, U.astype(np.float64))
    xs = (12 * np.arange(l1.w) + 1) / 10.0
    assert np.all(np.abs(L1 - (2 * xs + 20)[None, :]) <= 0.5 + 2.0 / 512 + 1e-12)


def test_cascade_first_step_equals_rounded_direct():
    """One 5/6 step from the frame is the direct level 1 (R2, resampled from
    the frame with the fixed-point inverse scale) rounded to grey levels,
    wherever the two tap tables agree: an independent route to the same
    numbers."""
    from paper_2006_00816_amd import synth
    U = synth.ClipGenerator(3, 240, 320, face_h=100.0).frame()
    casc = hog.cascade_levels(U)
    lv1 = hog.pyramid(240, 320)[1]
    dy = hog.axis_taps(lv1.h, 240, lv1)
    dx = hog.axis_taps(lv1.w, 320, lv1)
    cy = hog.cascade_taps(lv1.h, 240)
    cx = hog.cascade_taps(lv1.w, 320)
    assert all(np.array_equal(a, b) for a, b in zip(dy, cy)) and all(np.array_equal(a, b) for a, b in zip(dx, cx))
    assert np.array_equal(casc[1][1], hog.round_grey(hog.resample(U, lv1)))


def test_cascade_candidates_boxes_use_nominal_scale():
    """Windows of a cascade level map back to the frame with the level's
    nominal scale u (5/6)^k, as in the direct pyramid: the same box for
    the same anchor."""
    from paper_2006_00816_amd import synth
    U = synth.ClipGenerator(4, 240, 320, face_h=100.0).frame()
    W, b = synth.filters([101], bias=0.5)
    c = hog.candidates(U, W, b, cascade=True)
    assert len(c) > 0
    for lv in hog.pyramid_cascade(240, 320):
        sel = c[c["k"] == lv.k]
        x0, y0, x1, y1 = hog.window_box(lv, sel["r"], sel["c"])
        assert np.array_equal(sel["x0"], x0) and np.array_equal(sel["y1"], y1)
