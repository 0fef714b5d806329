"""Gradients through the C ABI against the float64 oracle: window scores,
the hinge loss and its score gradient, the filter gradient (also against
float64 central finite differences, h = 1e-6), top-k windows, and the
pixel gradient of summed top-10 scores (against the oracle's analytic
gradient everywhere and its finite differences at 64 pixels)."""
import numpy as np
import pytest
import torch

from oracle import hog as oracle
from paper_2006_00816_amd import synth
from test_gpu_parity import H, cu  # noqa: F401

pytestmark = pytest.mark.gpu

LV80 = oracle.Level(0, 1, 1, 80, 80)


@pytest.fixture(scope="module")
def crops():
    c, y = synth.config3(seed=3, n_pos=16, n_neg=16)
    F = np.stack([oracle.level_features(x, LV80) for x in c])
    return c, y, F


def test_window_scores_match_oracle(H, crops):
    c, y, F = crops
    W, b = synth.filters([7])
    win = H.windows_tensor(torch.arange(len(c), dtype=torch.int32), 0, 0, 0, 0)
    s = H.window_scores(cu(c), cu(W), cu(b), win).cpu().numpy()
    want = b[0] + np.tensordot(F, W[0].astype(np.float64), axes=3)
    assert np.allclose(s, want, rtol=1e-5, atol=2e-5), float(np.abs(s - want).max())


def test_filter_gradient_matches_oracle_and_finite_differences(H, crops):
    c, y, F = crops
    W, b = synth.filters([7])
    Wt, bt = cu(W), cu(b)
    win = H.windows_tensor(torch.arange(len(c), dtype=torch.int32), 0, 0, 0, 0)
    s = H.window_scores(cu(c), Wt, bt, win)
    loss, dscore, dW = H.hinge_loss(s, cu(y), Wt, 1e-4)
    dW, db, _ = H.filter_backward(cu(c), Wt, win, dscore, dW=dW)
    S64 = b[0] + np.tensordot(F, W[0].astype(np.float64), axes=3)
    assert abs(float(loss.item()) - oracle.hinge_loss(S64, y, W, 1e-4)) <= 1e-5
    ds64 = oracle.hinge_dscore(S64, y)
    assert np.allclose(dscore.cpu().numpy(), ds64, rtol=1e-6, atol=1e-9)
    gW, gb = oracle.filter_grad(F, ds64)
    gW = gW + 2e-4 * W[0].astype(np.float64)
    assert np.allclose(dW.cpu().numpy()[0], gW, rtol=1e-5, atol=2e-6), float(np.abs(dW.cpu().numpy()[0] - gW).max())
    assert abs(float(db.cpu().numpy()[0]) - gb) <= 1e-6

    # float64 central finite differences of the oracle loss, h = 1e-6, on
    # 200 random filter entries and the bias
    def L(Wv, bv):
        return oracle.hinge_loss(bv + np.tensordot(F, Wv, axes=3), y, Wv, 1e-4)

    W64 = W[0].astype(np.float64)
    b0 = float(b[0])          # float64: a float32 bias would quantise the step
    rng = np.random.default_rng(0)
    idx = [tuple(rng.integers(0, n) for n in W64.shape) for _ in range(200)]
    for ix in idx:
        Wp, Wm = W64.copy(), W64.copy()
        Wp[ix] += 1e-6
        Wm[ix] -= 1e-6
        fd = (L(Wp, b0) - L(Wm, b0)) / 2e-6
        assert abs(float(dW.cpu().numpy()[0][ix]) - fd) <= 1e-5 * abs(fd) + 2e-6, (ix, fd)
    fdb = (L(W64, b0 + 1e-6) - L(W64, b0 - 1e-6)) / 2e-6
    assert abs(float(db.cpu().numpy()[0]) - fdb) <= 1e-6


def test_autograd_function(H, crops):
    c, y, F = crops
    W, b = synth.filters([8])
    Wt = cu(W).requires_grad_(True)
    bt = cu(b).requires_grad_(True)
    win = H.windows_tensor(torch.arange(len(c), dtype=torch.int32), 0, 0, 0, 0)
    s = H.HogScore.apply(Wt, bt, cu(c), win)
    wts = torch.linspace(-1, 1, len(c), device="cuda")
    (s * wts).sum().backward()
    want = np.tensordot(wts.cpu().numpy().astype(np.float64), F, axes=(0, 0))
    assert np.allclose(Wt.grad.cpu().numpy()[0], want, rtol=1e-5, atol=2e-6)
    assert abs(float(bt.grad.cpu().numpy()[0]) - float(wts.sum())) <= 1e-5


def _small_frames():
    out = []
    for seed, (h, w), u in ((61, (104, 120), 1), (62, (60, 68), 2), (63, (150, 170), 1)):
        rng = np.random.default_rng(seed)
        U = synth.background(rng, h, w)
        synth.paint_face(U, h / 2, w / 2, 0.6 * min(h, w), 200.0)
        out.append((np.clip(np.rint(U), 0, 255).astype(np.uint8), u))
    return out


@pytest.mark.parametrize("case", range(3))
def test_topk_windows_match_oracle(H, case):
    frame, u = _small_frames()[case]
    W, b = synth.filters([201, 202, 203])
    win, sc = H.topk_windows(cu(frame[None]), cu(W), cu(b), 10, u)
    ow = oracle.top_windows(frame, W, b, 12, u)
    got = [tuple(x) for x in win.cpu().numpy()[0][:, 1:].tolist()]
    want = [(int(r["f"]), int(r["k"]), int(r["r"]), int(r["c"])) for r in ow[:10]]
    # ranks may differ only where oracle scores of neighbouring ranks are
    # closer than 1e-4 (including the boundary between ranks 10 and 11)
    s = ow["score"]
    near = [i for i in range(11) if abs(s[i] - s[i + 1]) < 1e-4]
    amb = set(near) | set(i + 1 for i in near)
    for i in range(10):
        if got[i] != want[i]:
            assert i in amb, (i, got, want)
    assert np.allclose(sc.cpu().numpy()[0], ow["score"][:10], rtol=1e-5, atol=2e-5)


@pytest.mark.parametrize("case", range(3))
def test_pixel_gradient_matches_oracle(H, case):
    frame, u = _small_frames()[case]
    W, b = synth.filters([201, 202])
    win, sc = H.topk_windows(cu(frame[None]), cu(W), cu(b), 10, u)
    recs = win.cpu().numpy()[0]
    ow = np.zeros(10, oracle.CAND_DTYPE)
    ow["f"], ow["k"], ow["r"], ow["c"] = recs[:, 1], recs[:, 2], recs[:, 3], recs[:, 4]
    dpix = H.pixel_gradient(cu(frame[None]), cu(W), win.reshape(-1, 5).contiguous(),
                            torch.ones(10, device="cuda"), u)[0].cpu().numpy().astype(np.float64)
    want, _ = oracle.topk_pixel_grad(frame, W, b, 10, u, windows=ow)
    scale = np.abs(want).max()
    assert scale > 0
    err = np.abs(dpix - want)
    assert np.all(err <= 1e-4 * np.abs(want) + 1e-5 * scale), (float(err.max()), scale)


def test_pixel_gradient_matches_finite_differences(H):
    """64 pixels where the bins, clip states and the top-10 set are the same
    at U - h, U and U + h (U as float64, h = 1e-6)."""
    rng = np.random.default_rng(71)
    frame, u = _small_frames()[0]
    W, b = synth.filters([201, 202])
    win, _ = H.topk_windows(cu(frame[None]), cu(W), cu(b), 10, u)
    recs = win.cpu().numpy()[0]
    ow = np.zeros(10, oracle.CAND_DTYPE)
    ow["f"], ow["k"], ow["r"], ow["c"] = recs[:, 1], recs[:, 2], recs[:, 3], recs[:, 4]
    dpix = H.pixel_gradient(cu(frame[None]), cu(W), win.reshape(-1, 5).contiguous(),
                            torch.ones(10, device="cuda"), u)[0].cpu().numpy().astype(np.float64)
    U = frame.astype(np.float64)
    from test_oracle_grad import _same_state, _state
    s0 = _state(U, W, b, ow, u)
    cand = np.argwhere(np.abs(dpix) > 1e-3)
    pick = cand[rng.choice(len(cand), min(len(cand), 200), replace=False)]
    checked = 0
    for y, x in pick:
        Up, Um = U.copy(), U.copy()
        Up[y, x] += 1e-6
        Um[y, x] -= 1e-6
        if not (_same_state(_state(Up, W, b, ow, u), s0) and _same_state(_state(Um, W, b, ow, u), s0)):
            continue
        fd = (oracle.topk_objective(Up, W, b, ow, u) - oracle.topk_objective(Um, W, b, ow, u)) / 2e-6
        assert abs(dpix[y, x] - fd) <= 2e-4 * abs(fd) + 1e-5, (y, x, dpix[y, x], fd)
        checked += 1
        if checked == 64:
            break
    assert checked == 64


def test_config4_frame_topk_and_pixel_gradient(H):
    """One 1920x1080 frame of the large-batch workload on the pyramid from
    2x (19 levels, 32-bit NMS records): top-10 windows and the pixel
    gradient of their summed scores against the oracle at every pixel."""
    wl = synth.config4(seed=4, n=1)
    frame, W, b, u = wl.frames[0], wl.W, wl.b, 2
    print("config-4 frame 1920x1080 u=2", flush=True)
    win, sc = H.topk_windows(cu(frame[None]), cu(W), cu(b), 10, u)
    ow = oracle.top_windows(frame, W, b, 12, u)
    got = [tuple(x) for x in win.cpu().numpy()[0][:, 1:].tolist()]
    want = [(int(r["f"]), int(r["k"]), int(r["r"]), int(r["c"])) for r in ow[:10]]
    s = ow["score"]
    near = [i for i in range(11) if abs(s[i] - s[i + 1]) < 1e-4]
    amb = set(near) | set(i + 1 for i in near)
    for i in range(10):
        if got[i] != want[i]:
            assert i in amb, (i, got, want)
    assert np.allclose(sc.cpu().numpy()[0], s[:10], rtol=1e-5, atol=2e-5)
    recs = win.cpu().numpy()[0]
    w10 = np.zeros(10, oracle.CAND_DTYPE)
    w10["f"], w10["k"], w10["r"], w10["c"] = recs[:, 1], recs[:, 2], recs[:, 3], recs[:, 4]
    dpix = H.pixel_gradient(cu(frame[None]), cu(W), win.reshape(-1, 5).contiguous(),
                            torch.ones(10, device="cuda"), u)[0].cpu().numpy().astype(np.float64)
    g, _ = oracle.topk_pixel_grad(frame, W, b, 10, u, windows=w10)
    scale = np.abs(g).max()
    assert scale > 0
    err = np.abs(dpix - g)
    assert np.all(err <= 1e-4 * np.abs(g) + 1e-5 * scale), (float(err.max()), scale)


def test_hinge_kernel_hand_case(H):
    """The hand case of the oracle pins on the GPU: loss 0.240031, score
    gradient (0, -0.2, 0.2, 0, 0) with zero at the kink, dW = 2e-4 W."""
    S = cu(np.array([2.0, 0.5, -0.3, -2.0, 1.0], np.float32))
    y = cu(np.array([1.0, 1.0, -1.0, -1.0, 1.0], np.float32))
    W = cu(np.full((1, 10, 10, 31), 0.01, np.float32))
    loss, dscore, dW = H.hinge_loss(S, y, W, 1e-4)
    assert abs(float(loss.item()) - 0.240031) <= 1e-6
    assert np.array_equal(dscore.cpu().numpy(), np.array([0.0, -0.2, 0.2, 0.0, 0.0], np.float32))
    assert np.allclose(dW.cpu().numpy(), 2e-6, rtol=1e-6, atol=0)


def test_topk_includes_sub_threshold_windows(H):
    """Constant 80x96 frame: every window of filter f scores b_f (3 window
    anchors per filter).  With b = (0.3, -0.5, 0.2, -0.1) the top 10 are
    filter 0's three windows, filter 2's, filter 3's (below the threshold)
    and the first of filter 1's."""
    fr = cu(np.full((1, 80, 96), 140, np.uint8))
    W, _ = synth.filters([11, 12, 13, 14])
    b = np.array([0.3, -0.5, 0.2, -0.1], np.float32)
    win, sc = H.topk_windows(fr, cu(W), cu(b), 10)
    got = [tuple(x) for x in win.cpu().numpy()[0].tolist()]
    want = [(0, f, 0, 0, c) for f in (0, 2, 3) for c in range(3)] + [(0, 1, 0, 0, 0)]
    assert got == want
    assert np.array_equal(sc.cpu().numpy()[0], np.repeat(b[[0, 2, 3, 1]], [3, 3, 3, 1]))
    ow = oracle.top_windows(np.full((80, 96), 140, np.uint8), W, b, 10)
    assert [(0, int(r["f"]), int(r["k"]), int(r["r"]), int(r["c"])) for r in ow] == want


def test_out_of_range_windows_are_skipped(H):
    """Windows outside the batch are refused by the binding, and through the
    raw C ABI the kernels skip them without reading: their scores are NaN,
    the other scores are unchanged, and dfilters[0] turns NaN."""
    import ctypes
    frames, u = _small_frames()[0]
    W, b = synth.filters([201, 202])
    Wt, bt = cu(W), cu(b)
    fr = cu(frames[None])
    lv = oracle.pyramid(*frames.shape, u)
    good = [[0, 0, 0, 0, 0], [0, 1, len(lv) - 1, lv[-1].rows - 1, lv[-1].cols - 1]]
    bad = [[1, 0, 0, 0, 0], [0, 2, 0, 0, 0], [0, 0, len(lv), 0, 0], [0, 0, 0, lv[0].rows, 0],
           [0, 0, 0, 0, -1], [-5, 0, 0, 0, 0]]
    win = torch.tensor(good + bad, dtype=torch.int32, device="cuda")
    with pytest.raises(H.HogError):
        H.window_scores(fr, Wt, bt, win)
    s = H.window_scores(fr, Wt, bt, win, check=False).cpu().numpy()
    ref = H.window_scores(fr, Wt, bt, win[:2].contiguous()).cpu().numpy()
    assert np.array_equal(s[:2], ref) and np.all(np.isnan(s[2:]))
    ds = torch.ones(len(good) + len(bad), device="cuda")
    with pytest.raises(H.HogError):
        H.filter_backward(fr, Wt, win, ds)
    dW, db, dpix = H.filter_backward(fr, Wt, win, ds, pixels=True, check=False)
    dW_ok, db_ok, dpix_ok = H.filter_backward(fr, Wt, win[:2].contiguous(), ds[:2].contiguous(), pixels=True)
    torch.cuda.synchronize()
    assert np.isnan(dW.view(-1)[0].item())
    assert torch.equal(db, db_ok)
    assert torch.allclose(dpix, dpix_ok, rtol=1e-5, atol=1e-7)


def test_pixel_autograd_function(H):
    """HogPixelScore: autograd reaches the pixels, the filters and the bias;
    the pixel gradient of the summed top-10 scores equals the oracle's."""
    frame, u = _small_frames()[0]
    W, b = synth.filters([201, 202])
    win, _ = H.topk_windows(cu(frame[None]), cu(W), cu(b), 10, u)
    win = win.reshape(-1, 5).contiguous()
    px = cu(frame[None].astype(np.float32)).requires_grad_(True)
    Wt = cu(W).requires_grad_(True)
    bt = cu(b).requires_grad_(True)
    s = H.HogPixelScore.apply(px, Wt, bt, win, u)
    s.sum().backward()
    recs = win.cpu().numpy()
    ow = np.zeros(10, oracle.CAND_DTYPE)
    ow["f"], ow["k"], ow["r"], ow["c"] = recs[:, 1], recs[:, 2], recs[:, 3], recs[:, 4]
    want, _ = oracle.topk_pixel_grad(frame, W, b, 10, u, windows=ow)
    g = px.grad.cpu().numpy()[0].astype(np.float64)
    scale = np.abs(want).max()
    assert np.all(np.abs(g - want) <= 1e-4 * np.abs(want) + 1e-5 * scale), float(np.abs(g - want).max())
    dW, db, _ = H.filter_backward(cu(frame[None]), cu(W), win, torch.ones(10, device="cuda"), u)
    assert torch.equal(Wt.grad, dW) and torch.equal(bt.grad, db)
    with pytest.raises(H.HogError):
        H.HogPixelScore.apply(px.detach() + 0.5, Wt, bt, win, u)
