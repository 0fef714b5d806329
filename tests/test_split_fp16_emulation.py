"""The split-fp16 scoring arithmetic (HOG_ARITH_F16X3), emulated on the CPU
with numpy float16 from the oracle's float64 features and weights: each
operand v becomes hi = fp16(v) and lo = fp16((v - hi) 2^11), both rounded
to nearest, and a product x w becomes
x_hi w_hi + 2^-11 (x_hi w_lo + x_lo w_hi).  The scores must stay within the
tolerance the GPU parity tests use (1e-5 relative + 2e-5 absolute), and the
plain fp16 product (x_hi w_hi alone) must not, so that the test can tell
the two apart."""
import numpy as np
import pytest

from oracle import hog as oracle
from paper_2006_00816_amd import synth

RTOL, ATOL = 1e-5, 2e-5


def _split(v):
    v32 = np.asarray(v, np.float32)
    hi = v32.astype(np.float16)
    lo = ((v32 - hi.astype(np.float32)) * np.float32(2048.0)).astype(np.float16)
    return hi.astype(np.float64), lo.astype(np.float64)


def _case(name):
    if name == "c0":
        return synth.config0(0).frames[0]
    rng = np.random.default_rng(5)
    img = synth.background(rng, 200, 240)
    synth.paint_face(img, 100, 120, 120, 205.0)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("name,nf,scale", [("c0", 5, 1.0), ("face", 5, 1.0), ("face", 3, 2.0 ** 10),
                                           ("c0", 2, 2.0 ** -12)])
def test_split_products_within_tolerance(name, nf, scale):
    frame = _case(name)
    W, b = synth.filters(range(700, 700 + nf))
    W = (W.astype(np.float64) * scale).astype(np.float32)
    b = (b.astype(np.float64) * scale).astype(np.float32)
    lv = oracle.pyramid(*frame.shape, 1)[0]
    F = oracle.level_features(frame, lv)
    S = oracle.window_scores(F, W.astype(np.float64), b.astype(np.float64))
    xh, xl = _split(F)
    wh, wl = _split(W)
    zero = np.zeros(nf)
    split = (oracle.window_scores(xh, wh, zero)
             + 2.0 ** -11 * (oracle.window_scores(xh, wl, zero) + oracle.window_scores(xl, wh, zero))
             + b.astype(np.float64)[:, None, None])
    err = np.abs(split - S) / scale
    assert (err <= ATOL + RTOL * np.abs(S) / scale).all(), float(err.max())
    plain = oracle.window_scores(xh, wh, zero) + b.astype(np.float64)[:, None, None]
    perr = np.abs(plain - S) / scale
    assert (perr > ATOL + RTOL * np.abs(S) / scale).any(), float(perr.max())


def test_split_reconstructs_operands():
    """hi + 2^-11 lo recovers a float32 operand to within 2^-23 |v| + 2^-36 (one FP32 ulp):
    relative for normal fp16 high parts, absolute near zero (where the low
    part is an fp16 subnormal)."""
    rng = np.random.default_rng(9)
    v = np.concatenate([rng.uniform(0, 1, 10000), rng.uniform(0, 1e-6, 1000), rng.uniform(0, 1e-9, 1000),
                        rng.normal(0, 0.1, 10000), rng.normal(0, 1000.0, 1000)]).astype(np.float32)
    hi, lo = _split(v)
    err = np.abs(hi + 2.0 ** -11 * lo - v.astype(np.float64))
    bound = 2.0 ** -23 * np.abs(v.astype(np.float64)) + 2.0 ** -36
    assert (err <= bound).all(), float((err / bound).max())
