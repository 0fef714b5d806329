"""Pure-Python loop statement of the HOG detector, for tiny inputs.

TEST INFRASTRUCTURE ONLY.  It pins the vectorised float64 oracle in
``oracle/hog.py`` by computing the same quantities a second way, written
from the paper's description rather than from that module:

* pyramid taps with exact rational arithmetic (``fractions.Fraction``)
  on the fixed-point inverse scale;
* orientation from the gradient angle (``math.atan2``) as the nearest of
  the 18 directions 0, 20, ..., 340 degrees, instead of projections;
* cell votes from the tent weight max(0, 1 - |distance to cell centre|)
  evaluated for every cell, instead of floor/fraction splitting;
* normalisation, features, scores and NMS as explicit loops, IoU as an
  exact fraction.

It is far too slow for anything but frames of about 100x100 pixels.
"""
from __future__ import annotations

import math
from fractions import Fraction


def pyramid_sizes(h, w, upsample=1):
    out = []
    k = 0
    while True:
        s = Fraction(upsample * 5 ** k, 6 ** k)
        hk, wk = math.floor(h * s), math.floor(w * s)
        if hk < 80 or wk < 80:
            return out
        out.append((k, s, hk, wk))
        k += 1


def inverse_scale(s):
    """1/s rounded half-up to a multiple of 2^-40."""
    return Fraction(math.floor(Fraction(1, 1) / s * 2 ** 40 + Fraction(1, 2)), 2 ** 40)


def taps(i, n_in, s):
    """Source taps of output sample i at scale s (pixel centres aligned,
    inverse scale in 2^-40 fixed point, weight of the second tap rounded
    half-up to 1/256)."""
    xs = Fraction(2 * i + 1, 2) * inverse_scale(s) - Fraction(1, 2)
    i0 = math.floor(xs)
    a = math.floor(256 * (xs - i0) + Fraction(1, 2))
    if a == 256:
        i0, a = i0 + 1, 0
    cl = lambda v: min(max(v, 0), n_in - 1)
    return [(cl(i0), Fraction(256 - a, 256)), (cl(i0 + 1), Fraction(a, 256))]


def level_image(U, s, hk, wk):
    H, W = len(U), len(U[0])
    out = [[0.0] * wk for _ in range(hk)]
    for y in range(hk):
        ty = taps(y, H, s)
        for x in range(wk):
            tx = taps(x, W, s)
            v = Fraction(0)
            for yy, wy in ty:
                for xx, wx in tx:
                    v += wy * wx * Fraction(U[yy][xx])
            out[y][x] = float(v)
    return out


def angle_bin(gx, gy):
    if gx == 0 and gy == 0:
        return 0
    if gx == 0:
        return 4 if gy > 0 else 13
    deg = math.degrees(math.atan2(gy, gx)) % 360.0
    return int(math.floor((deg + 10.0) / 20.0)) % 18


def level_hist(L):
    hk, wk = len(L), len(L[0])
    cy, cx = hk // 8, wk // 8
    hist = [[[0.0] * 18 for _ in range(cx)] for _ in range(cy)]
    for y in range(8 * cy):
        for x in range(8 * cx):
            if not (1 <= x <= wk - 2 and 1 <= y <= hk - 2):
                continue
            gx = L[y][x + 1] - L[y][x - 1]
            gy = L[y + 1][x] - L[y - 1][x]
            mag = math.sqrt(gx * gx + gy * gy)
            b = angle_bin(gx, gy)
            yc = (y + 0.5) / 8 - 0.5
            xc = (x + 0.5) / 8 - 0.5
            for i in range(cy):
                wy = max(0.0, 1.0 - abs(yc - i))
                if wy == 0.0:
                    continue
                for j in range(cx):
                    wx = max(0.0, 1.0 - abs(xc - j))
                    if wx > 0.0:
                        hist[i][j][b] += mag * wy * wx
    return hist


def features(hist, clip=0.2, eps=1e-4):
    cy, cx = len(hist), len(hist[0])

    def energy(i, j):
        if 0 <= i < cy and 0 <= j < cx:
            h = hist[i][j]
            return sum((h[o] + h[o + 9]) ** 2 for o in range(9))
        return 0.0

    F = [[None] * cx for _ in range(cy)]
    for i in range(cy):
        for j in range(cx):
            h = hist[i][j]
            norms = []
            for dy, dx in ((-1, -1), (-1, 1), (1, -1), (1, 1)):
                blk = energy(i, j) + energy(i + dy, j) + energy(i, j + dx) + energy(i + dy, j + dx)
                norms.append(1.0 / math.sqrt(blk + eps))
            f = [0.0] * 31
            for n_k in norms:
                for b in range(18):
                    f[b] += 0.5 * min(h[b] * n_k, clip)
                for o in range(9):
                    f[18 + o] += 0.5 * min((h[o] + h[o + 9]) * n_k, clip)
            for k, n_k in enumerate(norms):
                f[27 + k] = sum(min(h[b] * n_k, clip) for b in range(18)) / math.sqrt(18.0)
            F[i][j] = f
    return F


def scores(F, W, b):
    cy, cx = len(F), len(F[0])
    out = []
    for f in range(len(W)):
        rows = []
        for r in range(cy - 9):
            row = []
            for c in range(cx - 9):
                acc = float(b[f])
                for dr in range(10):
                    for dc in range(10):
                        fv = F[r + dr][c + dc]
                        wv = W[f][dr][dc]
                        for ch in range(31):
                            acc += float(wv[ch]) * fv[ch]
                row.append(acc)
            rows.append(row)
        out.append(rows)
    return out


def box(s, r, c):
    def rnd(v):
        return math.floor(v + Fraction(1, 2))
    inv = inverse_scale(s)
    return (rnd(8 * c * inv), rnd(8 * r * inv), rnd((8 * c + 80) * inv), rnd((8 * r + 80) * inv))


def detect(U, W, b, thresh=0.0, iou=0.5, upsample=1):
    H, Wd = len(U), len(U[0])
    cands = []
    for k, s, hk, wk in pyramid_sizes(H, Wd, upsample):
        S = scores(features(level_hist(level_image(U, s, hk, wk))), W, b)
        for f in range(len(S)):
            for r in range(len(S[f])):
                for c in range(len(S[f][r])):
                    if S[f][r][c] > thresh:
                        cands.append((S[f][r][c], f, k, r, c, box(s, r, c)))
    cands.sort(key=lambda t: (-t[0], t[1], t[2], t[3], t[4]))
    kept = []
    lim = Fraction(iou)
    for cand in cands:
        x0, y0, x1, y1 = cand[5]
        ok = True
        for kc in kept:
            a0, b0, a1, b1 = kc[5]
            inter = max(0, min(x1, a1) - max(x0, a0)) * max(0, min(y1, b1) - max(y0, b0))
            union = (x1 - x0) * (y1 - y0) + (a1 - a0) * (b1 - b0) - inter
            if Fraction(inter, union) > lim:
                ok = False
                break
        if ok:
            kept.append(cand)
    return kept
