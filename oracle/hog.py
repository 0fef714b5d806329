"""FP64 CPU oracle of the HOG sliding-window face detector.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
calls this module; it exists so that tests, the smoke check and the CPU
baseline leg of the benchmark can check the HIP path against a plain,
slow, obviously correct statement of what the detector computes.

Every function follows the paper's algorithm breakdown of the face
detector (Sec. IV-A, "Algorithm breakdown") in order: image pyramid,
gradient computation, histogramisation, normalisation, feature
computation, linear classification and non-maximum suppression.  Where the
paper is silent or ambiguous, the reading taken is named (R1..R16) and the
same numbering is used in the design notes.

Arithmetic is numpy float64 unless a step is integer by definition.  The
code is vectorised over pixels and cells only; there is no tiling,
fusion or reordering of the steps.
"""
from __future__ import annotations

import dataclasses
import math
from functools import lru_cache

import mpmath
import numpy as np

CELL = 8            # 8x8-pixel cells (Sec. IV-A, histogramisation)
NBINS = 18          # eighteen signed orientations (Sec. IV-A, gradient computation)
NORIENT = 9         # unsigned orientations: bins o and o+9 are opposite directions
WIN = 10            # 80x80 px = 10x10-cell detection window (Sec. IV-A, classification)
NFEAT = 31          # 18 signed + 9 unsigned + 4 energy features (Sec. IV-A, features)
MIN_SIDE = 80       # pyramid stops below the 80 px window (Sec. IV-A)
SCALE_NUM, SCALE_DEN = 5, 6   # 5/6 downscale step (Sec. IV-A)
CLIP = 0.2          # truncation of normalised values (R8)
EPS = 1e-4          # added to block energies before the square root (R7)
TEXTURE = 1.0 / math.sqrt(18.0)   # weight of the 4 energy features (R8)


# ---------------------------------------------------------------- pyramid
@dataclasses.dataclass(frozen=True)
class Level:
    """One pyramid level: scale s = p/q relative to the frame."""
    k: int
    p: int
    q: int
    h: int
    w: int

    @property
    def cy(self) -> int:
        return self.h // CELL

    @property
    def cx(self) -> int:
        return self.w // CELL

    @property
    def rows(self) -> int:          # window rows r = 0 .. cy-10
        return self.cy - WIN + 1

    @property
    def cols(self) -> int:
        return self.cx - WIN + 1


def pyramid(h: int, w: int, upsample: int = 1) -> list[Level]:
    """Pyramid levels k = 0, 1, ... with s_k = upsample * (5/6)^k, sizes
    floor(h*s_k) x floor(w*s_k), kept while both sides are >= 80 px.

    Sec. IV-A: the image is scaled down in 5/6 steps until a side is
    smaller than the 80x80 window.  R1: every level is sized directly from
    the frame with exact integer arithmetic.  R3: ``upsample`` = 2 applies
    the 2x enlargement (Sec. III-B upscales test images 2x) in the same
    composite scale."""
    out = []
    k = 0
    while True:
        p, q = upsample * SCALE_NUM ** k, SCALE_DEN ** k
        hk, wk = (h * p) // q, (w * p) // q
        if min(hk, wk) < MIN_SIDE:
            return out
        out.append(Level(k, p, q, hk, wk))
        k += 1


def pyramid_cascade(h: int, w: int, upsample: int = 1) -> list[Level]:
    """Levels of the recursive pyramid (R20): level k is scaled down from
    level k-1 by 5/6, so its size is floor(5 h_{k-1} / 6) x
    floor(5 w_{k-1} / 6) (Sec. V-A, image-scaling kernel: each scaled
    image is based on the image one scale higher; Sec. IV-A: down to the
    80x80 window).  Level 0 is the frame, or the 2x enlargement for
    upsample = 2.  The nominal scale of level k stays u (5/6)^k, which maps
    its pixel edges back to the frame as for the direct pyramid."""
    out = []
    hk, wk = h * upsample, w * upsample
    k = 0
    while min(hk, wk) >= MIN_SIDE:
        out.append(Level(k, upsample * SCALE_NUM ** k, SCALE_DEN ** k, hk, wk))
        hk, wk = (hk * SCALE_NUM) // SCALE_DEN, (wk * SCALE_NUM) // SCALE_DEN
        k += 1
    return out


def cascade_taps(n_out: int, n_in: int):
    """Bilinear taps of one 5/6 step along an axis (R20): output sample i
    of the smaller image sits at (i + 1/2) 6/5 - 1/2 = (12 i + 1) / 10 of
    the larger one (pixel centres aligned); its integer part i0 and its
    fractional part, rounded half-up to a multiple of 1/256, give taps i0,
    i0 + 1 (clamped) with weights (256 - a)/256 and a/256."""
    i = np.arange(n_out, dtype=np.int64)
    num = 12 * i + 1
    i0 = num // 10
    a = (256 * (num % 10) + 5) // 10
    return np.minimum(i0, n_in - 1), np.minimum(i0 + 1, n_in - 1), a


def round_grey(v):
    """Round half up to integer grey levels, as images of 8-bit pixels."""
    return np.floor(np.asarray(v, np.float64) + 0.5)


def cascade_levels(frame: np.ndarray, upsample: int = 1):
    """Level images of the recursive pyramid (R20), as float64 arrays of
    integer grey levels: level 0 is the frame (upsample 1) or its 2x
    bilinear enlargement (R3) rounded to grey levels; level k is the
    bilinear 5/6 reduction of level k-1 (cascade_taps) rounded to grey
    levels, as an image of 8-bit pixels is (Sec. V-A: the scaling kernel
    writes each scaled image, which the next step reads)."""
    U = np.asarray(frame, np.float64)
    H, W = U.shape
    levels = pyramid_cascade(H, W, upsample)
    out = []
    prev = None
    for lv in levels:
        if lv.k == 0:
            img = U.copy() if upsample == 1 else round_grey(resample(U, pyramid(H, W, upsample)[0]))
        else:
            y0, y1, ay = cascade_taps(lv.h, prev.shape[0])
            x0, x1, ax = cascade_taps(lv.w, prev.shape[1])
            wy0, wy1 = (256 - ay) / 256.0, ay / 256.0
            wx0, wx1 = (256 - ax) / 256.0, ax / 256.0
            img = round_grey((wy0[:, None] * wx0[None, :]) * prev[np.ix_(y0, x0)]
                             + (wy0[:, None] * wx1[None, :]) * prev[np.ix_(y0, x1)]
                             + (wy1[:, None] * wx0[None, :]) * prev[np.ix_(y1, x0)]
                             + (wy1[:, None] * wx1[None, :]) * prev[np.ix_(y1, x1)])
        out.append((lv, img))
        prev = img
    return out


SIG_BITS = 40


def inverse_scale_fixed(lv: Level) -> int:
    """The inverse scale q/p of a level as a fixed-point integer with 40
    fractional bits, rounded half-up (R2)."""
    return (lv.q * (1 << (SIG_BITS + 1)) + lv.p) // (2 * lv.p)


def axis_taps(n_out: int, n_in: int, lv: Level):
    """Bilinear taps along one axis of level lv (R2).

    Output sample i sits at source coordinate (i + 1/2) * q/p - 1/2
    (pixel centres aligned), with q/p taken as the fixed-point value SIG
    of :func:`inverse_scale_fixed`: xs = ((2i + 1) * SIG - 2^40) / 2^41.
    Its integer part i0 and the fractional part, rounded half-up to a
    multiple of 1/256, give the taps i0 and i0 + 1 (clamped to the
    source) with weights (256 - a)/256 and a/256.  All of it is exact
    integer arithmetic."""
    sig = inverse_scale_fixed(lv)
    one = 1 << (SIG_BITS + 1)
    i0 = np.empty(n_out, np.int64)
    i1 = np.empty(n_out, np.int64)
    a8 = np.empty(n_out, np.int64)
    for i in range(n_out):
        t = (2 * i + 1) * sig - (1 << SIG_BITS)
        base = t // one                  # floor, also for negative t
        frac = t - base * one            # in [0, 2^41)
        a = (256 * frac + one // 2) // one
        if a == 256:
            base, a = base + 1, 0
        i0[i] = min(max(base, 0), n_in - 1)
        i1[i] = min(max(base + 1, 0), n_in - 1)
        a8[i] = a
    return i0, i1, a8


def resample(frame: np.ndarray, lv: Level) -> np.ndarray:
    """Level image L_k = bilinear resample of the frame itself at scale
    s_k (R2).  With integer frames every value is a multiple of 2^-16
    below 256, so the float64 result is exact."""
    U = np.asarray(frame, np.float64)
    H, W = U.shape
    y0, y1, ay = axis_taps(lv.h, H, lv)
    x0, x1, ax = axis_taps(lv.w, W, lv)
    wy0, wy1 = (256 - ay) / 256.0, ay / 256.0
    wx0, wx1 = (256 - ax) / 256.0, ax / 256.0
    L = ((wy0[:, None] * wx0[None, :]) * U[np.ix_(y0, x0)]
         + (wy0[:, None] * wx1[None, :]) * U[np.ix_(y0, x1)]
         + (wy1[:, None] * wx0[None, :]) * U[np.ix_(y1, x0)]
         + (wy1[:, None] * wx1[None, :]) * U[np.ix_(y1, x1)])
    return L


def resample_transpose(dL: np.ndarray, lv: Level, H: int, W: int) -> np.ndarray:
    """Adjoint of :func:`resample`: scatters level values back onto the
    frame with the same tap weights."""
    y0, y1, ay = axis_taps(lv.h, H, lv)
    x0, x1, ax = axis_taps(lv.w, W, lv)
    wy = ((256 - ay) / 256.0, ay / 256.0)
    wx = ((256 - ax) / 256.0, ax / 256.0)
    dU = np.zeros((H, W))
    for ys, wyv in zip((y0, y1), wy):
        for xs, wxv in zip((x0, x1), wx):
            np.add.at(dU, (ys[:, None], xs[None, :]),
                      (wyv[:, None] * wxv[None, :]) * dL)
    return dU


# -------------------------------------------------------------- gradients
def gradients(L: np.ndarray):
    """Central differences [-1, 0, 1] along x and y (y pointing down).
    The one-pixel border of the level has zero gradient (R4)."""
    gx = np.zeros_like(L)
    gy = np.zeros_like(L)
    gx[1:-1, 1:-1] = L[1:-1, 2:] - L[1:-1, :-2]
    gy[1:-1, 1:-1] = L[2:, 1:-1] - L[:-2, 1:-1]
    return gx, gy


def _nearest_double(x) -> float:
    return float(mpmath.nstr(x, 40, strip_zeros=False))


@lru_cache(maxsize=1)
def orientation_table():
    """c_o = cos(o*pi/9), s_o = sin(o*pi/9), o = 0..8, each the float64
    nearest to the exact value.  Correct rounding makes the table mirror
    exactly: c_{9-o} = -c_o and s_{9-o} = s_o (R5)."""
    mpmath.mp.dps = 60
    c = np.array([_nearest_double(mpmath.cos(o * mpmath.pi / 9)) for o in range(NORIENT)])
    s = np.array([_nearest_double(mpmath.sin(o * mpmath.pi / 9)) for o in range(NORIENT)])
    for o in range(1, 5):
        assert c[9 - o] == -c[o] and s[9 - o] == s[o]
    return c, s


def orientation_bins(gx: np.ndarray, gy: np.ndarray) -> np.ndarray:
    """Hard orientation bin in 0..17 (Sec. IV-A: one of eighteen signed
    directions; R5).

    For o = 0..8 the projection d_o = gx*c_o + gy*s_o is formed as two
    rounded float64 products and a rounded sum (no fused multiply-add).
    Scanning o upwards from best = 0, d_o > best selects bin o and
    -d_o > best selects the opposite bin o + 9; ties keep the earlier
    choice."""
    c, s = orientation_table()
    best = np.zeros(gx.shape)
    bins = np.zeros(gx.shape, np.int64)
    for o in range(NORIENT):
        d = gx * c[o] + gy * s[o]
        up = d > best
        best = np.where(up, d, best)
        bins = np.where(up, o, bins)
        dn = -d > best
        best = np.where(dn, -d, best)
        bins = np.where(dn, o + NORIENT, bins)
    return bins


# ---------------------------------------------------------- histograms
def _tent(n_pix: int):
    """Cell index and weight of the lower cell along one axis for each
    pixel: cell j is centred on pixel 8j + 3.5 (R6)."""
    xp = (np.arange(n_pix) + 0.5) / CELL - 0.5
    ix = np.floor(xp).astype(np.int64)
    return ix, xp - ix


def cell_histograms(L: np.ndarray, gx=None, gy=None):
    """18-bin histograms of 8x8 cells, hist[cy][cx][18] (Sec. IV-A,
    histogramisation).  Every pixel of the cell grid (x < 8*cx,
    y < 8*cy) adds mag * (bilinear weight) to its bin in the four nearest
    cells; weights of cells outside the grid are dropped (R4, R6)."""
    if gx is None:
        gx, gy = gradients(L)
    mag = np.sqrt(gx * gx + gy * gy)
    bins = orientation_bins(gx, gy)
    H, W = L.shape
    cy, cx = H // CELL, W // CELL
    hist = np.zeros((cy, cx, NBINS))
    iy, ay = _tent(CELL * cy)
    ix, ax = _tent(CELL * cx)
    m = mag[:CELL * cy, :CELL * cx]
    b = bins[:CELL * cy, :CELL * cx]
    for di, wy in ((0, 1.0 - ay), (1, ay)):
        ci = iy + di
        for dj, wx in ((0, 1.0 - ax), (1, ax)):
            cj = ix + dj
            v = m * wy[:, None] * wx[None, :]
            ci2 = np.broadcast_to(ci[:, None], v.shape)
            cj2 = np.broadcast_to(cj[None, :], v.shape)
            ok = (ci2 >= 0) & (ci2 < cy) & (cj2 >= 0) & (cj2 < cx)
            np.add.at(hist, (ci2[ok], cj2[ok], b[ok]), v[ok])
    return hist


def cell_energy(hist: np.ndarray) -> np.ndarray:
    """energy = sum_{n=0..8} (h_n + h_{n+9})^2 (Sec. IV-A, normalisation;
    Sec. V-A, energy kernel)."""
    u = hist[..., :NORIENT] + hist[..., NORIENT:]
    return (u * u).sum(-1)


BLOCKS = ((-1, -1), (-1, 1), (1, -1), (1, 1))


def block_energies(E: np.ndarray) -> np.ndarray:
    """B[cy][cx][4]: summed energy of the four 2x2-cell blocks that contain
    each cell, in the order of BLOCKS, with zero energy outside the grid
    (R7: the cell and its eight neighbours, grouped into four blocks)."""
    cy, cx = E.shape
    P = np.zeros((cy + 2, cx + 2))
    P[1:-1, 1:-1] = E
    B = np.empty((cy, cx, 4))
    for k, (dy, dx) in enumerate(BLOCKS):
        B[..., k] = (E + P[1 + dy:1 + dy + cy, 1:1 + cx]
                     + P[1:1 + cy, 1 + dx:1 + dx + cx]
                     + P[1 + dy:1 + dy + cy, 1 + dx:1 + dx + cx])
    return B


def features_from_hist(hist: np.ndarray) -> np.ndarray:
    """31-d cell features (Sec. IV-A, feature computation; R8):
    n_k = (B_k + eps)^-1/2 for the four blocks, T(v) = min(v, 0.2),
      F[b]      = 1/2 sum_k T(h_b n_k)                 b < 18 (signed)
      F[18 + o] = 1/2 sum_k T((h_o + h_{o+9}) n_k)     o < 9  (unsigned)
      F[27 + k] = 1/sqrt(18) sum_b T(h_b n_k)          k < 4  (energy)"""
    n = 1.0 / np.sqrt(block_energies(cell_energy(hist)) + EPS)
    u = hist[..., :NORIENT] + hist[..., NORIENT:]
    cy, cx, _ = hist.shape
    F = np.zeros((cy, cx, NFEAT))
    for k in range(4):
        nk = n[..., k:k + 1]
        t = np.minimum(hist * nk, CLIP)
        F[..., :NBINS] += 0.5 * t
        F[..., NBINS:NBINS + NORIENT] += 0.5 * np.minimum(u * nk, CLIP)
        F[..., 27 + k] = TEXTURE * t.sum(-1)
    return F


def level_features(frame: np.ndarray, lv: Level) -> np.ndarray:
    return features_from_hist(cell_histograms(resample(frame, lv)))


def pyramid_features(frame: np.ndarray, upsample: int = 1):
    H, W = np.asarray(frame).shape
    return [(lv, level_features(frame, lv)) for lv in pyramid(H, W, upsample)]


# ------------------------------------------------------------- scoring
def window_scores(F: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """S[f][r][c] = b_f + sum_{dr,dc<10} sum_{ch<31} W_f[dr][dc][ch] F[r+dr][c+dc][ch]
    for every 10x10-cell window anchored at its top-left cell (Sec. IV-A,
    classification; R9)."""
    W = np.asarray(W, np.float64)
    b = np.asarray(b, np.float64)
    cy, cx, _ = F.shape
    R, C = cy - WIN + 1, cx - WIN + 1
    S = np.zeros((W.shape[0], R, C)) + b[:, None, None]
    for dr in range(WIN):
        for dc in range(WIN):
            S += np.einsum("rcx,fx->frc", F[dr:dr + R, dc:dc + C], W[:, dr, dc])
    return S


def separable_filters(row: np.ndarray, col: np.ndarray) -> np.ndarray:
    """Full filters of row and column factors.  The paper's classifier
    kernels (Sec. V-A) filter each feature channel along the 10 horizontal
    neighbours of a cell with one set of weights (row filter, into a
    scratch image) and then along the 10 vertical neighbours with another
    (column filter), and add the channels up: a window score is then
    sum_ch sum_dr col[dr][ch] sum_dc row[dc][ch] F[r+dr][c+dc][ch], the
    linear filter W[dr][dc][ch] = col[dr][ch] row[dc][ch].  With `rank`
    such pairs per filter (row, col: [nf][rank][10][31]) the filter is
    their sum:  W_f[dr][dc][ch] = sum_i col_f,i[dr][ch] row_f,i[dc][ch]."""
    row = np.asarray(row, np.float64)
    col = np.asarray(col, np.float64)
    return np.einsum("fiaq,fibq->fabq", col, row)


def window_box(lv: Level, r, c):
    """Half-open frame-pixel box of window (r, c) of level lv: the window
    covers level pixels [8c, 8c+80) x [8r, 8r+80); each edge is mapped back
    by the fixed-point inverse scale SIG/2^40 and rounded half-up to an
    integer (R12)."""
    sig = inverse_scale_fixed(lv)
    half = 1 << (SIG_BITS - 1)

    def edge(v):
        return (np.asarray(v, np.int64) * sig + half) >> SIG_BITS

    c = np.asarray(c, np.int64)
    r = np.asarray(r, np.int64)
    return edge(8 * c), edge(8 * r), edge(8 * c + 80), edge(8 * r + 80)


# ------------------------------------ analysed levels and search regions
def face_levels(levels, min_face: int):
    """The levels analysed when every face spans at least ``min_face``
    frame pixels (R17).  Sec. V-A ("image sequence with constant size")
    skips the largest scale of 640x480 frames whose faces cover at least
    20 % of the image: there the 80x80 window is smaller than the
    smallest face (128x96), and one 5/6 step down that face is
    window-sized (107x80), so no face can be missed.  Stated per level: a
    level whose window spans fewer than min_face frame pixels,
    80 q/p < min_face, only matches faces below the minimum and is
    skipped; every later level is kept.  Exact integer test.  Sec. VI
    (scalability) uses the same rule to keep the analysed work of larger
    frames independent of their size.  min_face = 0 keeps every level."""
    return [lv for lv in levels if WIN * CELL * lv.q >= min_face * lv.p]


def window_in_region(lv: Level, r, c, region):
    """True where window (r, c) of level lv is searched under ``region`` =
    (x0, y0, x1, y1, k_lo, k_hi) (R18): its level lies in [k_lo, k_hi] and
    its frame-pixel box (R12) lies inside the half-open rectangle
    [x0, x1) x [y0, y1).  Sec. VII proposes restricting the scales and
    locations analysed in a frame, as faces move little between
    consecutive frames; None searches every window."""
    r = np.asarray(r, np.int64)
    c = np.asarray(c, np.int64)
    if region is None:
        return np.ones(np.broadcast(r, c).shape, bool)
    x0, y0, x1, y1, k_lo, k_hi = (int(v) for v in region)
    bx0, by0, bx1, by1 = window_box(lv, r, c)
    return (k_lo <= lv.k) & (lv.k <= k_hi) & (bx0 >= x0) & (by0 >= y0) & (bx1 <= x1) & (by1 <= y1)


def track_region(kept, h: int, w: int, margin: int, span: int):
    """The search region of the next frame from the kept detections of
    this one (R19; Sec. VII: faces move little between consecutive frames,
    so both the locations and the scales searched can be limited): the box
    of the best kept detection grown by ``margin`` pixels on every side and
    clipped to the h x w frame, with the levels of that detection +- span
    (clipped at level 0).  With no detection the whole frame at every
    level.  ``kept`` is in rank order (:func:`detect`)."""
    if len(kept) == 0:
        return (0, 0, w, h, 0, HUGE_LEVEL)
    d = kept[0]
    return (max(int(d["x0"]) - margin, 0), max(int(d["y0"]) - margin, 0),
            min(int(d["x1"]) + margin, w), min(int(d["y1"]) + margin, h),
            max(int(d["k"]) - span, 0), int(d["k"]) + span)


HUGE_LEVEL = 1 << 30   # level bound of a region that does not restrict levels


CAND_DTYPE = np.dtype([("score", "f8"), ("f", "i4"), ("k", "i4"), ("r", "i4"), ("c", "i4"),
                       ("x0", "i8"), ("y0", "i8"), ("x1", "i8"), ("y1", "i8")])


def level_images(frame, upsample: int = 1, cascade: bool = False):
    """(level, level image) pairs of the direct pyramid (R1, R2) or of the
    recursive one (R20)."""
    if cascade:
        return cascade_levels(frame, upsample)
    H, Wd = np.asarray(frame).shape
    return [(lv, resample(frame, lv)) for lv in pyramid(H, Wd, upsample)]


def candidates(frame, W, b, thresh: float = 0.0, upsample: int = 1, levels_out=None, min_face: int = 0,
               region=None, cascade: bool = False):
    """All windows with score strictly above the threshold, over every
    filter and pyramid level (Sec. IV-A; Sec. V-A, detection kernel;
    R10); only the levels of :func:`face_levels` and the windows of
    :func:`window_in_region`."""
    rows = []
    imgs = level_images(frame, upsample, cascade)
    keep = set(lv.k for lv in face_levels([lv for lv, _ in imgs], min_face))
    for lv, L in imgs:
        if lv.k not in keep:
            continue
        S = window_scores(features_from_hist(cell_histograms(L)), W, b)
        if levels_out is not None:
            levels_out.append((lv, S))
        f, r, c = np.nonzero(S > thresh)
        inside = window_in_region(lv, r, c, region)
        f, r, c = f[inside], r[inside], c[inside]
        if len(f) == 0:
            continue
        x0, y0, x1, y1 = window_box(lv, r, c)
        a = np.empty(len(f), CAND_DTYPE)
        a["score"], a["f"], a["k"], a["r"], a["c"] = S[f, r, c], f, lv.k, r, c
        a["x0"], a["y0"], a["x1"], a["y1"] = x0, y0, x1, y1
        rows.append(a)
    return np.concatenate(rows) if rows else np.empty(0, CAND_DTYPE)


def rank_order(c: np.ndarray) -> np.ndarray:
    """Total order of candidates: score descending, then filter, level,
    row and column ascending (R13)."""
    return np.lexsort((c["c"], c["r"], c["k"], c["f"], -c["score"]))


def nms(c: np.ndarray, iou: float = 0.5) -> np.ndarray:
    """Greedy non-maximum suppression pooled over filters and levels of a
    frame (Sec. IV-A: detections of one face reduced to the best-scoring
    one; R13).  In rank order a candidate is kept unless its IoU with an
    already kept box exceeds ``iou``; the test I > iou * U is done on exact
    integer areas (for 0.5: 2I > U)."""
    num, den = float(iou).as_integer_ratio()
    c = c[rank_order(c)]
    keep = np.zeros(len(c), bool)
    kx0 = np.empty(0, np.int64)
    ky0, kx1, ky1 = kx0.copy(), kx0.copy(), kx0.copy()
    for i in range(len(c)):
        x0, y0, x1, y1 = int(c["x0"][i]), int(c["y0"][i]), int(c["x1"][i]), int(c["y1"][i])
        if len(kx0):
            iw = np.maximum(0, np.minimum(kx1, x1) - np.maximum(kx0, x0))
            ih = np.maximum(0, np.minimum(ky1, y1) - np.maximum(ky0, y0))
            inter = iw * ih
            union = (x1 - x0) * (y1 - y0) + (kx1 - kx0) * (ky1 - ky0) - inter
            if np.any(inter * den > num * union):
                continue
        keep[i] = True
        kx0 = np.append(kx0, x0)
        ky0 = np.append(ky0, y0)
        kx1 = np.append(kx1, x1)
        ky1 = np.append(ky1, y1)
    return c[keep]


def detect(frame, W, b, thresh: float = 0.0, iou: float = 0.5, upsample: int = 1, min_face: int = 0,
           region=None, cascade: bool = False):
    """Frame in, kept face boxes and scores out, in rank order."""
    return nms(candidates(frame, W, b, thresh, upsample, min_face=min_face, region=region, cascade=cascade), iou)


# ------------------------------------------------- training (dW, db)
def hinge_loss(S, y, W, lam: float = 1e-4) -> float:
    """Mean hinge loss plus lam * ||W||^2 (bias not regularised; R15)."""
    S = np.asarray(S, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.maximum(0.0, 1.0 - y * S).mean() + lam * np.sum(np.asarray(W, np.float64) ** 2))


def hinge_dscore(S, y) -> np.ndarray:
    """d loss / d S_i = -y_i / N where y_i S_i < 1, else 0."""
    S = np.asarray(S, np.float64)
    y = np.asarray(y, np.float64)
    return np.where(y * S < 1.0, -y, 0.0) / len(S)


def filter_grad(Fw: np.ndarray, dS: np.ndarray):
    """dS/dW_f is the window's feature block and dS/db = 1, so
    dW = sum_i dS_i F_i and db = sum_i dS_i."""
    return np.tensordot(dS, Fw, axes=(0, 0)), float(np.sum(dS))


# --------------------------------------------- pixel gradient (dpixels)
def top_windows(frame, W, b, k: int = 10, upsample: int = 1):
    """The k highest window scores of a frame over every filter and level
    (all windows, before thresholding and NMS), in rank order (R14)."""
    H, Wd = np.asarray(frame).shape
    rows = []
    for lv in pyramid(H, Wd, upsample):
        S = window_scores(level_features(frame, lv), W, b)
        f, r, c = np.meshgrid(np.arange(S.shape[0]), np.arange(S.shape[1]),
                              np.arange(S.shape[2]), indexing="ij")
        a = np.empty(S.size, CAND_DTYPE)
        a["score"], a["f"], a["k"] = S.ravel(), f.ravel(), lv.k
        a["r"], a["c"] = r.ravel(), c.ravel()
        a["x0"] = a["y0"] = a["x1"] = a["y1"] = 0
        rows.append(a)
    allw = np.concatenate(rows)
    return allw[rank_order(allw)[:k]]


def level_forward(frame, lv: Level) -> dict:
    """Every intermediate of one level, for the backward pass."""
    L = resample(frame, lv)
    gx, gy = gradients(L)
    mag = np.sqrt(gx * gx + gy * gy)
    bins = orientation_bins(gx, gy)
    hist = cell_histograms(L, gx, gy)
    E = cell_energy(hist)
    B = block_energies(E)
    return dict(L=L, gx=gx, gy=gy, mag=mag, bins=bins, hist=hist, E=E, B=B,
                n=1.0 / np.sqrt(B + EPS))


def dfeatures_to_dhist(st: dict, dF: np.ndarray) -> np.ndarray:
    """Backward of the 31-d projection and the block normalisation:
    d(loss)/d(hist) from d(loss)/d(F).  Clip states (v < 0.2 passes, else
    the derivative is 0) are those of the forward pass."""
    hist, n, B = st["hist"], st["n"], st["B"]
    u = hist[..., :NORIENT] + hist[..., NORIENT:]
    dh = np.zeros_like(hist)
    du = np.zeros_like(u)
    dn = np.zeros_like(n)
    for k in range(4):
        nk = n[..., k:k + 1]
        hn = hist * nk
        pas = (hn < CLIP).astype(np.float64)
        g = 0.5 * dF[..., :NBINS] + TEXTURE * dF[..., 27 + k:28 + k]
        dh += g * pas * nk
        dn[..., k] += (g * pas * hist).sum(-1)
        un = u * nk
        pu = (un < CLIP).astype(np.float64)
        gu = 0.5 * dF[..., NBINS:NBINS + NORIENT]
        du += gu * pu * nk
        dn[..., k] += (gu * pu * u).sum(-1)
    dB = dn * (-0.5) * (B + EPS) ** -1.5
    cy, cx = dB.shape[:2]
    dE = np.zeros((cy + 2, cx + 2))
    for k, (dy, dx) in enumerate(BLOCKS):
        g = dB[..., k]
        dE[1:1 + cy, 1:1 + cx] += g
        dE[1 + dy:1 + dy + cy, 1:1 + cx] += g
        dE[1:1 + cy, 1 + dx:1 + dx + cx] += g
        dE[1 + dy:1 + dy + cy, 1 + dx:1 + dx + cx] += g
    dE = dE[1:-1, 1:-1]
    du += 2.0 * u * dE[..., None]
    dh[..., :NORIENT] += du
    dh[..., NORIENT:] += du
    return dh


def dhist_to_dlevel(st: dict, dh: np.ndarray) -> np.ndarray:
    """Backward of histogramisation, magnitude and central differences:
    d/d(level pixels) from d/d(hist).  Bins and bilinear weights are
    constants; d mag / d(gx, gy) = (gx, gy)/mag, taken as 0 at mag = 0."""
    L, gx, gy, mag, bins = st["L"], st["gx"], st["gy"], st["mag"], st["bins"]
    cy, cx, _ = dh.shape
    iy, ay = _tent(CELL * cy)
    ix, ax = _tent(CELL * cx)
    b = bins[:CELL * cy, :CELL * cx]
    dmag = np.zeros_like(L)
    acc = np.zeros((CELL * cy, CELL * cx))
    for di, wy in ((0, 1.0 - ay), (1, ay)):
        ci = iy + di
        for dj, wx in ((0, 1.0 - ax), (1, ax)):
            cj = ix + dj
            ci2 = np.broadcast_to(ci[:, None], b.shape)
            cj2 = np.broadcast_to(cj[None, :], b.shape)
            ok = (ci2 >= 0) & (ci2 < cy) & (cj2 >= 0) & (cj2 < cx)
            g = np.zeros(b.shape)
            g[ok] = dh[ci2[ok], cj2[ok], b[ok]]
            acc += g * wy[:, None] * wx[None, :]
    dmag[:CELL * cy, :CELL * cx] = acc
    safe = np.where(mag > 0, mag, 1.0)
    dgx = np.where(mag > 0, dmag * gx / safe, 0.0)
    dgy = np.where(mag > 0, dmag * gy / safe, 0.0)
    dL = np.zeros_like(L)
    dL[1:-1, 2:] += dgx[1:-1, 1:-1]
    dL[1:-1, :-2] -= dgx[1:-1, 1:-1]
    dL[2:, 1:-1] += dgy[1:-1, 1:-1]
    dL[:-2, 1:-1] -= dgy[1:-1, 1:-1]
    return dL


def topk_pixel_grad(frame, W, b, k: int = 10, upsample: int = 1, windows=None):
    """d(sum of the top-k window scores)/d(frame pixels), analytic, float64.
    Bins, clip states and the top-k membership are held at their values
    at the given frame (R14)."""
    U = np.asarray(frame, np.float64)
    H, Wd = U.shape
    if windows is None:
        windows = top_windows(U, W, b, k, upsample)
    W64 = np.asarray(W, np.float64)
    dU = np.zeros((H, Wd))
    for lv in pyramid(H, Wd, upsample):
        sel = windows[windows["k"] == lv.k]
        if len(sel) == 0:
            continue
        st = level_forward(U, lv)
        dF = np.zeros((lv.cy, lv.cx, NFEAT))
        for w in sel:
            dF[w["r"]:w["r"] + WIN, w["c"]:w["c"] + WIN] += W64[w["f"]]
        dL = dhist_to_dlevel(st, dfeatures_to_dhist(st, dF))
        dU += resample_transpose(dL, lv, H, Wd)
    return dU, windows


def topk_objective(frame, W, b, windows, upsample: int = 1) -> float:
    """Sum of the scores of the given windows, recomputed from the frame."""
    U = np.asarray(frame, np.float64)
    H, Wd = U.shape
    tot = 0.0
    for lv in pyramid(H, Wd, upsample):
        sel = windows[windows["k"] == lv.k]
        if len(sel) == 0:
            continue
        S = window_scores(level_features(U, lv), W, b)
        tot += float(S[sel["f"], sel["r"], sel["c"]].sum())
    return tot
