"""Seeded synthetic workloads for the HOG face detector.

The paper measures on private eyeblink-conditioning videos (grayscale
640x480, one face covering at least 20 % of the frame, blinking eyes) and
on public face datasets that are not available here.  These generators
produce frames with the same shape, value range and structure instead:
smoothed Gaussian noise as background, bright elliptical "faces" with two
dark eye blobs, and a blink cycle over a clip.

This module holds no part of the detector's arithmetic.  It is shared by
the tests, the benchmark and the CPU reference only as an input source.
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import ndimage

WIN_CELLS = 10
NFEAT = 31


def background(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """White N(0,1) noise, Gaussian-smoothed (sigma 2 px, reflect border),
    re-standardised to mean 110 / sd 30, clipped to [0,255] and rounded
    half-to-even.  Returned as float64 so callers can paint on it."""
    n = rng.standard_normal((h, w))
    s = ndimage.gaussian_filter(n, sigma=2.0, mode="reflect")
    s = (s - s.mean()) / s.std()
    return np.clip(np.rint(s * 30.0 + 110.0), 0.0, 255.0)


def _to_u8(img: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(img), 0.0, 255.0).astype(np.uint8)


def paint_face(img: np.ndarray, cy: float, cx: float, height: float,
               intensity: float, eye_h: float = 5.0, eye_w: float = 8.0,
               angle_deg: float = 0.0) -> None:
    """Paint a bright ellipse (height x 0.75*height) with two dark eye
    blobs (eye_w x eye_h px, intensity 40) in place.  Pixel centres that
    fall inside a shape take its intensity.  ``angle_deg`` rotates the
    whole face about its centre."""
    h, w = img.shape
    a = 0.5 * height          # semi-axis along y
    b = 0.375 * height        # semi-axis along x (width = 0.75 * height)
    t = np.deg2rad(angle_deg)
    ct, st = np.cos(t), np.sin(t)
    r = int(np.ceil(a)) + 2
    y0, y1 = max(0, int(cy) - r), min(h, int(cy) + r + 1)
    x0, x1 = max(0, int(cx) - r), min(w, int(cx) + r + 1)
    if y0 >= y1 or x0 >= x1:
        return
    yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    dy, dx = yy - cy, xx - cx
    # face-aligned coordinates
    u = ct * dx + st * dy
    v = -st * dx + ct * dy
    inside = (u / b) ** 2 + (v / a) ** 2 <= 1.0
    reg = img[y0:y1, x0:x1]
    reg[inside] = intensity
    width = 0.75 * height
    for sx in (-1.0, 1.0):
        eu, ev = sx * 0.22 * width, -0.12 * height
        if eye_h <= 0:
            continue
        eye = (np.abs(u - eu) <= 0.5 * eye_w) & (np.abs(v - ev) <= 0.5 * eye_h)
        reg[eye] = 40.0


def filters(seeds, sigma: float = 0.1, bias: float = -0.5):
    """Linear window filters W[f][10][10][31] ~ N(0, sigma^2), one seed per
    filter, and a constant bias per filter.  The workload's "N(0, 0.01)" is
    read as variance 0.01 (sigma 0.1)."""
    ws = [np.random.default_rng(s).normal(0.0, sigma, (WIN_CELLS, WIN_CELLS, NFEAT))
          for s in seeds]
    W = np.stack(ws).astype(np.float32)
    b = np.full(len(ws), bias, dtype=np.float32)
    return W, b


def separable_filters(seeds, rank: int = 1, bias: float = -0.5):
    """Separable filters: row and column factors [nf][rank][10][31] with
    N(0, s^2) entries, one seed per filter, s = (0.01 / rank)^(1/4), so that
    the combined weights sum_i col * row have the variance 0.01 of the full
    random filters; and a constant bias per filter."""
    sd = (0.01 / rank) ** 0.25
    rows, cols = [], []
    for s in seeds:
        rng = np.random.default_rng(s)
        rows.append(rng.normal(0.0, sd, (rank, WIN_CELLS, NFEAT)))
        cols.append(rng.normal(0.0, sd, (rank, WIN_CELLS, NFEAT)))
    b = np.full(len(rows), bias, dtype=np.float32)
    return np.stack(rows).astype(np.float32), np.stack(cols).astype(np.float32), b


@dataclasses.dataclass
class Workload:
    frames: np.ndarray            # uint8 [n][h][w]
    W: np.ndarray                 # float32 [nf][10][10][31]
    b: np.ndarray                 # float32 [nf]
    thresh: float = 0.0
    iou: float = 0.5
    upsample: int = 1


def config0(seed: int = 0) -> Workload:
    """Plain single-frame detect: one 320x240 frame with three
    non-overlapping faces 60-100 px tall; one filter."""
    rng = np.random.default_rng(seed)
    h, w = 240, 320
    img = background(rng, h, w)
    boxes = []
    while len(boxes) < 3:
        hgt = rng.uniform(60, 100)
        wid = 0.75 * hgt
        cy = rng.uniform(hgt / 2 + 1, h - hgt / 2 - 1)
        cx = rng.uniform(wid / 2 + 1, w - wid / 2 - 1)
        bb = (cy - hgt / 2, cx - wid / 2, cy + hgt / 2, cx + wid / 2)
        if any(not (bb[2] < o[0] or o[2] < bb[0] or bb[3] < o[1] or o[3] < bb[1])
               for o in boxes):
            continue
        boxes.append(bb)
        paint_face(img, cy, cx, hgt, rng.uniform(190, 215))
    W, b = filters([100])
    return Workload(_to_u8(img)[None], W, b)


def blink_height(t: int) -> int:
    """Eye-blob height over a 20-frame blink cycle: 8 -> 1 -> 8 px."""
    return 8 - int(round(7 * (1 - abs(((t % 20) - 10) / 10.0))))


class ClipGenerator:
    """Clip of consecutive frames: a static background plus N(0, 2^2)
    sensor noise per frame, one face drifting by a random walk of at most
    2 px per axis per frame (reflected at the borders), whose eye blobs
    blink over a 20-frame cycle."""

    def __init__(self, seed: int, h: int = 480, w: int = 640, face_h: float = 160.0):
        self.rng = np.random.default_rng(seed)
        self.h, self.w, self.face_h = h, w, face_h
        self.bg = background(self.rng, h, w)
        self.intensity = self.rng.uniform(190, 215)
        self.cy = self.rng.uniform(face_h / 2 + 2, h - face_h / 2 - 2)
        self.cx = self.rng.uniform(0.375 * face_h + 2, w - 0.375 * face_h - 2)
        self.t = 0

    def _step(self):
        for attr, lim in (("cy", (self.face_h / 2 + 2, self.h - self.face_h / 2 - 2)),
                          ("cx", (0.375 * self.face_h + 2, self.w - 0.375 * self.face_h - 2))):
            v = getattr(self, attr) + int(self.rng.integers(-2, 3))
            lo, hi = lim
            if v < lo:
                v = 2 * lo - v
            if v > hi:
                v = 2 * hi - v
            setattr(self, attr, min(max(v, lo), hi))

    def frame(self) -> np.ndarray:
        img = self.bg + self.rng.normal(0.0, 2.0, self.bg.shape)
        paint_face(img, self.cy, self.cx, self.face_h, self.intensity,
                   eye_h=blink_height(self.t))
        self.t += 1
        self._step()
        return _to_u8(img)

    def frames(self, n: int) -> np.ndarray:
        return np.stack([self.frame() for _ in range(n)])


def config1(seed: int = 1, n: int = 64) -> Workload:
    """Batched clip: n consecutive 640x480 frames, 5 filters."""
    W, b = filters(range(101, 106))
    return Workload(ClipGenerator(seed).frames(n), W, b)


SERVE_MIX = ((0.4, 240, 320), (0.4, 480, 640), (0.2, 720, 1280))


def config2_pools(seed: int = 2, per_res: int = 256):
    """Served stream: pre-generated frame pools per resolution (from the
    clip generator) plus the 5 clip filters."""
    pools = {}
    for i, (_, h, w) in enumerate(SERVE_MIX):
        fh = max(80.0, 160.0 * h / 480.0)
        pools[(h, w)] = ClipGenerator(seed * 1000 + i, h, w, face_h=fh).frames(per_res)
    W, b = filters(range(101, 106))
    return pools, W, b


def poisson_arrivals(seed: int, rate: float, duration_s: float):
    """Poisson arrival times (s) and resolutions drawn from SERVE_MIX."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    t = t[t < duration_s]
    probs = np.array([m[0] for m in SERVE_MIX])
    res = rng.choice(len(SERVE_MIX), size=len(t), p=probs)
    return t, [SERVE_MIX[i][1:] for i in res]


def config3(seed: int = 3, n_pos: int = 4096, n_neg: int = 16384):
    """Training crops: 80x80 positives (a face ~64 px tall, rotated within
    +-15 deg, scaled within +-10 %, shifted within +-4 px) and negatives
    (background crops).  Returns (crops u8 [n][80][80], labels +-1)."""
    rng = np.random.default_rng(seed)
    big = background(rng, 512, 512)
    crops = np.empty((n_pos + n_neg, 80, 80), np.uint8)
    for i in range(n_pos):
        img = background(rng, 80, 80)
        hgt = 64.0 * rng.uniform(0.9, 1.1)
        paint_face(img, 40 + rng.uniform(-4, 4), 40 + rng.uniform(-4, 4), hgt,
                   rng.uniform(190, 215), angle_deg=rng.uniform(-15, 15))
        crops[i] = _to_u8(img)
    for i in range(n_neg):
        y, x = rng.integers(0, 512 - 80, 2)
        crops[n_pos + i] = _to_u8(big[y:y + 80, x:x + 80])
    labels = np.concatenate([np.ones(n_pos), -np.ones(n_neg)]).astype(np.float32)
    return crops, labels


def config4(seed: int = 4, n: int = 256) -> Workload:
    """Large batch: n frames of 1920x1080 from the clip generator with a
    400 px face, analysed on a pyramid that starts at 2x the frame."""
    W, b = filters(range(101, 106))
    g = ClipGenerator(seed, 1080, 1920, face_h=400.0)
    return Workload(g.frames(n), W, b, upsample=2)
