// Device helpers shared by the gfx950 kernels.
#pragma once

#include "hog_internal.h"

namespace hog {

// cos(o*pi/9), sin(o*pi/9) for o = 0..8 as the doubles nearest to the exact
// values.  Correct rounding keeps the table mirror-symmetric:
// cos(pi - a) = -cos(a) and sin(pi - a) = sin(a) hold bit for bit.
#define HOG_C1 0.9396926207859083840541093
#define HOG_C2 0.7660444431189780352023927
#define HOG_C4 0.1736481776669303488517166
#define HOG_S1 0.3420201433256687330440996
#define HOG_S2 0.6427876096865393263226434
#define HOG_S3 0.8660254037844386467637232
#define HOG_S4 0.984807753012208059366743

static __device__ __host__ inline double dir_cos(int o) {
    switch (o) {
        case 0: return 1.0;
        case 1: return HOG_C1;
        case 2: return HOG_C2;
        case 3: return 0.5;
        case 4: return HOG_C4;
        case 5: return -HOG_C4;
        case 6: return -0.5;
        case 7: return -HOG_C2;
        default: return -HOG_C1;
    }
}
static __device__ __host__ inline double dir_sin(int o) {
    switch (o) {
        case 0: return 0.0;
        case 1: case 8: return HOG_S1;
        case 2: case 7: return HOG_S2;
        case 3: case 6: return HOG_S3;
        default: return HOG_S4;
    }
}

// Reference decision in float64: the projections d_o = gx*c_o + gy*s_o are
// formed as two rounded products and a rounded sum (no fused multiply-add);
// scanning o = 0..8 from best = 0, d_o > best picks bin o and -d_o > best
// picks the opposite bin o + 9.  Gradients are integers in units of 2^-16;
// a power-of-two scale changes no rounding, so they are used as is.
static __device__ __noinline__ int orient_bin_f64(int gxi, int gyi) {
#pragma clang fp contract(off)
    const double gx = (double)gxi, gy = (double)gyi;
    double best = 0.0;
    int bin = 0;
#pragma unroll
    for (int o = 0; o < NORIENT; ++o) {
        const double px = gx * dir_cos(o);
        const double py = gy * dir_sin(o);
        const double d = px + py;
        if (d > best) {
            best = d;
            bin = o;
        } else if (-d > best) {
            best = -d;
            bin = o + NORIENT;
        }
    }
    return bin;
}

// Orientation bin of an integer gradient (0 for a zero gradient).
//
// Fast path: fold the gradient into the first quadrant (|gx|, |gy|) and
// count how many of the sector boundaries 10, 30, 50, 70 degrees lie below
// its angle, from the signs of t_b = |gy| - |gx| tan b (the sign of
// |gy| cos b - |gx| sin b, as cos b > 0); unfold by the signs of gx, gy (an
// angle of exactly 90 or 270 degrees goes to bin 4 or 13, the first of the
// two tied directions).  |gx|, |gy| < 2^24 are exact in float32; each t_b,
// one fused multiply-add with a rounded tan b, carries an error below
// 3.3e-7 (|gx| + |gy|).  When every |t_b| exceeds 1e-6 (|gx| + |gy|) the
// signs are exact and the float64 scan above, whose own error is some
// 1e-16 of the magnitude, picks the same bin.  Otherwise the float64 scan
// itself decides.
//
// Unfolding, branch-free: j = 4 - (number of negative t_b) (no t_b is 0
// on this path).  With sx = "points left, or straight up" (gx < 0, or
// gx = 0 and gy < 0) and sy = "points up" (gy < 0), quadrant I (neither)
// has bin j, II (sx) 9 - j, III (both) 9 + j and IV (sy) 18 - j, which is
// bin 0 for j = 0.
static __device__ inline int orient_bin(int gxi, int gyi) {
    const float ax = fabsf((float)gxi), ay = fabsf((float)gyi);
    const float t0 = fmaf(-ax, 0.176326980708f, ay);   // tan 10
    const float t1 = fmaf(-ax, 0.577350269190f, ay);   // tan 30
    const float t2 = fmaf(-ax, 1.191753592594f, ay);   // tan 50
    const float t3 = fmaf(-ax, 2.747477419455f, ay);   // tan 70
    const float m = fminf(fminf(fabsf(t0), fabsf(t1)), fminf(fabsf(t2), fabsf(t3)));
    if (m <= 1e-6f * (ax + ay)) return orient_bin_f64(gxi, gyi);
    const int j = 4 - (int)((__float_as_uint(t0) >> 31) + (__float_as_uint(t1) >> 31) +
                            (__float_as_uint(t2) >> 31) + (__float_as_uint(t3) >> 31));
    const bool sy = gyi < 0;
    const bool sx = gxi < 0 || (gxi == 0 && sy);
    const int base = sx ? NORIENT : (sy ? NBINS : 0);
    const int b = (sx != sy) ? base - j : base + j;
    return b == NBINS ? 0 : b;
}

// Gradient magnitude of a voting pixel as the fixed-point integer
// round(|g| 2^6) (|g| in units of 2^-16 of a grey level, so the vote
// weight is |g| 2^22).  The square root is the hardware one (within an ulp
// of the rounded root): the quantised magnitude carries a relative error
// near 1e-7 either way, far inside the tolerance of the histograms.
static __device__ inline unsigned vote_magnitude(int gxi, int gyi) {
    const float fx = (float)gxi, fy = (float)gyi;
    const float mag = __builtin_amdgcn_sqrtf(fmaf(fx, fx, fy * fy));
    return (unsigned)(mag * 64.0f + 0.5f);
}

// Fixed-point resampling tap: returns {i0, i1, a8, 0} for output index i
// of an axis with n_in source samples at inverse scale sig (40 fractional
// bits): source coordinate ((2i+1) sig - 2^40) / 2^41, weight a8/256 on
// the second tap, rounded half-up; taps clamped to the source.
static __device__ inline int4 axis_tap(int i, int n_in, long long sig) {
    const long long t = (long long)(2 * i + 1) * sig - (1LL << SIG_BITS);
    long long base = t >> (SIG_BITS + 1);                       // floor
    const long long frac = t - (base << (SIG_BITS + 1));        // [0, 2^41)
    int a = (int)((frac + (1LL << 32)) >> 33);                  // round(256 frac / 2^41)
    if (a == 256) { base += 1; a = 0; }
    const int i0 = (int)min(max(base, 0LL), (long long)(n_in - 1));
    const int i1 = (int)min(max(base + 1, 0LL), (long long)(n_in - 1));
    return make_int4(i0, i1, a, 0);
}

// Tap i of a level axis with n_level samples: from the frame axis of
// n_src samples at the level's inverse scale, or the identity for a level
// image of the recursive pyramid (read as is).
static __device__ inline int4 level_tap(const DevLevel& L, int i, int n_level, int n_src) {
    return L.src ? make_int4(i, min(i + 1, n_level - 1), 0, 0) : axis_tap(i, n_src, L.sig);
}

// Orders a wave's LDS accesses on either side (LDS operations of one wave
// execute in program order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Frame-pixel edge of level-pixel coordinate v: round(v * sig / 2^40).
static __host__ __device__ inline int box_edge(long long v, long long sig) {
    return (int)((v * sig + (1LL << (SIG_BITS - 1))) >> SIG_BITS);
}

// Search region of a frame (hog_region): the windows of table level L
// (pyramid level k_true) whose frame-pixel boxes lie inside the region's
// rectangle, as anchor ranges [r_lo, r_hi] x [c_lo, c_hi] (empty when
// r_lo > r_hi or c_lo > c_hi, or when k_true is outside [k_lo, k_hi]).
// Box edges grow with the anchor, so the windows inside form exactly this
// product of ranges.  The first guesses invert the edge map up to a unit;
// the loops then settle the exact bounds.
struct RegionRange {
    int r_lo, r_hi, c_lo, c_hi;
    __host__ __device__ bool empty() const { return r_lo > r_hi || c_lo > c_hi; }
};

// Region coordinates are clamped to [0, 2^20] (beyond any frame side), so
// the shifted values below stay inside 64 bits.
static __host__ __device__ inline int region_lo(int lo_px, long long sig, int n) {
    // smallest a in [0, n] with box_edge(8a) >= lo_px (n: none)
    lo_px = min(max(lo_px, 0), 1 << 20);
    const long long g = ((((long long)lo_px << SIG_BITS) / sig) >> 3) - 1;
    int a = (int)min(max(g, 0LL), (long long)n);
    while (a < n && box_edge(8LL * a, sig) < lo_px) ++a;
    while (a > 0 && box_edge(8LL * (a - 1), sig) >= lo_px) --a;
    return a;
}

static __host__ __device__ inline int region_hi(int hi_px, long long sig, int n) {
    // largest a in [-1, n - 1] with box_edge(8a + 80) <= hi_px (-1: none)
    hi_px = min(max(hi_px, 0), 1 << 20);
    const long long g = ((((long long)hi_px << SIG_BITS) / sig) - 80) >> 3;
    int a = (int)min(max(g + 1, -1LL), (long long)(n - 1));
    while (a >= 0 && box_edge(8LL * a + 80, sig) > hi_px) --a;
    while (a + 1 < n && box_edge(8LL * (a + 1) + 80, sig) <= hi_px) ++a;
    return a;
}

static __host__ __device__ inline RegionRange region_range(const DevLevel& L, int k_true, const hog_region& g) {
    RegionRange R;
    if (k_true < g.k_lo || k_true > g.k_hi || L.rows <= 0 || L.cols <= 0) {
        R.r_lo = R.c_lo = 1;
        R.r_hi = R.c_hi = 0;
        return R;
    }
    R.r_lo = region_lo(g.y0, L.sig, L.rows);
    R.r_hi = region_hi(g.y1, L.sig, L.rows);
    R.c_lo = region_lo(g.x0, L.sig, L.cols);
    R.c_hi = region_hi(g.x1, L.sig, L.cols);
    return R;
}

}  // namespace hog
