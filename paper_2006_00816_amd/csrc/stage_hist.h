// Device stage: pyramid resampling, gradients, orientation and cell
// histograms of one tile of cells (Sec. IV-A: image pyramid, gradient
// computation, histogramisation; Sec. V-A: image-scaling and
// gradient-histogram kernels).  Used by the per-stage histogram kernel and
// by the fused persistent kernel.
#pragma once
#include "hog_device.h"

namespace hog {

// Level-pixel tile in LDS, swizzled so that the 64 lanes of a wave, which
// read the same offset (oy, ox) inside 64 different 8x8 pixel blocks, hit
// 64 different banks: plane (ty % 8, tx % 8), then (ty / 8, tx / 8).
constexpr int PL_W = TPX / 8 + 1;                 // 17 block columns
constexpr int PL_H = TPY / 8 + 1;                 // 9 block rows
constexpr int PLANE = PL_W * PL_H;                // 153 (odd)
constexpr int LC_W = TCX + 2, LC_H = TCY + 2;     // local cell grid 17 x 9
constexpr int CS = NBINS + 1;                     // u64 words per local cell (odd: spreads LDS banks)

// LDS of one histogram tile (64 KB).
struct HistSmem {
    int4 Ty[TPY], Tx[TPX];                        // row / column taps of the tile (see resample_tile)
    int Row[TPY];                                 // swizzled offset of each tile row
    unsigned long long H[LC_H * LC_W * CS];       // fixed-point cell histograms (see quad_votes)
    int V[64 * PLANE];                            // swizzled level pixels (value * 2^16)
};

__device__ __forceinline__ int swz(int ty, int tx) {
    return ((ty & 7) * 8 + (tx & 7)) * PLANE + (ty >> 3) * PL_W + (tx >> 3);
}

// Offset of pixel (ty, tx) relative to its quad block's origin pixel,
// ty, tx in 0..9, in the swizzled level tile.
__host__ __device__ constexpr int qoff(int ty, int tx) {
    return ((ty & 7) * 8 + (tx & 7)) * PLANE + (ty >> 3) * PL_W + (tx >> 3);
}

// Sixteen pixels (offsets 16Q .. 16Q+15 of an 8x8 quad block) of one lane:
// central differences, orientation, magnitude and four fixed-point votes.
// All LDS offsets and weights are compile-time constants.
//
// A vote is the integer M w, M = round(|g| 2^6) (|g| in units of 2^-16)
// below 2^31 and w the integer weight product (at most 225), so below
// 2^39; a cell's sum of at most 256 votes stays below 2^47.  The votes
// are summed with 64-bit integer LDS atomics, so the sums are the exact
// fixed-point totals whatever the order of the additions.  (Forming and
// summing them as float64, exact as well, made the kernel 0.29 -> 0.37 ms
// per 64-frame clip: the float64 LDS atomics are the slower path.)
template <int Q, bool CHECK>
__device__ __forceinline__ void quad_votes(const int* __restrict__ sV, int lb, unsigned long long* __restrict__ h00,
                                           int ylb, int xlb, int ylim, int xlim) {
    // the two pixel rows 2Q, 2Q + 1 of the quad block and their central
    // differences need level rows 2Q .. 2Q + 3 (tile coordinates, one-pixel
    // halo), columns 0 .. 9 of the middle two and 1 .. 8 of the outer two:
    // 36 LDS reads for 16 pixels, all issued before the first use
    int V[4][10];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 10; ++c)
            V[i][c] = ((i == 0 || i == 3) && (c == 0 || c == 9)) ? 0 : sV[lb + qoff(2 * Q + i, c)];
#pragma unroll
    for (int oo = 0; oo < 16; ++oo) {
        const int o = 16 * Q + oo;
        const int oy = o >> 3, ox = o & 7;
        const int di = oy - 2 * Q;
        if (CHECK) {
            const int yl = ylb + oy, xl = xlb + ox;
            if (yl < 1 || yl > ylim || xl < 1 || xl > xlim) continue;
        }
        const int gx = V[di + 1][ox + 2] - V[di + 1][ox];
        const int gy = V[di + 2][ox + 1] - V[di][ox + 1];
        if ((gx | gy) == 0) continue;
        const int bin = orient_bin(gx, gy);
        const unsigned long long M = vote_magnitude(gx, gy);
        atomicAdd(h00 + bin, M * (unsigned)((15 - 2 * oy) * (15 - 2 * ox)));
        atomicAdd(h00 + CS + bin, M * (unsigned)((15 - 2 * oy) * (2 * ox + 1)));
        atomicAdd(h00 + LC_W * CS + bin, M * (unsigned)((2 * oy + 1) * (15 - 2 * ox)));
        atomicAdd(h00 + (LC_W + 1) * CS + bin, M * (unsigned)((2 * oy + 1) * (2 * ox + 1)));
    }
}

template <bool CHECK>
__device__ __forceinline__ void quad_votes_q(int q, const int* sV, int lb, unsigned long long* h00, int ylb, int xlb,
                                             int ylim, int xlim) {
    switch (q) {
        case 0: quad_votes<0, CHECK>(sV, lb, h00, ylb, xlb, ylim, xlim); break;
        case 1: quad_votes<1, CHECK>(sV, lb, h00, ylb, xlb, ylim, xlim); break;
        case 2: quad_votes<2, CHECK>(sV, lb, h00, ylb, xlb, ylim, xlim); break;
        default: quad_votes<3, CHECK>(sV, lb, h00, ylb, xlb, ylim, xlim); break;
    }
}

// Level pixels of a tile from the frame, exact in integers (value * 2^16).
// Thread t takes column t mod 128 in every fourth row from row t / 128
// (rows 0 .. 63), so a column's taps stay in registers and a row's taps
// are one LDS broadcast; its seventeenth pixel is row 64 or 65 (row sets
// 0, 1) or one of the 132 pixels of columns 128, 129 (row sets 2, 3).  All
// seventeen pixels' frame loads are issued together, the histogram
// accumulators are cleared while they are in flight, then the arithmetic
// and the stores follow.
//
// Row taps a = {row 0 offset, row 1 offset, wy0, wy1}; column taps b =
// {xs, sel, wx0, wx1}: the two column samples x0, x1 (x1 = x0 + 1, or x0
// where the tap is clamped to the frame edge) are bytes x0 - xs and
// x1 - xs of the 16-bit pair at xs = min(x0, w - 2) of a row, read with
// one unaligned 16-bit load that stays inside the row; sel holds their bit
// offsets (8 (x0 - xs) and 8 (x1 - xs), in bits 0..7 and 8..15).  Weights
// in 1/256.  Taps outside the level carry zero weights, so such a pixel is
// zero (its offsets are 0: every load is in bounds).  24-bit products
// (samples < 2^8, weights <= 2^8, row sums < 2^16).  IDENT: the second
// taps have zero weight and are not read (b.x is x0 itself); the weights
// are 256 or 0, so the pixel is the sample times (wy0 & wx0) 2^8.
constexpr int RS_COLS = 128, RS_SETS = HIST_THREADS / RS_COLS, RS_PX = 17;
static_assert(RS_SETS == 4 && TPY == 66 && TPX == 130, "pixel slots below assume a 66 x 130 tile");

template <bool IDENT>
__device__ __forceinline__ unsigned resample_value(const int4& a, const int4& b, const unsigned* u) {
    if (IDENT) return __umul24((unsigned)(a.z & b.z) << 8, u[0]);
    const unsigned s0 = (unsigned)b.y & 0xffu, s1 = (unsigned)b.y >> 8;
    const unsigned top = __umul24((unsigned)b.z, __builtin_amdgcn_ubfe(u[0], s0, 8)) +
                         __umul24((unsigned)b.w, __builtin_amdgcn_ubfe(u[0], s1, 8));
    const unsigned bot = __umul24((unsigned)b.z, __builtin_amdgcn_ubfe(u[1], s0, 8)) +
                         __umul24((unsigned)b.w, __builtin_amdgcn_ubfe(u[1], s1, 8));
    return __umul24((unsigned)a.z, top) + __umul24((unsigned)a.w, bot);
}

template <bool IDENT>
__device__ __forceinline__ void resample_load(const int4& a, const int4& b, const uint8_t* __restrict__ U,
                                              unsigned* u) {
    if (IDENT) {
        u[0] = U[(unsigned)(a.x + b.x)];
    } else {
        unsigned short p0, p1;
        __builtin_memcpy(&p0, U + (unsigned)(a.x + b.x), 2);
        __builtin_memcpy(&p1, U + (unsigned)(a.y + b.x), 2);
        u[0] = p0;
        u[1] = p1;
    }
}

template <bool IDENT>
__device__ __forceinline__ void resample_tile(const int4* __restrict__ sTy, const int* __restrict__ sRow,
                                              const int4* __restrict__ sTx, const uint8_t* __restrict__ U,
                                              int* __restrict__ sV, unsigned long long* __restrict__ sH, int tid) {
    const int set = tid / RS_COLS, tx = tid % RS_COLS;
    const int4 b = sTx[tx];
    const int cp = (tx & 7) * PLANE + (tx >> 3);
    // the seventeenth pixel
    int ty16 = set + 64, cp16 = cp;
    int4 b16 = b;
    bool w16 = true;
    if (set >= 2) {
        const int e = tid - 2 * RS_COLS;   // 0 .. 255, pixels 0 .. 131 of columns 128, 129
        const int ee = min(e, 2 * TPY - 1);
        const int x = RS_COLS + (ee & 1);
        ty16 = ee >> 1;
        b16 = sTx[x];
        cp16 = (x & 7) * PLANE + (x >> 3);
        w16 = e < 2 * TPY;
    }
    unsigned u[RS_PX][2];
#pragma unroll
    for (int i = 0; i < RS_PX - 1; ++i) resample_load<IDENT>(sTy[set + RS_SETS * i], b, U, u[i]);
    resample_load<IDENT>(sTy[ty16], b16, U, u[RS_PX - 1]);
    for (int h = tid; h < LC_H * LC_W * CS; h += HIST_THREADS) sH[h] = 0ull;
#pragma unroll
    for (int i = 0; i < RS_PX - 1; ++i) {
        const int ty = set + RS_SETS * i;
        sV[sRow[ty] + cp] = (int)resample_value<IDENT>(sTy[ty], b, u[i]);
    }
    if (w16) sV[sRow[ty16] + cp16] = (int)resample_value<IDENT>(sTy[ty16], b16, u[RS_PX - 1]);
}

// One tile of TCY x TCX cells of one level of one frame, by 512 threads
// (HIST_THREADS) of a workgroup:
//  1. Level pixels of the tile (plus the pixels whose votes reach it and a
//     one-pixel gradient halo) are resampled from the frame: 8-bit
//     bilinear weights, exact in integers (value * 2^16).
//  2. Each lane owns one 8x8 quad block (the pixels between four cell
//     centres, which all vote into the same four cells) and a quarter of
//     its pixels: central differences, orientation bin, magnitude, and
//     four votes mag * wy * wx.  Votes are accumulated as 64-bit fixed
//     point (mag * 2^22 times the integer weight product out of 256) with
//     LDS integer atomics, so the sums do not depend on the order of the
//     additions.
//  3. Complete cells are converted to float (value * 2^-30) and written
//     with their energy sum_o (h_o + h_{o+9})^2 (Sec. IV-A normalisation,
//     Sec. V-A energy kernel).
// Every thread of the workgroup passes the same three barriers; tile < 0
// only takes part in them (a workgroup running two tiles side by side).
__device__ __forceinline__ void hist_tile(const LevelTable& T, const uint8_t* __restrict__ frames, long long fstride,
                                          int pitch, float* __restrict__ hist,
                                          int frame, int tile, int tid, HistSmem& sm,
                                          const uint8_t* __restrict__ casc = nullptr) {
    int* __restrict__ sV = sm.V;
    unsigned long long* __restrict__ sH = sm.H;
    int4* __restrict__ sTy = sm.Ty;
    int4* __restrict__ sTx = sm.Tx;
    int* __restrict__ sRow = sm.Row;
    const bool on = tile >= 0;
    const int k = on ? HOG_FIND_LEVEL(T, tile, th_off) : 0;
    const DevLevel& L = T.L[k];
    const int t = tile - L.th_off;
    const int tiles_x = (L.cx + TCX - 1) / TCX;
    const int i0 = (t / tiles_x) * TCY, j0 = (t % tiles_x) * TCX;
    const int ybase = 8 * i0 - 5, xbase = 8 * j0 - 5;   // level coords of tile pixel (0, 0)
    // the level's source: the frame (sampled through the taps), or its
    // 8-bit image of the recursive pyramid (identity taps)
    const bool own = on && L.src && casc != nullptr;
    const uint8_t* __restrict__ U = frames + (long long)frame * fstride;
    int spitch = pitch;
    if (own) {
        U = casc + (long long)frame * T.casc_frame + L.src_off;
        spitch = L.w;
    }

    if (on) {
        // taps {offset 0, offset 1, weight 0, weight 1} of the tile's rows
        // and columns, computed from the level's scale: row offsets in
        // bytes; zero weights outside the level
        for (int e = tid; e < TPY + TPX; e += HIST_THREADS) {
            if (e < TPY) {
                const int y = ybase + e;
                int4 a = make_int4(0, 0, 0, 0);
                if (y >= 0 && y < L.h) {
                    const int4 tp = level_tap(L, y, L.h, T.h);
                    a = make_int4(tp.x * spitch, tp.y * spitch, 256 - tp.z, tp.z);
                }
                sTy[e] = a;
                sRow[e] = (e & 7) * 8 * PLANE + (e >> 3) * PL_W;
            } else {
                const int x = xbase + e - TPY;
                int4 b = make_int4(0, 0, 0, 0);
                if (x >= 0 && x < L.w) {
                    const int4 tp = level_tap(L, x, L.w, T.w);
                    // the source row's width: the level image's, or the frame's
                    const int ws = L.src ? L.w : T.w;
                    const int xs = L.ident ? tp.x : max(min(tp.x, ws - 2), 0);
                    b = make_int4(xs, 8 * (tp.x - xs) | (8 * (tp.y - xs)) << 8, 256 - tp.z, tp.z);
                }
                sTx[e - TPY] = b;
            }
        }
    }
    __syncthreads();

    // 1. resample (a level at scale 1, or a level image, is a copy of its
    // source: its taps have zero weights on the second sample)
    if (on) {
        if (L.ident) resample_tile<true>(sTy, sRow, sTx, U, sV, sH, tid);
        else resample_tile<false>(sTy, sRow, sTx, U, sV, sH, tid);
    }
    __syncthreads();

    // 2. gradients, orientation, votes
    if (on) {
        const int wave = tid >> 6, lane = tid & 63;
        const int qa = (wave & 1) * 4 + (lane >> 4);      // quad-block row 0..7
        const int qb = lane & 15;                         // quad-block column 0..15
        const int q = wave >> 1;                          // quarter of the 64 pixel offsets
        const int lb = qa * PL_W + qb;                    // swizzled base of the quad block
        unsigned long long* h00 = &sH[(qa * LC_W + qb) * CS];
        // valid pixels: 1 <= y <= min(8 cy - 1, h - 2), same for x
        const int ylim = min(8 * L.cy - 1, L.h - 2), xlim = min(8 * L.cx - 1, L.w - 2);
        const bool inner =
            ybase + 1 >= 1 && ybase + TPY - 2 <= ylim && xbase + 1 >= 1 && xbase + TPX - 2 <= xlim;
        const int ylb = ybase + 8 * qa + 1, xlb = xbase + 8 * qb + 1;
        if (inner) quad_votes_q<false>(q, sV, lb, h00, ylb, xlb, ylim, xlim);
        else quad_votes_q<true>(q, sV, lb, h00, ylb, xlb, ylim, xlim);
    }
    __syncthreads();

    // 3. complete cells -> float histograms + energy
    if (on && tid < TCY * TCX) {
        const int li = tid / TCX, lj = tid - li * TCX;
        const int gi = i0 + li, gj = j0 + lj;
        if (gi < L.cy && gj < L.cx) {
            const unsigned long long* src = &sH[((li + 1) * LC_W + lj + 1) * CS];
            float h[NBINS];
#pragma unroll
            for (int b = 0; b < NBINS; ++b) h[b] = (float)((double)src[b] * 0x1p-30);
            float E = 0.f;
#pragma unroll
            for (int o = 0; o < NORIENT; ++o) {
                const float u = h[o] + h[o + NORIENT];
                E = fmaf(u, u, E);
            }
            // part-major records: part q of cell c at plane q, entry c
            const long long ncell = (long long)L.cy * L.cx;
            float4* dst = reinterpret_cast<float4*>(hist + ((long long)frame * T.hist_frame + L.hist_off) * HSTRIDE) +
                          (long long)gi * L.cx + gj;
            dst[0] = make_float4(h[0], h[1], h[2], h[3]);
            dst[ncell] = make_float4(h[4], h[5], h[6], h[7]);
            dst[2 * ncell] = make_float4(h[8], h[9], h[10], h[11]);
            dst[3 * ncell] = make_float4(h[12], h[13], h[14], h[15]);
            dst[4 * ncell] = make_float4(h[16], h[17], E, 0.f);
        }
    }
}

}  // namespace hog
