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
    int4 Ty[TPY], Tx[TPX];                        // row / column taps of the tile
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

// Level pixels of a tile from the frame, RS pixels per thread at a time
// with all their frame loads in flight together (taps are clamped to the
// frame, so every load is in bounds; a zero weight or a pixel outside the
// level discards the value).  IDENT: every tap weight is zero, so only the
// first sample is read.
template <bool IDENT>
__device__ __forceinline__ void resample_tile(const int4* __restrict__ sTy, const int4* __restrict__ sTx,
                                              const uint8_t* __restrict__ U, int* __restrict__ sV, int tid) {
    constexpr int RS = 6;
    for (int e0 = tid; e0 < TPY * TPX; e0 += RS * HIST_THREADS) {
        int ty[RS], tx[RS], ay[RS], bx[RS], inside[RS];
        int u00[RS], u01[RS], u10[RS], u11[RS];
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const int e = min(e0 + r * HIST_THREADS, TPY * TPX - 1);
            ty[r] = e / TPX;
            tx[r] = e - ty[r] * TPX;
            const int4 a = sTy[ty[r]], b = sTx[tx[r]];
            ay[r] = a.z;
            bx[r] = b.z;
            inside[r] = (a.w | b.w) == 0;
            u00[r] = U[(unsigned)(a.x + b.x)];
            if (!IDENT) {
                u01[r] = U[(unsigned)(a.x + b.y)];
                u10[r] = U[(unsigned)(a.y + b.x)];
                u11[r] = U[(unsigned)(a.y + b.y)];
            }
        }
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            // 24-bit multiplies (samples < 2^8, weights <= 2^8, rows < 2^16):
            // full-rate v_mul_u32_u24, where 32-bit products are quarter rate
            unsigned v;
            if (IDENT) {
                v = (unsigned)u00[r] << 16;
            } else {
                const unsigned wx1 = (unsigned)bx[r], wx0 = 256u - wx1;
                const unsigned wy1 = (unsigned)ay[r], wy0 = 256u - wy1;
                const unsigned top = __umul24(wx0, (unsigned)u00[r]) + __umul24(wx1, (unsigned)u01[r]);
                const unsigned bot = __umul24(wx0, (unsigned)u10[r]) + __umul24(wx1, (unsigned)u11[r]);
                v = __umul24(wy0, top) + __umul24(wy1, bot);
            }
            if (e0 + r * HIST_THREADS < TPY * TPX) sV[swz(ty[r], tx[r])] = inside[r] ? (int)v : 0;
        }
    }
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
                                          int pitch, const int4* __restrict__ taps, float* __restrict__ hist,
                                          int frame, int tile, int tid, HistSmem& sm,
                                          const uint8_t* __restrict__ casc = nullptr) {
    int* __restrict__ sV = sm.V;
    unsigned long long* __restrict__ sH = sm.H;
    int4* __restrict__ sTy = sm.Ty;
    int4* __restrict__ sTx = sm.Tx;
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
        for (int e = tid; e < LC_H * LC_W * CS; e += HIST_THREADS) sH[e] = 0ull;
        for (int e = tid; e < TPY + TPX; e += HIST_THREADS) {
            if (e < TPY) {
                const int y = ybase + e;
                int4 a = make_int4(0, 0, 0, -1);
                if (y >= 0 && y < L.h) {
                    const int4 tp = taps[L.tap_y + y];
                    a = make_int4(tp.x * spitch, tp.y * spitch, tp.z, 0);   // row byte offsets
                }
                sTy[e] = a;
            } else {
                const int x = xbase + e - TPY;
                sTx[e - TPY] = (x >= 0 && x < L.w) ? taps[L.tap_x + x] : make_int4(0, 0, 0, -1);
            }
        }
    }
    __syncthreads();

    // 1. resample (a level at scale 1, or a level image, is a copy of its
    // source: its taps have zero weights on the second sample)
    if (on) {
        if (L.ident) resample_tile<true>(sTy, sTx, U, sV, tid);
        else resample_tile<false>(sTy, sTx, U, sV, tid);
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
            float4* dst = reinterpret_cast<float4*>(
                hist + ((long long)frame * T.hist_frame + L.hist_off + (long long)gi * L.cx + gj) * HSTRIDE);
            dst[0] = make_float4(h[0], h[1], h[2], h[3]);
            dst[1] = make_float4(h[4], h[5], h[6], h[7]);
            dst[2] = make_float4(h[8], h[9], h[10], h[11]);
            dst[3] = make_float4(h[12], h[13], h[14], h[15]);
            dst[4] = make_float4(h[16], h[17], E, 0.f);
        }
    }
}

}  // namespace hog
