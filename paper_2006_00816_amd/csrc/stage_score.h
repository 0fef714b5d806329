// Device stage: linear window scoring on the matrix cores (Sec. IV-A
// linear classification; Sec. V-A classifier and detection kernels).  Used
// by the per-stage scoring kernel and by the fused persistent kernel.
#pragma once
#include "hog_device.h"

namespace hog {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// LDS of one scoring item of ROWS window rows (one wave each): the filter
// group's packed B (62.5 KB) and, per wave, the partial products of one M
// tile stored column-major, P[(f, dc)][x] (4 KB).
template <int ROWS>
struct ScoreSmemT {
    float4 B[BPACK_PER_GROUP];
    float P[ROWS][SC_RING];
};
using ScoreSmem = ScoreSmemT<ROWS_PER_ITEM>;

// LDS of one scoring item with split fp16 operands (HOG_ARITH_F16X3): the
// group's packed B16 (80 KB) and the per-wave partial-product tiles.
template <int ROWS>
struct Score16SmemT {
    uint4 B[B16_PER_GROUP];
    float P[ROWS][SC_RING];
};

template <int ROWS>
__device__ __forceinline__ void load_bpack(ScoreSmemT<ROWS>& sm, const float4* __restrict__ bpack, int grp,
                                           int tid) {
    const float4* __restrict__ g = bpack + (long long)grp * BPACK_PER_GROUP;
    for (int e = tid; e < BPACK_PER_GROUP; e += ROWS * 64) sm.B[e] = g[e];
}

template <int ROWS>
__device__ __forceinline__ void load_bpack(Score16SmemT<ROWS>& sm, const float4* __restrict__ bpack, int grp,
                                           int tid) {
    const uint4* __restrict__ g = reinterpret_cast<const uint4*>(bpack) + (long long)grp * B16_PER_GROUP;
    for (int e = tid; e < B16_PER_GROUP; e += ROWS * 64) sm.B[e] = g[e];
}

// Tiles [tb, te) of part `part` of a row of ntiles M tiles split over
// `parts` slots.  Every part after the first recomputes the tile before
// its range for the carry, so the first part takes one tile more: with
// c = ceil((ntiles + parts - 1) / parts) the parts' costs in tile times
// are all at most c (5 tiles: 3 + 2 for two parts, 2 + 1 + 1 + 1 for four).
__device__ __forceinline__ void row_part_tiles(int ntiles, int part, int parts, int& tb, int& te) {
    const int c = (ntiles + 2 * parts - 2) / parts;
    tb = part == 0 ? 0 : min(ntiles, c + (part - 1) * (c - 1));
    te = min(ntiles, c + part * (c - 1));
}

// Window scores of M tile t of window row r from the tile's partial
// products in `ring`, stored column-major: P[(f, dc)][x] at
// ring[(10 f + dc) * SC_RSTR + x] for the 16 cells x of the tile (f the
// filter of the group, dc the window column).  Lane (g4, j) sums filter g4
// (and, with XTRA, filter 4) for window c = 16 t - 9 + j; the terms of
// window c + 16 that lie in this tile are carried to the next tile in
// carry0 / carry1.  Writes the dense scores (optional) and the best
// candidate key per window position, as score_row describes.
template <bool XTRA>
__device__ __forceinline__ void tile_windows(const DevLevel& L, int k, int r, int t, int t_begin,
                                             const float* __restrict__ ring, float& carry0, float& carry1, int g4,
                                             int j, int f0, int f1, bool f0ok, bool f1ok, float b0, float b1,
                                             float thresh, float* __restrict__ D, unsigned long long* __restrict__ PK,
                                             int atomic_key, int c_lo, int c_hi) {
    // Window c = 16 t - 9 + j takes P[c + dc] for dc >= 9 - j (cells of
    // this tile) and window c + 16 starts its carry with the cells
    // 7 + j + dc <= 15 of this tile; both are cell (7 + j + dc) mod 16,
    // so one read per dc, added to one sum or the other (zeros keep
    // the order of the additions).
    float s0 = carry0, s1 = carry1, n0 = 0.f, n1 = 0.f;
#pragma unroll
    for (int dc = 0; dc < WIN; ++dc) {
        const bool mine = dc >= WIN - 1 - j;
        const float* p = ring + dc * SC_RSTR + ((j + 7 + dc) & 15);
        const float v0 = p[WIN * SC_RSTR * g4];
        s0 += mine ? v0 : 0.f;
        n0 += mine ? 0.f : v0;
        if (XTRA) {
            const float v1 = p[WIN * SC_RSTR * 4];
            s1 += mine ? v1 : 0.f;
            n1 += mine ? 0.f : v1;
        }
    }
    carry0 = n0;
    carry1 = n1;
    wave_lds_order();
    if (t < t_begin) return;   // carry-only tile

    const int c = 16 * t - (WIN - 1) + j;
    const bool cok = c >= 0 && c < L.cols;
    // only windows inside the search region become candidates
    const bool cin = c >= c_lo && c <= c_hi;
    unsigned long long key = 0ull;
    if (cok) {
        s0 += b0;
        s1 += b1;
        if (D) {
            if (f0ok) D[((long long)f0 * L.rows + r) * L.cols + c] = s0;
            if (f1ok) D[((long long)f1 * L.rows + r) * L.cols + c] = s1;
        }
    }
    if (cok && cin) {
        if (f0ok && s0 > thresh)
            key = ((unsigned long long)score_order(s0) << 32) | (unsigned long long)(~pack_window(f0, k, r, c));
        if (f1ok && s1 > thresh) {
            const unsigned long long k1 =
                ((unsigned long long)score_order(s1) << 32) | (unsigned long long)(~pack_window(f1, k, r, c));
            key = k1 > key ? k1 : key;
        }
    }
    // best over the group's filters of the same window: lanes j, j + 16, j + 32, j + 48
#pragma unroll
    for (int sft = 16; sft < 64; sft <<= 1) {
        const unsigned long long o = __shfl_xor(key, sft, 64);
        key = o > key ? o : key;
    }
    if (PK && cok && g4 == 0) {
        if (atomic_key) {
            if (key) atomicMax(PK + c, key);
        } else {
            PK[c] = key;
        }
    }
}

// Search region of one window row (wave-uniform): narrows the tiles
// [tb, te) of the row to those holding windows inside the frame's region
// (empty if the row has none) and returns the region's window columns
// [c_lo, c_hi].  Positions of [tb, te) outside the narrowed tiles get key 0
// here (the tile walk writes the others), unless keys merge by atomic max,
// which start at zero.  Without a region nothing changes.
__device__ __forceinline__ void region_row(const LevelTable& T, const DevLevel& L, int k, int r,
                                           const hog_region* __restrict__ reg, unsigned long long* __restrict__ PKfr,
                                           int atomic_key, int lane, int& tb, int& te, int& c_lo, int& c_hi) {
    c_lo = 0;
    c_hi = L.cols - 1;
    if (!reg) return;
    const RegionRange R = region_range(L, k + T.k_base, *reg);
    int nb = te, ne = te;
    if (!R.empty() && r >= R.r_lo && r <= R.r_hi) {
        c_lo = R.c_lo;
        c_hi = R.c_hi;
        // window c = 16 t - 9 + j lies in tile (c + 9) / 16
        nb = max(tb, (R.c_lo + WIN - 1) >> 4);
        ne = min(te, ((R.c_hi + WIN - 1) >> 4) + 1);
        if (nb >= ne) nb = ne = te;
    }
    if (PKfr && !atomic_key) {
        unsigned long long* __restrict__ PK = PKfr + L.pos_off + (long long)r * L.cols;
        const int a0 = max(16 * tb - (WIN - 1), 0), a1 = min(16 * nb - (WIN - 1), L.cols);
        for (int c = a0 + lane; c < a1; c += 64) PK[c] = 0ull;
        const int b0 = max(16 * ne - (WIN - 1), 0), b1 = min(16 * te - (WIN - 1), L.cols);
        for (int c = b0 + lane; c < b1; c += 64) PK[c] = 0ull;
    }
    tb = nb;
    te = ne;
}

// The score of filter f at window (r, c) is bias_f plus the 3100-term dot
// product of the filter with the window's 10x10x31 features.  For one
// window row r:
//   P[x][(f, dc)] = sum over dr, ch of F[r + dr][x][ch] W_f[dr][dc][ch]
//     (M = cell column x, N = (filter f of a group of 5, window column
//      dc), K = (dr, ch) = 320 with channel 31 zero),
//   S_f(r, c) = bias_f + sum over dc = 0..9 of P[c + dc][(f, dc)].
// Columns 0..16 NT - 1 run on v_mfma_f32_16x16x4_f32: a lane reads 4
// consecutive channels of one cell as a float4 and feeds them to 4
// consecutive MFMAs against B packed to match.  With XTRA the columns
// (f = 4, dc = 8, 9) run on the vector ALUs from the same float4: each lane
// sums its 4 channels over all K chunks, then the 4 lanes of a cell are
// added in a fixed tree.
//
// The row is walked in M tiles of 16 cells.  Window c = 16 t - 9 + j of
// lane j takes the terms dc >= 9 - j from tile t and carries, in a
// register, the terms dc < 9 - j from tile t - 1; the sum runs over dc in
// increasing order either way.  Outputs: the dense score map (optional)
// and, per window position, the best candidate key over the group's
// filters (0 if no filter's score exceeds the threshold), stored or merged
// with atomic max.
//
// Tiles [t_begin, t_end) of the row are output.  A range that starts
// inside the row first recomputes tile t_begin - 1 for the carry alone, so
// every output takes the same operands in the same order as a whole-row
// walk: the same bits.
template <int NT, bool XTRA, int ROWS>
__device__ __forceinline__ void score_row(const DevLevel& L, int k, int r, const float* __restrict__ Ffr,
                                          const ScoreSmemT<ROWS>& sm, float* __restrict__ ring, int grp, int nf,
                                          const float* __restrict__ bias, float thresh, float* __restrict__ Dfr,
                                          unsigned long long* __restrict__ PKfr, int atomic_key, int lane,
                                          int t_begin, int t_end, int c_lo, int c_hi) {
    const int g4 = lane >> 4, j = lane & 15;
    // row pitch and half-plane stride of the feature maps (channels 0..15
    // of the row's cells, then 16..31)
    const int pitch = (L.cx + 2) * FPAD, hp = (L.cx + 2) * FHALF;
    const float* __restrict__ Fr = Ffr + L.feat_off + (long long)r * pitch + 4 * g4;
    const int f0 = grp * FGROUP + g4, f1 = f0 + 4;
    const bool f0ok = f0 < nf, f1ok = XTRA && g4 == 0;
    const float b0 = f0ok ? bias[f0] : 0.f, b1 = f1ok ? bias[f1] : 0.f;
    float* __restrict__ D = Dfr ? Dfr + L.sc_off : nullptr;
    unsigned long long* __restrict__ PK = PKfr ? PKfr + L.pos_off + (long long)r * L.cols : nullptr;
    const float4* __restrict__ X = sm.B + BPACK_MFMA + 2 * g4;
    const int ntiles = t_end;
    const int t_first = max(t_begin - 1, 0);
    float carry0 = 0.f, carry1 = 0.f;
    // the first two K chunks of the next tile, loaded while the current
    // tile's epilogue runs
    float4 a0n, a1n;
    {
        const float* __restrict__ a = Fr + min(16 * t_first + j, L.cx + 1) * FHALF;
        a0n = *reinterpret_cast<const float4*>(a);
        a1n = *reinterpret_cast<const float4*>(a + hp);
    }

    for (int t = t_first; t < ntiles; ++t) {
        floatx4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        float x8 = 0.f, x9 = 0.f;
        // cells past the last window's reach (x >= cx) are never summed.
        // The operand of K chunk kc + 2 is loaded while chunk kc computes;
        // the MFMAs of one chunk alternate between the N tiles so that
        // consecutive ones are independent.
        const float* __restrict__ a = Fr + min(16 * t + j, L.cx + 1) * FHALF;
        auto load_a = [&](int kc) {
            return *reinterpret_cast<const float4*>(a + (kc >> 1) * pitch + (kc & 1) * hp);
        };
        float4 av[SC_KC];
        av[0] = a0n;
        av[1] = a1n;
        // B of chunk kc + 1 is read from LDS while chunk kc computes
        float4 bb[2][NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bb[0][nt] = sm.B[nt * 64 + lane];
#pragma unroll
        for (int kc = 0; kc < SC_KC; ++kc) {
            if (kc + 2 < SC_KC) av[kc + 2] = load_a(kc + 2);
            if (kc + 1 < SC_KC) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) bb[(kc + 1) & 1][nt] = sm.B[((kc + 1) * SC_NT + nt) * 64 + lane];
            }
            const float4* b = bb[kc & 1];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kc].x, b[nt].x, acc[nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kc].y, b[nt].y, acc[nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kc].z, b[nt].z, acc[nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kc].w, b[nt].w, acc[nt], 0, 0, 0);
            if (XTRA) {
                const float4 w8 = X[kc * 8], w9 = X[kc * 8 + 1];
                x8 = fmaf(av[kc].x, w8.x, x8);
                x8 = fmaf(av[kc].y, w8.y, x8);
                x8 = fmaf(av[kc].z, w8.z, x8);
                x8 = fmaf(av[kc].w, w8.w, x8);
                x9 = fmaf(av[kc].x, w9.x, x9);
                x9 = fmaf(av[kc].y, w9.y, x9);
                x9 = fmaf(av[kc].z, w9.z, x9);
                x9 = fmaf(av[kc].w, w9.w, x9);
            }
        }
        if (XTRA) {
            x8 += __shfl_xor(x8, 16, 64);
            x9 += __shfl_xor(x9, 16, 64);
            x8 += __shfl_xor(x8, 32, 64);
            x9 += __shfl_xor(x9, 32, 64);
        }
        // lane (g4, j) holds P[16 t + 4 g4 + i][16 nt + j], i = 0..3: one
        // 16-byte store per N tile into the column-major tile
        wave_lds_order();
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            *reinterpret_cast<float4*>(ring + (16 * nt + j) * SC_RSTR + 4 * g4) =
                make_float4(acc[nt][0], acc[nt][1], acc[nt][2], acc[nt][3]);
        if (XTRA && g4 == 0) {
            ring[48 * SC_RSTR + j] = x8;
            ring[49 * SC_RSTR + j] = x9;
        }
        if (t + 1 < ntiles) {
            const float* __restrict__ an = Fr + min(16 * (t + 1) + j, L.cx + 1) * FHALF;
            a0n = *reinterpret_cast<const float4*>(an);
            a1n = *reinterpret_cast<const float4*>(an + hp);
        }
        wave_lds_order();

        tile_windows<XTRA>(L, k, r, t, t_begin, ring, carry0, carry1, g4, j, f0, f1, f0ok, f1ok, b0, b1, thresh, D,
                           PK, atomic_key, c_lo, c_hi);
    }
}

// ------------------------- FP32-accurate scoring from fp16 matrix products
// With HOG_ARITH_F16X3 every operand v (feature or weight) is split into
// v_hi = fp16(v) and v_lo = fp16((v - v_hi) 2^11), both rounded to
// nearest, so that v = v_hi + 2^-11 v_lo to within 2^-23 |v| + 2^-36 (for
// |v| below 2^15; v - v_hi and the scaling are exact in FP32).  A product is
//   x w = x_hi w_hi + 2^-11 (x_hi w_lo + x_lo w_hi) + 2^-22 x_lo w_lo,
// of which the last term (at most 2^-22 |x w|) is dropped.  Products of
// fp16 values are exact in FP32 and v_mfma_f32_16x16x32_f16 sums them in
// FP32, the first term into one accumulator and the two cross terms into
// another: P = acc_hi + 2^-11 acc_cross.  This is the split-operand
// scheme of Ootomo and Yokota (2022), which recovers single-precision
// accuracy from half-precision matrix units; the scale 2^11 keeps the
// low parts out of the fp16 subnormal range.
//
// Operand layout (the same for A and B, so any K order the hardware uses
// pairs them alike): one MFMA per feature row dr of the window, K = the
// 32 channels; lane (g4, j) holds channels 8 g4 .. 8 g4 + 7 of cell
// 16 t + j (A) or of column 16 nt + j (B).  The feature kernel stores
// each cell's split operands in its 128 bytes (32 hi halves, then 32 lo
// halves), so a lane's A operands are two 16-byte loads.  B16 entry
// ((dr B16_NT + nt) 2 + part) 64 + lane holds the hi (part 0) or lo
// (part 1) halves of that lane.  All 50 columns (f, dc) run on the matrix
// cores: N tile 3 holds columns 48, 49 (f = 4, dc = 8, 9).
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// One window row r with split fp16 operands; NT N tiles (4 for a group of
// 5 filters, fewer for smaller groups); arguments and outputs as score_row,
// with the same tile walk, carry and epilogue.
template <int NT, bool XTRA, int ROWS>
__device__ __forceinline__ void score_row16(const DevLevel& L, int k, int r, const float* __restrict__ Ffr,
                                            const Score16SmemT<ROWS>& sm, float* __restrict__ ring, int grp, int nf,
                                            const float* __restrict__ bias, float thresh, float* __restrict__ Dfr,
                                            unsigned long long* __restrict__ PKfr, int atomic_key, int lane,
                                            int t_begin, int t_end, int c_lo, int c_hi) {
    static_assert(!XTRA || NT == 4, "a group of 5 filters needs 4 N tiles");
    const int g4 = lane >> 4, j = lane & 15;
    const int pitch = (L.cx + 2) * FPAD, hp = (L.cx + 2) * FHALF;
    // the cell's hi halves of channels 8 g4 .. 8 g4 + 7 at float 4 g4 of its
    // 16 floats in the first half-plane, the lo halves in the second
    const float* __restrict__ Fr = Ffr + L.feat_off + (long long)r * pitch + 4 * g4;
    const int f0 = grp * FGROUP + g4, f1 = f0 + 4;
    const bool f0ok = f0 < nf, f1ok = XTRA && g4 == 0;
    const float b0 = f0ok ? bias[f0] : 0.f, b1 = f1ok ? bias[f1] : 0.f;
    float* __restrict__ D = Dfr ? Dfr + L.sc_off : nullptr;
    unsigned long long* __restrict__ PK = PKfr ? PKfr + L.pos_off + (long long)r * L.cols : nullptr;
    const uint4* __restrict__ Bl = sm.B + lane;
    const int t_first = max(t_begin - 1, 0);
    float carry0 = 0.f, carry1 = 0.f;
    for (int t = t_first; t < t_end; ++t) {
        const float* __restrict__ a = Fr + min(16 * t + j, L.cx + 1) * FHALF;
        floatx4 ah[NT], ac[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) ah[nt] = ac[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
        // feature rows dr + 1 and dr + 2 are loaded while row dr computes
        uint4 x[3][2];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            x[d][0] = *reinterpret_cast<const uint4*>(a + d * pitch);
            x[d][1] = *reinterpret_cast<const uint4*>(a + d * pitch + hp);
        }
#pragma unroll
        for (int dr = 0; dr < WIN; ++dr) {
            if (dr + 2 < WIN) {
                x[(dr + 2) % 3][0] = *reinterpret_cast<const uint4*>(a + (dr + 2) * pitch);
                x[(dr + 2) % 3][1] = *reinterpret_cast<const uint4*>(a + (dr + 2) * pitch + hp);
            }
            const halfx8 hi = __builtin_bit_cast(halfx8, x[dr % 3][0]);
            const halfx8 lo = __builtin_bit_cast(halfx8, x[dr % 3][1]);
            const uint4* __restrict__ b = Bl + dr * (B16_NT * 2 * 64);
            halfx8 bh[NT], bl[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                bh[nt] = __builtin_bit_cast(halfx8, b[(2 * nt) * 64]);
                bl[nt] = __builtin_bit_cast(halfx8, b[(2 * nt + 1) * 64]);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) ah[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, bh[nt], ah[nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) ac[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, bl[nt], ac[nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) ac[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, bh[nt], ac[nt], 0, 0, 0);
        }
        // lane (g4, j) holds P[16 t + 4 g4 + i][16 nt + j], i = 0..3
        wave_lds_order();
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const float4 v = make_float4(fmaf(ac[nt][0], 0x1p-11f, ah[nt][0]), fmaf(ac[nt][1], 0x1p-11f, ah[nt][1]),
                                         fmaf(ac[nt][2], 0x1p-11f, ah[nt][2]), fmaf(ac[nt][3], 0x1p-11f, ah[nt][3]));
            if (nt < 3 || j < 2) *reinterpret_cast<float4*>(ring + (16 * nt + j) * SC_RSTR + 4 * g4) = v;
        }
        wave_lds_order();
        tile_windows<XTRA>(L, k, r, t, t_begin, ring, carry0, carry1, g4, j, f0, f1, f0ok, f1ok, b0, b1, thresh, D,
                           PK, atomic_key, c_lo, c_hi);
    }
}

// One scoring item: window rows q = ROWS * item + wave of the frame's list
// of rows (levels in order), filter group grp; sm.B holds the group's B.
// Waves past the last row do nothing.  part < 0: whole rows; part =
// 0 .. parts - 1: that part of the row's M tiles (row_part_tiles; a part
// can be empty).
template <int ROWS, bool F16 = false, class SM>
__device__ __forceinline__ void score_item(const LevelTable& T, int frame, int grp, int item, const SM& sm,
                                           float* __restrict__ ring, const float* __restrict__ feat, int nf,
                                           const float* __restrict__ bias, float thresh, float* __restrict__ dense,
                                           unsigned long long* __restrict__ poskey, int atomic_key, int tid,
                                           int part = -1, const hog_region* __restrict__ regions = nullptr,
                                           int parts = 2) {
    // the wave's row, made wave-uniform so that the level's fields live in
    // scalar registers
    const int q = item * ROWS + __builtin_amdgcn_readfirstlane(tid >> 6);
    if (q >= T.rows_total) return;
    const int k = HOG_FIND_LEVEL(T, q, row_off);
    const DevLevel& L = T.L[k];
    const int r = q - L.row_off;
    const float* Ffr = feat + (long long)frame * T.feat_frame;
    float* Dfr = dense ? dense + (long long)frame * T.dense_frame : nullptr;
    unsigned long long* PKfr = poskey ? poskey + (long long)frame * T.pos_frame : nullptr;
    const int fg = min(FGROUP, nf - grp * FGROUP);
    const int lane = tid & 63;
    const int ntiles = (L.cx + 15) >> 4;
    int tb = 0, te = ntiles;
    if (part >= 0) {
        row_part_tiles(ntiles, part, parts, tb, te);
        if (tb >= te) return;
    }
    int c_lo, c_hi;
    region_row(T, L, k, r, regions ? regions + frame : nullptr, PKfr, atomic_key, lane, tb, te, c_lo, c_hi);
    if (tb >= te) return;
    if constexpr (F16) {
        // N tiles of 16 columns (f, dc) that the group's filters fill
        if (fg == 5)
            score_row16<4, true, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane, tb,
                                       te, c_lo, c_hi);
        else if (fg >= 4)
            score_row16<3, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane,
                                        tb, te, c_lo, c_hi);
        else if (fg >= 2)
            score_row16<2, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane,
                                        tb, te, c_lo, c_hi);
        else
            score_row16<1, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane,
                                        tb, te, c_lo, c_hi);
    } else {
        if (fg == 5)
            score_row<3, true, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane, tb,
                                     te, c_lo, c_hi);
        else if (fg == 4)
            score_row<3, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane, tb,
                                      te, c_lo, c_hi);
        else if (fg >= 2)
            score_row<2, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane, tb,
                                      te, c_lo, c_hi);
        else
            score_row<1, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane, tb,
                                      te, c_lo, c_hi);
    }
}

// ------------------------------------------- separable (row / column) filters
// The paper's classifier kernels (Sec. V-A) filter every feature channel
// along the 10 horizontal neighbours of a cell with a row filter and then
// along the 10 vertical neighbours with a column filter.  A filter made of
// RANK such pairs per channel, W_f[dr][dc][ch] = sum_i col_f,i[dr][ch]
// row_f,i[dc][ch], is scored here in the other order, which suits the
// matrix cores: for window row r,
//   G_f,i[x][ch] = sum_dr col_f,i[dr][ch] F[r + dr][x][ch]      (vector ALUs)
//   P[x][(f, dc)] = sum_i sum_ch G_f,i[x][ch] row_f,i[dc][ch]   (matrix cores)
// and then S_f(r, c) = bias_f + sum_dc P[c + dc][(f, dc)] exactly as for a
// full filter (tile_windows).  The contraction has K = 32 RANK per filter
// instead of 320, and the column pass 10 multiply-adds per (cell, channel,
// filter, pair).

// LDS of a separable scoring item: per filter f of the group and pair i the
// column factor colw[f][i][dr][32] (channel 31 zero) and the row factor as
// MFMA B operands B[f][i][kc][lane] = the four K values (channels)
// 16 kc + 4 (lane / 16) + s, s = 0..3, of column dc = lane % 16 (zero for
// dc >= 10); then per wave the partial-product tile.
template <int ROWS, int RANK>
struct SepSmemT {
    float4 B[FGROUP * RANK * 2 * 64];
    float colw[FGROUP * RANK * WIN * FPAD];
    float P[ROWS][SC_RING];
};

// Fills the factors of filter group grp from row / col [nf][RANK][10][31].
template <int ROWS, int RANK>
__device__ __forceinline__ void load_sep(SepSmemT<ROWS, RANK>& sm, const float* __restrict__ row,
                                         const float* __restrict__ col, int nf, int grp, int tid) {
    for (int e = tid; e < FGROUP * RANK * WIN * FPAD; e += ROWS * 64) {
        const int ch = e % FPAD, dr = (e / FPAD) % WIN, fi = e / (FPAD * WIN);
        const int f = grp * FGROUP + fi / RANK, i = fi % RANK;
        sm.colw[e] = (f < nf && ch < NFEAT) ? col[((f * RANK + i) * WIN + dr) * NFEAT + ch] : 0.f;
    }
    for (int e = tid; e < FGROUP * RANK * 2 * 64; e += ROWS * 64) {
        const int ln = e & 63, kc = (e >> 6) & 1, fi = e >> 7;
        const int f = grp * FGROUP + fi / RANK, i = fi % RANK;
        const int dc = ln & 15, ch0 = 16 * kc + 4 * (ln >> 4);
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ch = ch0 + q;
            v[q] = (f < nf && dc < WIN && ch < NFEAT) ? row[((f * RANK + i) * WIN + dc) * NFEAT + ch] : 0.f;
        }
        sm.B[e] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// One window row r with separable filters; arguments and outputs as
// score_row.  Lane (g4, j) reads the float4 of channels 16 kc + 4 g4 ..
// + 3 of cell 16 t + j in the ten feature rows r .. r + 9, forms G for
// those channels (the A operand of four MFMAs per chunk kc), and holds
// P[16 t + 4 g4 + q][dc = j] of each filter after the contraction.
template <int RANK, bool XTRA, int ROWS>
__device__ __forceinline__ void score_row_sep(const DevLevel& L, int k, int r, const float* __restrict__ Ffr,
                                              const SepSmemT<ROWS, RANK>& sm, float* __restrict__ ring, int grp,
                                              int nf, const float* __restrict__ bias, float thresh,
                                              float* __restrict__ Dfr, unsigned long long* __restrict__ PKfr,
                                              int atomic_key, int lane, int t_begin, int t_end, int c_lo,
                                              int c_hi) {
    const int g4 = lane >> 4, j = lane & 15;
    const int pitch = (L.cx + 2) * FPAD, hp = (L.cx + 2) * FHALF;
    const float* __restrict__ Fr = Ffr + L.feat_off + (long long)r * pitch + 4 * g4;
    const int fg = min(FGROUP, nf - grp * FGROUP);
    const int f0 = grp * FGROUP + g4, f1 = f0 + 4;
    const bool f0ok = f0 < nf, f1ok = XTRA && g4 == 0;
    const float b0 = f0ok ? bias[f0] : 0.f, b1 = f1ok ? bias[f1] : 0.f;
    float* __restrict__ D = Dfr ? Dfr + L.sc_off : nullptr;
    unsigned long long* __restrict__ PK = PKfr ? PKfr + L.pos_off + (long long)r * L.cols : nullptr;
    const int t_first = max(t_begin - 1, 0);
    float carry0 = 0.f, carry1 = 0.f;
    for (int t = t_first; t < t_end; ++t) {
        const float* __restrict__ a = Fr + min(16 * t + j, L.cx + 1) * FHALF;
        // the K chunks (channels 0..15, 16..31) one after the other, so that
        // only one chunk's ten operands are live; the five filters'
        // accumulators carry over (a filter past the group's end has zero
        // factors and is skipped)
        floatx4 acc[FGROUP];
#pragma unroll
        for (int f = 0; f < FGROUP; ++f) acc[f] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            float4 av[WIN];
#pragma unroll
            for (int dr = 0; dr < WIN; ++dr) av[dr] = *reinterpret_cast<const float4*>(a + dr * pitch + kc * hp);
#pragma unroll
            for (int f = 0; f < FGROUP; ++f) {
                if (f >= fg) break;
#pragma unroll
                for (int i = 0; i < RANK; ++i) {
                    const float* __restrict__ cw = sm.colw + ((f * RANK + i) * WIN) * FPAD + 16 * kc + 4 * g4;
                    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int dr = 0; dr < WIN; ++dr) {
                        const float4 w = *reinterpret_cast<const float4*>(cw + dr * FPAD);
                        g.x = fmaf(w.x, av[dr].x, g.x);
                        g.y = fmaf(w.y, av[dr].y, g.y);
                        g.z = fmaf(w.z, av[dr].z, g.z);
                        g.w = fmaf(w.w, av[dr].w, g.w);
                    }
                    const float4 bq = sm.B[((f * RANK + i) * 2 + kc) * 64 + lane];
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(g.x, bq.x, acc[f], 0, 0, 0);
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(g.y, bq.y, acc[f], 0, 0, 0);
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(g.z, bq.z, acc[f], 0, 0, 0);
                    acc[f] = __builtin_amdgcn_mfma_f32_16x16x4f32(g.w, bq.w, acc[f], 0, 0, 0);
                }
            }
        }
        wave_lds_order();
#pragma unroll
        for (int f = 0; f < FGROUP; ++f)
            if (f < fg && j < WIN)
                *reinterpret_cast<float4*>(ring + (WIN * f + j) * SC_RSTR + 4 * g4) =
                    make_float4(acc[f][0], acc[f][1], acc[f][2], acc[f][3]);
        wave_lds_order();
        tile_windows<XTRA>(L, k, r, t, t_begin, ring, carry0, carry1, g4, j, f0, f1, f0ok, f1ok, b0, b1, thresh, D,
                           PK, atomic_key, c_lo, c_hi);
    }
}

// One separable scoring item; as score_item.
template <int ROWS, int RANK>
__device__ __forceinline__ void score_item_sep(const LevelTable& T, int frame, int grp, int item,
                                               const SepSmemT<ROWS, RANK>& sm, float* __restrict__ ring,
                                               const float* __restrict__ feat, int nf, const float* __restrict__ bias,
                                               float thresh, float* __restrict__ dense,
                                               unsigned long long* __restrict__ poskey, int atomic_key, int tid,
                                               int part = -1, const hog_region* __restrict__ regions = nullptr,
                                               int parts = 2) {
    const int q = item * ROWS + __builtin_amdgcn_readfirstlane(tid >> 6);
    if (q >= T.rows_total) return;
    const int k = HOG_FIND_LEVEL(T, q, row_off);
    const DevLevel& L = T.L[k];
    const int r = q - L.row_off;
    const float* Ffr = feat + (long long)frame * T.feat_frame;
    float* Dfr = dense ? dense + (long long)frame * T.dense_frame : nullptr;
    unsigned long long* PKfr = poskey ? poskey + (long long)frame * T.pos_frame : nullptr;
    const int fg = min(FGROUP, nf - grp * FGROUP);
    const int lane = tid & 63;
    const int ntiles = (L.cx + 15) >> 4;
    int tb = 0, te = ntiles;
    if (part >= 0) {
        row_part_tiles(ntiles, part, parts, tb, te);
        if (tb >= te) return;
    }
    int c_lo, c_hi;
    region_row(T, L, k, r, regions ? regions + frame : nullptr, PKfr, atomic_key, lane, tb, te, c_lo, c_hi);
    if (tb >= te) return;
    if (fg == FGROUP)
        score_row_sep<RANK, true, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key, lane,
                                        tb, te, c_lo, c_hi);
    else
        score_row_sep<RANK, false, ROWS>(L, k, r, Ffr, sm, ring, grp, nf, bias, thresh, Dfr, PKfr, atomic_key,
                                         lane, tb, te, c_lo, c_hi);
}

}  // namespace hog
