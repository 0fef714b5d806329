// Device stage: block normalisation and the 31-d cell features (Sec.
// IV-A normalisation and feature computation; Sec. V-A feature kernel).
// Used by the per-stage feature kernel and by the fused persistent kernel.
#pragma once
#include "hog_device.h"

namespace hog {

// One thread per cell of the padded feature grid [cy][cx + 2] of a level.
// Each cell is normalised by the four 2x2-cell blocks that contain it,
// n_k = (B_k + 1e-4)^(-1/2) with B_k the summed energy of the block (zero
// outside the grid).  With T(v) = min(v, 0.2):
//   F[b]      = 1/2 sum_k T(h_b n_k)               (18 signed)
//   F[18 + o] = 1/2 sum_k T((h_o + h_{o+9}) n_k)   (9 unsigned)
//   F[27 + k] = 1/sqrt(18) sum_b T(h_b n_k)        (4 block energies)
// The padded layout stores 32 floats per cell (channel 31 = 0) and two
// zero cells after each row, which the scorer reads past the last column,
// in two half-planes per row (channels 0..15 of the row's cells, then
// 16..31).
// `packed`, when non-null, also receives [cy][cx][31] at the level's
// packed offset (single frame).  F16: the cell's 128 bytes hold instead
// the split fp16 operands of the scorer (HOG_ARITH_F16X3): the 32 high
// parts fp16(F[c]), then the 32 low parts fp16((F[c] - hi) 2^11), both
// rounded to nearest (zero cells are zero either way).
// Block `blk` (of FEAT_THREADS cells, within one level) of a frame; thread
// `tid` of the block.  With `stage` (LDS, 64 x 8 uint4 per wave) the
// wave's 64 cells, which are consecutive in the map, are exchanged through
// LDS so that each store writes 1 KB of consecutive bytes (a cell's own
// 128 bytes at a 128-byte lane stride would touch 64 lines per store).
template <bool F16 = false>
__device__ __forceinline__ void feat_cell(const LevelTable& T, const float* __restrict__ hist,
                                          float* __restrict__ feat, float* __restrict__ packed, int frame, int blk,
                                          int tid, uint4* __restrict__ stage = nullptr) {
    const int k = HOG_FIND_LEVEL(T, blk, tf_off);
    const DevLevel& L = T.L[k];
    const int pw = L.cx + 2;
    const int ncell = L.cy * pw;
    const int idx = (blk - L.tf_off) * FEAT_THREADS + tid;
    const int i = idx / pw, j = idx - i * pw;
    float* const fmap = feat + (long long)frame * T.feat_frame + L.feat_off;
    // the cell's 128 bytes; zero for the padding cells after each row
    uint4 q4[FPAD / 4];
#pragma unroll
    for (int q = 0; q < FPAD / 4; ++q) q4[q] = make_uint4(0u, 0u, 0u, 0u);
    if (idx < ncell && j < L.cx) {
        // part-major records (plane q holds part q of every cell): the
        // lanes of a wave read consecutive float4s of each plane
        const long long ncell = (long long)L.cy * L.cx;
        const float4* H4 = reinterpret_cast<const float4*>(hist + ((long long)frame * T.hist_frame + L.hist_off) * HSTRIDE);
        const float4* hc = H4 + (long long)i * L.cx + j;
        float h[20];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const float4 v = hc[q * ncell];
            h[4 * q] = v.x; h[4 * q + 1] = v.y; h[4 * q + 2] = v.z; h[4 * q + 3] = v.w;
        }
        // the energy is float 2 of part 4 (bins 16, 17, energy, 0)
        const float* E4 = reinterpret_cast<const float*>(H4 + 4 * ncell) + 2;
        auto E = [&](int y, int x) -> float {
            return (y >= 0 && y < L.cy && x >= 0 && x < L.cx) ? E4[((long long)y * L.cx + x) * 4] : 0.f;
        };
        const float e0 = h[NBINS];
        const float eu = E(i - 1, j), ed = E(i + 1, j), el = E(i, j - 1), er = E(i, j + 1);
        const float eul = E(i - 1, j - 1), eur = E(i - 1, j + 1), edl = E(i + 1, j - 1), edr = E(i + 1, j + 1);
        float n[4];
        n[0] = 1.0f / sqrtf(e0 + eu + el + eul + 1e-4f);   // block (-1, -1)
        n[1] = 1.0f / sqrtf(e0 + eu + er + eur + 1e-4f);   // block (-1, +1)
        n[2] = 1.0f / sqrtf(e0 + ed + el + edl + 1e-4f);   // block (+1, -1)
        n[3] = 1.0f / sqrtf(e0 + ed + er + edr + 1e-4f);   // block (+1, +1)
        float F[FPAD];
#pragma unroll
        for (int c = 0; c < FPAD; ++c) F[c] = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float tsum = 0.f;
#pragma unroll
            for (int b = 0; b < NBINS; ++b) {
                const float tv = fminf(h[b] * n[q], 0.2f);
                F[b] += 0.5f * tv;
                tsum += tv;
            }
#pragma unroll
            for (int o = 0; o < NORIENT; ++o) F[NBINS + o] += 0.5f * fminf((h[o] + h[o + NORIENT]) * n[q], 0.2f);
            F[27 + q] = 0.23570226039551584f * tsum;   // 1/sqrt(18)
        }
        if (F16) {
            _Float16 hl[2 * FPAD];
#pragma unroll
            for (int c = 0; c < FPAD; ++c) {
                // both parts from the stored FP32 feature: the empty asm keeps
                // the compiler from forming the high part with a mixed-precision
                // FMA from the unrounded last sum
                float f = F[c];
                asm volatile("" : "+v"(f));
                const _Float16 hi = (_Float16)f;
                hl[c] = hi;
                hl[FPAD + c] = (_Float16)((f - (float)hi) * 2048.f);
            }
            __builtin_memcpy(q4, hl, sizeof q4);
        } else {
            __builtin_memcpy(q4, F, sizeof q4);
        }
        if (packed) {
            float* p = packed + L.pk_off + ((long long)i * L.cx + j) * NFEAT;
#pragma unroll
            for (int c = 0; c < NFEAT; ++c) p[c] = F[c];
        }
    }
    // 16-byte part q of cell (i, j): half-plane q / 4 of row i
    auto part_at = [&](int ci, int cj, int q) {
        return reinterpret_cast<uint4*>(fmap + (long long)ci * pw * FPAD + (q >> 2) * (pw * FHALF) + cj * FHALF) +
               (q & 3);
    };
    if (stage) {
        const int lane = tid & 63;
        const int base = idx - lane;   // the wave's first cell
        uint4* __restrict__ w = stage + (tid >> 6) * (64 * FPAD / 4);
        // 16-byte slots of a cell rotated by the cell's low bits: the eight
        // lanes of one store phase hit different banks
#pragma unroll
        for (int q = 0; q < FPAD / 4; ++q) w[lane * 8 + (q ^ (lane & 7))] = q4[q];
        wave_lds_order();
        // store r: half-plane r / 4, cells 16 (r % 4) .. + 15 of the wave, four
        // lanes per cell, so that the lanes write consecutive bytes of a row
#pragma unroll
        for (int r = 0; r < FPAD / 4; ++r) {
            const int cell = 16 * (r & 3) + (lane >> 2), part = 4 * (r >> 2) + (lane & 3);
            const uint4 v = w[cell * 8 + (part ^ (cell & 7))];
            const int ci = base + cell;
            if (ci < ncell) {
                const int ri = ci / pw;
                *part_at(ri, ci - ri * pw, part) = v;
            }
        }
    } else if (idx < ncell) {
#pragma unroll
        for (int q = 0; q < FPAD / 4; ++q) *part_at(i, j, q) = q4[q];
    }
}

}  // namespace hog
