// Linear window scoring on the matrix cores (Sec. IV-A linear
// classification; Sec. V-A classifier and detection kernels).
#include "hog_device.h"

namespace hog {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// The score of filter f at window (r, c) is bias_f plus the 3100-term dot
// product of the filter with the window's 10x10x31 features.  Written as a
// matrix product on v_mfma_f32_16x16x4_f32:
//   M = 16 anchors (r, c = 3a): each anchor covers windows c, c+1, c+2,
//   N = 16 columns (filter f of a group of 5, shift d of 0..2; one unused),
//   K = 10 window rows x 384: the 12 cells c .. c+11 x 32 channels,
// with B[dr][j][(f, d)] = W_f[dr][j/32 - d][j%32] (zero outside the
// window), so that C[anchor][(f, d)] = S_f(r, c + d) - bias_f.  A lane
// reads 4 consecutive K values as one float4 of the padded feature row and
// feeds them to 4 consecutive MFMAs; B was packed to match (set-up kernel).
//
// Each wave scores 4 M-tiles (64 anchors).  Outputs: the dense score map
// (optional) and, per window position, the best candidate key over the
// group's filters (0 if no filter's score exceeds the threshold).
__global__ __launch_bounds__(SCORE_THREADS) void hog_score_kernel(
    LevelTable T, const float* __restrict__ feat, const float4* __restrict__ bpack,
    const float* __restrict__ bias, int nf, float thresh, float* __restrict__ dense,
    unsigned long long* __restrict__ poskey, int atomic_key) {
    const int frame = blockIdx.y;
    const int grp = blockIdx.z;
    const int k = HOG_FIND_LEVEL(T, (int)blockIdx.x, ts_off);
    const DevLevel& L = T.L[k];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nanch = L.rows * L.apr;
    const int a0 = ((blockIdx.x - L.ts_off) * (SCORE_THREADS / 64) + wave) * ANCHORS_PER_WAVE;
    if (a0 >= nanch) return;

    const int g4 = lane >> 4, m = lane & 15;
    const int pitch = (L.cx + 2) * FPAD;
    const float* __restrict__ F = feat + (long long)frame * T.feat_frame + L.feat_off;
    const float* ap[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int a = min(a0 + 16 * t + m, nanch - 1);
        const int r = a / L.apr, c = SHIFT * (a - (a / L.apr) * L.apr);
        ap[t] = F + (long long)r * pitch + c * FPAD + 4 * g4;
    }
    floatx4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float4* __restrict__ B = bpack + (long long)grp * BPACK_PER_GROUP + lane;

    for (int dr = 0; dr < WIN; ++dr) {
#pragma unroll 4
        for (int kk = 0; kk < KK; ++kk) {
            const float4 b = B[(dr * KK + kk) * 64];
            float4 av[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                av[t] = *reinterpret_cast<const float4*>(ap[t] + (long long)dr * pitch + 16 * kk);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].x, b.x, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].y, b.y, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].z, b.z, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t].w, b.w, acc[t], 0, 0, 0);
            }
        }
    }

    // Epilogue.  Lane (g4, n) holds C[4 g4 + i][n], i = 0..3.
    const int n = m;
    const int d = n % SHIFT;
    const int f = grp * FGROUP + n / SHIFT;
    const bool fok = n < FGROUP * SHIFT && f < nf;
    const float bf = fok ? bias[f] : 0.f;
    unsigned long long* __restrict__ PK = poskey ? poskey + (long long)frame * T.pos_frame + L.pos_off : nullptr;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int a = a0 + 16 * t + 4 * g4 + i;
            const int r = a / L.apr;
            const int c = SHIFT * (a - r * L.apr) + d;
            const bool ok = fok && a < nanch && c < L.cols;
            const float s = acc[t][i] + bf;
            if (dense && ok)
                dense[(long long)frame * T.dense_frame + L.sc_off + ((long long)f * L.rows + r) * L.cols + c] = s;
            unsigned long long key = 0ull;
            if (ok && s > thresh)
                key = ((unsigned long long)score_order(s) << 32) | (unsigned long long)(~pack_window(f, k, r, c));
            // best over the group's filters of the same window: lanes n, n+3, ..., n+12
#pragma unroll
            for (int sft = SHIFT; sft < FGROUP * SHIFT; sft += SHIFT) {
                const int src = min(n + sft, 15);
                const unsigned long long o = __shfl(key, (lane & 48) | src, 64);
                key = o > key ? o : key;
            }
            if (PK && n < SHIFT && a < nanch && c < L.cols) {
                unsigned long long* dst = PK + (long long)r * L.cols + c;
                if (atomic_key) {
                    if (key) atomicMax(dst, key);
                } else {
                    *dst = key;
                }
            }
        }
    }
}

hipError_t launch_score(const LevelTable& T, int n, const float* feat, const float4* bpack, const float* bias,
                        int nf, float thresh, float* dense, unsigned long long* poskey, bool atomic_key,
                        hipStream_t s) {
    const int groups = (nf + FGROUP - 1) / FGROUP;
    hipLaunchKernelGGL(hog_score_kernel, dim3(T.ts_total, n, groups), dim3(SCORE_THREADS), 0, s, T, feat,
                       bpack, bias, nf, thresh, dense, poskey, atomic_key ? 1 : 0);
    return hipGetLastError();
}

}  // namespace hog
