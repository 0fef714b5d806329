// Per-call set-up: pyramid geometry tables, filter repacking for the
// matrix-core scorer, and clearing of the candidate-key map.
#include "hog_device.h"

namespace hog {

// Segment 0 (blockIdx.y == 0): resampling taps of every level (rows, then
// columns; Sec. IV-A pyramid) and the frame-pixel edges of every window row
// and column (used for boxes and NMS).
// Segment 1: filters [nf][10][10][31] -> MFMA B operands.  The B matrix of
// filter group g has K = (window row dr, 384 values j of three adjacent
// window columns' 12 cells x 32 channels) and N = (filter f in the group,
// window shift d in 0..2); B[dr][j][f,d] = W_f[dr][j/32 - d][j%32] where
// that cell exists and the channel is < 31, else 0.  Lane (g4, n) of the
// 16x16x4 MFMA supplies 4 consecutive K values per 16-wide chunk.
// Segment 2: zero the per-position candidate keys (when several filter
// groups merge their keys with atomic max).
__global__ __launch_bounds__(256) void hog_setup_kernel(
    LevelTable T, int4* __restrict__ taps, int2* __restrict__ boxes,
    const float* __restrict__ W, int nf, float4* __restrict__ bpack,
    unsigned long long* __restrict__ keys, long long nkeys) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.y == 0) {
        if (e < T.taps_total) {
            for (int k = 0; k < T.n; ++k) {
                const DevLevel& L = T.L[k];
                if (e >= L.tap_y && e < L.tap_y + L.h) {
                    taps[e] = axis_tap((int)(e - L.tap_y), T.h, L.sig);
                    return;
                }
                if (e >= L.tap_x && e < L.tap_x + L.w) {
                    taps[e] = axis_tap((int)(e - L.tap_x), T.w, L.sig);
                    return;
                }
            }
        } else if (e < (long long)T.taps_total + T.boxes_total) {
            const long long b = e - T.taps_total;
            for (int k = 0; k < T.n; ++k) {
                const DevLevel& L = T.L[k];
                long long i = -1;
                if (b >= L.box_r && b < L.box_r + L.rows) i = b - L.box_r;
                if (b >= L.box_c && b < L.box_c + L.cols) i = b - L.box_c;
                if (i >= 0) {
                    boxes[b] = make_int2(box_edge(8 * i, L.sig), box_edge(8 * i + 80, L.sig));
                    return;
                }
            }
        }
    } else if (blockIdx.y == 1) {
        const int ngroups = (nf + FGROUP - 1) / FGROUP;
        if (e >= (long long)ngroups * BPACK_PER_GROUP) return;
        const int grp = (int)(e / BPACK_PER_GROUP);
        const int rem = (int)(e % BPACK_PER_GROUP);
        const int dr = rem / (KK * 64);
        const int kk = (rem / 64) % KK;
        const int lane = rem % 64;
        const int g4 = lane >> 4, n = lane & 15;
        const int d = n % SHIFT, f = grp * FGROUP + n / SHIFT;
        float v[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = 16 * kk + 4 * g4 + s - FPAD * d;
            const int dc = j / FPAD, ch = j % FPAD;
            const bool ok = n < FGROUP * SHIFT && f < nf && j >= 0 && dc < WIN && ch < NFEAT;
            v[s] = ok ? W[((f * WIN + dr) * WIN + dc) * NFEAT + ch] : 0.f;
        }
        bpack[e] = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        if (e < nkeys) keys[e] = 0ull;
    }
}

hipError_t launch_setup(const LevelTable& T, int4* taps, int2* boxes, const float* filters, int nf,
                        float4* bpack, unsigned long long* poskey_zero, long long poskey_count,
                        hipStream_t s) {
    const long long geo = (long long)T.taps_total + T.boxes_total;
    const long long pk = filters ? (long long)((nf + FGROUP - 1) / FGROUP) * BPACK_PER_GROUP : 0;
    const long long zk = poskey_zero ? poskey_count : 0;
    long long m = geo > pk ? geo : pk;
    if (zk > m) m = zk;
    const int segs = poskey_zero ? 3 : (filters ? 2 : 1);
    dim3 grid((unsigned)((m + 255) / 256), segs);
    hipLaunchKernelGGL(hog_setup_kernel, grid, dim3(256), 0, s, T, taps, boxes, filters, nf, bpack,
                       poskey_zero, zk);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void hog_fill_kernel(int* __restrict__ p, int n, int v) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// A plain fill kernel instead of hipMemsetAsync, so that the sequence can
// be captured into a graph.
hipError_t launch_fill(int* p, int n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hog_fill_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace hog
