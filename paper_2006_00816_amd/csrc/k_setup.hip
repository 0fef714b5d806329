// Per-call set-up: pyramid geometry tables, filter repacking for the
// matrix-core scorer, and clearing of the candidate-key map.
#include "hog_device.h"

namespace hog {

// Segment 0 (blockIdx.y == 0): resampling taps of every level (rows, then
// columns; Sec. IV-A pyramid) and the frame-pixel edges of every window row
// and column (used for boxes and NMS).
// Segment 1: filters [nf][10][10][31] -> scorer operands, per group of 5
// filters.  Column n = 10 f + dc (filter f of the group, window column dc)
// and K index k = 32 dr + ch (window row dr, channel ch; ch = 31 is zero):
//  - matrix-core part, columns 0..47: entry [kc][nt][lane] holds the four
//    K values 16 kc + 4 (lane / 16) + s, s = 0..3, of column
//    16 nt + lane % 16, for four consecutive MFMAs;
//  - vector-ALU part, columns 48 and 49 (f = 4, dc = 8, 9): entry
//    [kc][g][col] holds the K values 16 kc + 4 g + s of that column.
// Segment 2: zero the per-position candidate keys (when several filter
// groups merge their keys with atomic max) and the counters of the fused
// persistent kernel.
__global__ __launch_bounds__(256) void hog_setup_kernel(
    LevelTable T, int4* __restrict__ taps, int2* __restrict__ boxes,
    const float* __restrict__ W, int nf, float4* __restrict__ bpack,
    unsigned long long* __restrict__ keys, long long nkeys, unsigned* __restrict__ sync, int nsync, int f16x3) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.y == 0) {
        if (e < T.taps_total) {
            for (int k = 0; k < T.n; ++k) {
                const DevLevel& L = T.L[k];
                // a level image of the recursive pyramid is read as is
                if (e >= L.tap_y && e < L.tap_y + L.h) {
                    const int i = (int)(e - L.tap_y);
                    taps[e] = level_tap(L, i, L.h, T.h);
                    return;
                }
                if (e >= L.tap_x && e < L.tap_x + L.w) {
                    const int i = (int)(e - L.tap_x);
                    taps[e] = level_tap(L, i, L.w, T.w);
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
    } else if (blockIdx.y == 1 && f16x3) {
        // split fp16 B operands: entry ((dr B16_NT + nt) 2 + part) 64 + lane
        // of group grp holds the hi (part 0) or lo (part 1) halves of the
        // weights of channels 8 (lane / 16) + i, column 16 nt + lane % 16
        const int ngroups = (nf + FGROUP - 1) / FGROUP;
        if (!W || e >= (long long)ngroups * B16_PER_GROUP) return;
        const int grp = (int)(e / B16_PER_GROUP);
        const int rem = (int)(e % B16_PER_GROUP);
        const int lane = rem & 63, part = (rem >> 6) & 1, nt = (rem >> 7) % B16_NT, dr = rem / (B16_NT * 128);
        const int n = 16 * nt + (lane & 15);
        const int f = grp * FGROUP + n / WIN, dc = n % WIN;
        _Float16 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int ch = 8 * (lane >> 4) + i;
            const bool ok = n < FGROUP * WIN && f < nf && ch < NFEAT;
            const float w = ok ? W[((f * WIN + dr) * WIN + dc) * NFEAT + ch] : 0.f;
            const _Float16 h = (_Float16)w;
            v[i] = part ? (_Float16)((w - (float)h) * 2048.f) : h;
        }
        uint4 q;
        __builtin_memcpy(&q, v, sizeof q);
        reinterpret_cast<uint4*>(bpack)[e] = q;
    } else if (blockIdx.y == 1) {
        const int ngroups = (nf + FGROUP - 1) / FGROUP;
        if (!W || e >= (long long)ngroups * BPACK_PER_GROUP) return;
        const int grp = (int)(e / BPACK_PER_GROUP);
        const int rem = (int)(e % BPACK_PER_GROUP);
        int n, k0;
        if (rem < BPACK_MFMA) {
            const int kc = rem / (SC_NT * 64);
            const int nt = (rem / 64) % SC_NT;
            const int lane = rem % 64;
            n = 16 * nt + (lane & 15);
            k0 = 16 * kc + 4 * (lane >> 4);
        } else {
            const int x = rem - BPACK_MFMA;
            n = 48 + (x & 1);
            k0 = 16 * (x >> 3) + 4 * ((x >> 1) & 3);
        }
        const int f = grp * FGROUP + n / WIN, dc = n % WIN;
        float v[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + s;
            const int dr = k / FPAD, ch = k % FPAD;
            const bool ok = f < nf && ch < NFEAT;
            v[s] = ok ? W[((f * WIN + dr) * WIN + dc) * NFEAT + ch] : 0.f;
        }
        bpack[e] = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        if (e < nkeys) keys[e] = 0ull;
        if (e < nsync) sync[e] = 0u;
    }
}

hipError_t launch_setup(const LevelTable& T, int4* taps, int2* boxes, const float* filters, int nf,
                        float4* bpack, unsigned long long* poskey_zero, long long poskey_count, unsigned* sync_zero,
                        int sync_count, hipStream_t s, bool f16x3) {
    const long long geo = (long long)T.taps_total + T.boxes_total;
    const long long pk =
        filters ? (long long)((nf + FGROUP - 1) / FGROUP) * (f16x3 ? B16_PER_GROUP : BPACK_PER_GROUP) : 0;
    const long long zk = poskey_zero ? poskey_count : 0;
    const int zs = sync_zero ? sync_count : 0;
    long long m = geo > pk ? geo : pk;
    if (zk > m) m = zk;
    if (zs > m) m = zs;
    const int segs = (zk || zs) ? 3 : (filters ? 2 : 1);
    dim3 grid((unsigned)((m + 255) / 256), segs);
    hipLaunchKernelGGL(hog_setup_kernel, grid, dim3(256), 0, s, T, taps, boxes, filters, nf, bpack,
                       poskey_zero, zk, sync_zero, zs, f16x3 ? 1 : 0);
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

// Search region of the next frame of each stream from this frame's
// detections (Sec. VII: faces move little between consecutive frames, so
// the locations and scales searched can be limited): the best detection's
// box (the first, in rank order) grown by `margin` px on every side and
// clipped to the frame, with its level +- span (clipped at 0); the whole
// frame at every level where the frame has no valid detection.
__global__ __launch_bounds__(256) void hog_track_kernel(const hog_det* __restrict__ dets,
                                                         const int* __restrict__ n_dets, int n, int cap, int h, int w,
                                                         int margin, int span, hog_region* __restrict__ regions) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    hog_region g;
    if (n_dets[i] > 0) {
        const hog_det d = dets[(long long)i * cap];
        g.x0 = max(d.x0 - margin, 0);
        g.y0 = max(d.y0 - margin, 0);
        g.x1 = min(d.x1 + margin, w);
        g.y1 = min(d.y1 + margin, h);
        g.k_lo = max(d.level - span, 0);
        g.k_hi = d.level + span;
    } else {
        g.x0 = 0;
        g.y0 = 0;
        g.x1 = w;
        g.y1 = h;
        g.k_lo = 0;
        g.k_hi = HOG_ALL_LEVELS;
    }
    regions[i] = g;
}

hipError_t launch_track(const hog_det* dets, const int* n_dets, int n, int cap, int h, int w, int margin, int span,
                        hog_region* regions, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hog_track_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dets, n_dets, n, cap, h, w, margin,
                       span, regions);
    return hipGetLastError();
}

}  // namespace hog
