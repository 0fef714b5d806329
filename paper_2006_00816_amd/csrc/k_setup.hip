// Per-call set-up: pyramid geometry tables, filter repacking for the
// matrix-core scorer, and clearing of the candidate-key map.
#include "stage_setup.h"

namespace hog {

__global__ __launch_bounds__(256) void hog_setup_kernel(LevelTable T, SetupArgs a) {
    setup_element(T, a, (int)blockIdx.y, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

SetupArgs setup_args(const LevelTable& T, int4* taps, int2* boxes, const float* filters, int nf, float4* bpack,
                     unsigned long long* poskey_zero, long long poskey_count, unsigned* sync_zero, int sync_count,
                     bool f16x3) {
    SetupArgs a;
    a.taps = taps;
    a.boxes = boxes;
    a.W = filters;
    a.nf = nf;
    a.bpack = bpack;
    a.keys = poskey_zero;
    a.nkeys = poskey_zero ? poskey_count : 0;
    a.sync = sync_zero;
    a.nsync = sync_zero ? sync_count : 0;
    a.f16x3 = f16x3 ? 1 : 0;
    const long long geo = (long long)T.taps_total + T.boxes_total;
    const long long pk =
        filters ? (long long)((nf + FGROUP - 1) / FGROUP) * (f16x3 ? B16_PER_GROUP : BPACK_PER_GROUP) : 0;
    long long m = geo > pk ? geo : pk;
    if (a.nkeys > m) m = a.nkeys;
    if (a.nsync > m) m = a.nsync;
    a.m = m > 0 ? m : 1;
    a.segs = (a.nkeys || a.nsync) ? 3 : (filters ? 2 : 1);
    return a;
}

hipError_t launch_setup(const LevelTable& T, int4* taps, int2* boxes, const float* filters, int nf,
                        float4* bpack, unsigned long long* poskey_zero, long long poskey_count, unsigned* sync_zero,
                        int sync_count, hipStream_t s, bool f16x3) {
    const SetupArgs a =
        setup_args(T, taps, boxes, filters, nf, bpack, poskey_zero, poskey_count, sync_zero, sync_count, f16x3);
    dim3 grid((unsigned)((a.m + 255) / 256), a.segs);
    hipLaunchKernelGGL(hog_setup_kernel, grid, dim3(256), 0, s, T, a);
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
