// Pyramid resampling, gradients, orientation and cell histograms
// (Sec. IV-A: image pyramid, gradient computation, histogramisation;
// Sec. V-A: image-scaling and gradient-histogram kernels), fused into one
// kernel per tile of cells.
#include "stage_hist.h"

namespace hog {

// One workgroup per tile.  The items (frame, tile) are listed frame by
// frame, each frame's tiles level by level, and cut into 8 contiguous
// ranges, one per XCD: block b runs on XCD b mod 8 (blocks are dealt to
// the XCDs in turn), and takes item b / 8 of range b mod 8.  A frame's
// tiles, which read overlapping frame rows, thus share one L2 instead of
// every XCD fetching every frame.
__global__ __launch_bounds__(HIST_THREADS) void hog_hist_kernel(
    LevelTable T, int n, const uint8_t* __restrict__ frames, long long fstride, int pitch,
    const int4* __restrict__ taps, float* __restrict__ hist) {
    __shared__ HistSmem sm;
    const long long items = (long long)T.th_total * n;
    const int x = (int)(blockIdx.x & 7);
    const long long lo = items * x / 8, hi = items * (x + 1) / 8;
    const long long item = lo + (blockIdx.x >> 3);
    if (item >= hi) return;
    const int frame = (int)(item / T.th_total);
    hist_tile(T, frames, fstride, pitch, taps, hist, frame, (int)(item - (long long)frame * T.th_total),
              (int)threadIdx.x, sm);
}

hipError_t launch_hist(const LevelTable& T, const uint8_t* frames, long long fstride, int pitch, int n,
                       const int4* taps, float* hist, hipStream_t s) {
    const long long items = (long long)T.th_total * n;
    if (items <= 0) return hipSuccess;
    const long long per_xcd = (items + 7) / 8;
    if (per_xcd * 8 > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hog_hist_kernel, dim3((unsigned)(per_xcd * 8)), dim3(HIST_THREADS), 0, s, T, n, frames,
                       fstride, pitch, taps, hist);
    return hipGetLastError();
}

// Inspection: level pixel and orientation bin of every pixel of one level,
// computed per pixel with the same taps and decision as the kernel above.
__global__ __launch_bounds__(256) void hog_level_maps_kernel(
    LevelTable T, int level, const uint8_t* __restrict__ U, int pitch, const int4* __restrict__ taps,
    float* __restrict__ level_px, uint8_t* __restrict__ bins) {
    const DevLevel& L = T.L[level];
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)L.h * L.w) return;
    const int y = (int)(e / L.w), x = (int)(e % L.w);
    auto px = [&](int yy, int xx) -> int {
        const int4 a = taps[L.tap_y + yy], b = taps[L.tap_x + xx];
        const uint8_t* r0 = U + (long long)a.x * pitch;
        const uint8_t* r1 = U + (long long)a.y * pitch;
        const int top = (256 - b.z) * r0[b.x] + b.z * r0[b.y];
        const int bot = (256 - b.z) * r1[b.x] + b.z * r1[b.y];
        return (256 - a.z) * top + a.z * bot;
    };
    const int v = px(y, x);
    if (level_px) level_px[e] = (float)v * 0x1p-16f;
    if (bins) {
        int bn = 0;
        if (y >= 1 && y <= L.h - 2 && x >= 1 && x <= L.w - 2) {
            const int gx = px(y, x + 1) - px(y, x - 1);
            const int gy = px(y + 1, x) - px(y - 1, x);
            if (gx | gy) bn = orient_bin(gx, gy);
        }
        bins[e] = (uint8_t)bn;
    }
}

hipError_t launch_level_maps(const LevelTable& T, int level, const uint8_t* frame, int pitch,
                             const int4* taps, float* level_px, uint8_t* bins, hipStream_t s) {
    const long long n = (long long)T.L[level].h * T.L[level].w;
    hipLaunchKernelGGL(hog_level_maps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T,
                       level, frame, pitch, taps, level_px, bins);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void hog_orient_kernel(const int32_t* __restrict__ gx,
                                                          const int32_t* __restrict__ gy, long long n,
                                                          uint8_t* __restrict__ bins) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int a = gx[e], b = gy[e];
    bins[e] = (uint8_t)((a | b) ? orient_bin(a, b) : 0);
}

hipError_t launch_orient(const int32_t* gx, const int32_t* gy, long long n, uint8_t* bins, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hog_orient_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gx, gy, n,
                       bins);
    return hipGetLastError();
}

void orientation_table_host(double* c, double* s) {
    for (int o = 0; o < NORIENT; ++o) {
        c[o] = dir_cos(o);
        s[o] = dir_sin(o);
    }
}

}  // namespace hog
