// Pyramid resampling, gradients, orientation and cell histograms
// (Sec. IV-A: image pyramid, gradient computation, histogramisation;
// Sec. V-A: image-scaling and gradient-histogram kernels), fused into one
// kernel per tile of cells.
#include "stage_hist.h"
#include "stage_setup.h"

namespace hog {

// Whether tile `tile` of a frame holds a cell that a window inside the
// frame's search region reads: the window's 10x10 cells, or the ring of
// cells whose energies normalise them.  The histograms of a skipped tile
// are left as they were; only windows outside the region read them, and
// those are not candidates.
__device__ __forceinline__ bool hist_tile_needed(const LevelTable& T, int tile, const hog_region& g) {
    const int k = HOG_FIND_LEVEL(T, tile, th_off);
    const DevLevel& L = T.L[k];
    const RegionRange R = region_range(L, k + T.k_base, g);
    if (R.empty()) return false;
    const int t = tile - L.th_off;
    const int tiles_x = (L.cx + TCX - 1) / TCX;
    const int i0 = (t / tiles_x) * TCY, j0 = (t % tiles_x) * TCX;
    return i0 <= R.r_hi + WIN && i0 + TCY - 1 >= R.r_lo - 1 && j0 <= R.c_hi + WIN && j0 + TCX - 1 >= R.c_lo - 1;
}

// One workgroup per tile.  The items (frame, tile) are listed frame by
// frame, each frame's tiles level by level, and cut into 8 contiguous
// ranges, one per XCD: block b runs on XCD b mod 8 (blocks are dealt to
// the XCDs in turn), and takes item b / 8 of range b mod 8.  A frame's
// tiles, which read overlapping frame rows, thus share one L2 instead of
// every XCD fetching every frame.  Blocks from hist_blocks on do the
// call's set-up instead (setup.segs > 0), HIST_THREADS elements each.
__global__ __launch_bounds__(HIST_THREADS) void hog_hist_kernel(
    LevelTable T, int n, const uint8_t* __restrict__ frames, long long fstride, int pitch,
    float* __restrict__ hist, const hog_region* __restrict__ regions, const uint8_t* __restrict__ casc,
    int hist_blocks, SetupArgs setup) {
    __shared__ HistSmem sm;
    if ((int)blockIdx.x >= hist_blocks) {
        setup_flat(T, setup, (long long)(blockIdx.x - hist_blocks) * HIST_THREADS + threadIdx.x);
        return;
    }
    const long long items = (long long)T.th_total * n;
    const int x = (int)(blockIdx.x & 7);
    const long long lo = items * x / 8, hi = items * (x + 1) / 8;
    const long long item = lo + (blockIdx.x >> 3);
    if (item >= hi) return;
    const int frame = (int)(item / T.th_total);
    const int tile = (int)(item - (long long)frame * T.th_total);
    // the whole workgroup leaves together, before any barrier
    if (regions && !hist_tile_needed(T, tile, regions[frame])) return;
    hist_tile(T, frames, fstride, pitch, hist, frame, tile, (int)threadIdx.x, sm, casc);
}

hipError_t launch_hist(const LevelTable& T, const uint8_t* frames, long long fstride, int pitch, int n,
                       float* hist, const hog_region* regions, const uint8_t* casc, hipStream_t s,
                       const SetupArgs* setup) {
    const long long items = (long long)T.th_total * n;
    if (items <= 0 && !setup) return hipSuccess;
    const long long per_xcd = (items + 7) / 8;
    SetupArgs sa{};
    long long extra = 0;
    if (setup) {
        sa = *setup;
        extra = (sa.m * sa.segs + HIST_THREADS - 1) / HIST_THREADS;
    }
    if (per_xcd * 8 + extra > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hog_hist_kernel, dim3((unsigned)(per_xcd * 8 + extra)), dim3(HIST_THREADS), 0, s, T, n,
                       frames, fstride, pitch, hist, regions, casc, (int)(per_xcd * 8), sa);
    return hipGetLastError();
}

// One level of the recursive pyramid (Sec. V-A, image-scaling kernel:
// each scaled image is computed from the image one scale higher), one
// thread per output pixel of every frame.  A 5/6 step puts output pixel i
// at (12 i + 1) / 10 of the input (pixel centres aligned); the fractional
// part rounded to 1/256 is the bilinear weight.  With sig > 0 the pixel is
// sampled from the frame at that inverse scale instead (the 2x level 0).
// The exact integer sum of weight products and samples (value * 2^16) is
// rounded half up to a grey level.
__global__ __launch_bounds__(256) void hog_cascade_kernel(const uint8_t* __restrict__ frames, long long fstride,
                                                           int pitch, uint8_t* __restrict__ casc, long long casc_frame,
                                                           int h_out, int w_out, int dst_off, int h_in, int w_in,
                                                           int src_off, long long sig) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)h_out * w_out) return;
    const int frame = blockIdx.y;
    const int y = (int)(e / w_out), x = (int)(e - (long long)y * w_out);
    const uint8_t* __restrict__ U;
    int sp;
    int4 ty, tx;
    if (sig > 0) {
        U = frames + (long long)frame * fstride;
        sp = pitch;
        ty = axis_tap(y, h_in, sig);
        tx = axis_tap(x, w_in, sig);
    } else {
        U = src_off < 0 ? frames + (long long)frame * fstride : casc + (long long)frame * casc_frame + src_off;
        sp = src_off < 0 ? pitch : w_in;
        const int ny = 12 * y + 1, nx = 12 * x + 1;
        ty = make_int4(min(ny / 10, h_in - 1), min(ny / 10 + 1, h_in - 1), (256 * (ny % 10) + 5) / 10, 0);
        tx = make_int4(min(nx / 10, w_in - 1), min(nx / 10 + 1, w_in - 1), (256 * (nx % 10) + 5) / 10, 0);
    }
    const uint8_t* r0 = U + (long long)ty.x * sp;
    const uint8_t* r1 = U + (long long)ty.y * sp;
    const unsigned top = (256u - tx.z) * r0[tx.x] + tx.z * r0[tx.y];
    const unsigned bot = (256u - tx.z) * r1[tx.x] + tx.z * r1[tx.y];
    const unsigned v = (256u - ty.z) * top + ty.z * bot;
    casc[(long long)frame * casc_frame + dst_off + e] = (uint8_t)((v + 32768u) >> 16);
}

hipError_t launch_cascade(const uint8_t* frames, long long fstride, int pitch, int n, uint8_t* casc,
                          long long casc_frame, int h_out, int w_out, int dst_off, int h_in, int w_in, int src_off,
                          long long sig, hipStream_t s) {
    const long long px = (long long)h_out * w_out;
    if (px <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hog_cascade_kernel, dim3((unsigned)((px + 255) / 256), (unsigned)n), dim3(256), 0, s, frames,
                       fstride, pitch, casc, casc_frame, h_out, w_out, dst_off, h_in, w_in, src_off, sig);
    return hipGetLastError();
}

// Inspection: level pixel and orientation bin of every pixel of one level,
// computed per pixel with the same taps and decision as the kernel above.
__global__ __launch_bounds__(256) void hog_level_maps_kernel(
    LevelTable T, int level, const uint8_t* __restrict__ frame, int frame_pitch, const int4* __restrict__ taps,
    float* __restrict__ level_px, uint8_t* __restrict__ bins, const uint8_t* __restrict__ casc) {
    const DevLevel& L = T.L[level];
    const uint8_t* __restrict__ U = L.src ? casc + L.src_off : frame;
    const int pitch = L.src ? L.w : frame_pitch;
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
                             const int4* taps, float* level_px, uint8_t* bins, const uint8_t* casc, hipStream_t s) {
    const long long n = (long long)T.L[level].h * T.L[level].w;
    hipLaunchKernelGGL(hog_level_maps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T,
                       level, frame, pitch, taps, level_px, bins, casc);
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
