// Non-maximum suppression on the GPU (Sec. IV-A: detections of one face
// are reduced to the best-scoring one; the paper runs this step on the
// CPU, Sec. V-A).
#include "hog_device.h"

namespace hog {

enum : int { UNDECIDED = 0, KEPT = 1, DROPPED = 2 };

__device__ __forceinline__ int ld_state(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_state(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Box {
    int x0, y0, x1, y1;
};

__device__ __forceinline__ Box window_box(const DevLevel& L, const int2* boxes, int r, int c) {
    const int2 ry = boxes[L.box_r + r], cx = boxes[L.box_c + c];
    return Box{cx.x, ry.x, cx.y, ry.y};
}

// Decide one candidate given the states of the better-ranked candidates it
// overlaps with IoU > iou: DROPPED if one of them is kept, KEPT if all of
// them are dropped, else UNDECIDED.  The neighbours are enumerated per
// level from a necessary condition on the horizontal (vertical) overlap:
// IoU > 1/2 needs 3 I > A + A', and I <= ov_x * min(h, h'), so
// ov_x > (A + A'_min) / (3 min(h, h'_max)); the exact test is made on
// integer areas.
__device__ int decide(const LevelTable& T, const unsigned long long* keys, const int* st, const int2* boxes,
                      unsigned long long kx, long long inum, long long iden) {
    const unsigned int pk = ~(unsigned int)(kx & 0xffffffffu);
    const int k = (pk >> 22) & 31, r = (pk >> 11) & 2047, c = pk & 2047;
    const DevLevel& L = T.L[k];
    const Box X = window_box(L, boxes, r, c);
    const long long wX = X.x1 - X.x0, hX = X.y1 - X.y0;
    const long long AX = wX * hX;
    bool blocked = false;
    for (int k2 = L.nms_klo; k2 <= L.nms_khi; ++k2) {
        const DevLevel& M = T.L[k2];
        const double inv8 = 0.125 * 1099511627776.0 / (double)M.sig;   // level px per frame px / 8
        const double amin = (double)M.wmin * M.hmin;
        const double tx = (AX + amin) / (3.0 * (double)min(hX, (long long)M.hmax)) * (1.0 - 1e-9);
        const double ty = (AX + amin) / (3.0 * (double)min(wX, (long long)M.wmax)) * (1.0 - 1e-9);
        // x0' in (X.x0 + tx - wmax', X.x1 - tx), |x0' - 8c' sig'| <= 1/2
        int c_lo = (int)floor((X.x0 + tx - M.wmax - 0.5) * inv8) - 1;
        int c_hi = (int)ceil((X.x1 - tx + 0.5) * inv8) + 1;
        int r_lo = (int)floor((X.y0 + ty - M.hmax - 0.5) * inv8) - 1;
        int r_hi = (int)ceil((X.y1 - ty + 0.5) * inv8) + 1;
        c_lo = max(c_lo, 0);
        r_lo = max(r_lo, 0);
        c_hi = min(c_hi, M.cols - 1);
        r_hi = min(r_hi, M.rows - 1);
        for (int r2 = r_lo; r2 <= r_hi; ++r2) {
            const int2 ry = boxes[M.box_r + r2];
            const long long ih = (long long)min(X.y1, ry.y) - max(X.y0, ry.x);
            if (ih <= 0) continue;
            const long long base = M.pos_off + (long long)r2 * M.cols;
            for (int c2 = c_lo; c2 <= c_hi; ++c2) {
                const unsigned long long ky = keys[base + c2];
                if (ky <= kx) continue;                 // worse rank, or not a candidate
                const int sy = ld_state(st + base + c2);
                if (sy == DROPPED) continue;
                const int2 cxy = boxes[M.box_c + c2];
                const long long iw = (long long)min(X.x1, cxy.y) - max(X.x0, cxy.x);
                if (iw <= 0) continue;
                const long long I = iw * ih;
                const long long U = AX + (long long)(cxy.y - cxy.x) * (ry.y - ry.x) - I;
                if (I * iden > inum * U) {
                    if (sy == KEPT) return DROPPED;
                    blocked = true;
                }
            }
        }
    }
    return blocked ? UNDECIDED : KEPT;
}

// One workgroup per frame.  Every window position holds its best candidate
// key over the filters (a window's other filters have the same box and a
// lower rank, so they are suppressed by it or by whatever suppresses it).
// Greedy NMS in rank order keeps a candidate iff no kept, better-ranked
// candidate overlaps it with IoU > iou.  Here every undecided candidate is
// decided as soon as all its better-ranked overlapping candidates are; the
// best undecided candidate always decides, so the rounds end, with the
// same result as the sequential greedy pass.  The kept keys are then
// sorted (the top min(cap, 4096) when there are more) and written out.
__global__ __launch_bounds__(NMS_THREADS) void hog_nms_kernel(
    LevelTable T, const unsigned long long* __restrict__ poskey, int* __restrict__ state,
    const int2* __restrict__ boxes, long long inum, long long iden, hog_det* __restrict__ dets, int cap,
    int* __restrict__ n_dets) {
    __shared__ unsigned long long sk[SORT_CAP];
    __shared__ unsigned int hist[256];
    __shared__ int s_count;
    __shared__ unsigned long long s_prefix, s_mask;
    __shared__ int s_remaining;

    const int tid = threadIdx.x;
    const int frame = blockIdx.x;
    const int P = T.pos_frame;
    const unsigned long long* keys = poskey + (long long)frame * P;
    int* st = state + (long long)frame * P;

    for (int p = tid; p < P; p += NMS_THREADS) st_state(st + p, keys[p] ? UNDECIDED : DROPPED);
    __syncthreads();

    for (int round = 0; round <= P; ++round) {
        int changed = 0, left = 0;
        for (int p = tid; p < P; p += NMS_THREADS) {
            if (ld_state(st + p) != UNDECIDED) continue;
            const int v = decide(T, keys, st, boxes, keys[p], inum, iden);
            if (v != UNDECIDED) {
                st_state(st + p, v);
                changed = 1;
            } else {
                left = 1;
            }
        }
        if (!__syncthreads_or(left)) break;
        (void)changed;
    }

    // count the kept candidates
    if (tid == 0) s_count = 0;
    __syncthreads();
    int mine = 0;
    for (int p = tid; p < P; p += NMS_THREADS) mine += ld_state(st + p) == KEPT;
    if (mine) atomicAdd(&s_count, mine);
    __syncthreads();
    const int nkept = s_count;
    const int want = min(nkept, min(cap, SORT_CAP));

    // threshold key: the want-th largest kept key (keys are unique)
    unsigned long long thr = 0ull;
    if (nkept > SORT_CAP) {
        if (tid == 0) { s_prefix = 0ull; s_mask = 0ull; s_remaining = want; }
        __syncthreads();
        for (int shift = 56; shift >= 0; shift -= 8) {
            for (int b = tid; b < 256; b += NMS_THREADS) hist[b] = 0u;
            __syncthreads();
            const unsigned long long pre = s_prefix, msk = s_mask;
            for (int p = tid; p < P; p += NMS_THREADS) {
                if (ld_state(st + p) != KEPT) continue;
                const unsigned long long kk = keys[p];
                if ((kk & msk) == pre) atomicAdd(&hist[(kk >> shift) & 255], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                int rem = s_remaining, cum = 0, dsel = 0;
                for (int dgt = 255; dgt >= 0; --dgt) {
                    if (cum + (int)hist[dgt] >= rem) { dsel = dgt; break; }
                    cum += hist[dgt];
                }
                s_remaining = rem - cum;
                s_prefix = pre | ((unsigned long long)dsel << shift);
                s_mask = msk | (255ull << shift);
            }
            __syncthreads();
        }
        thr = s_prefix;
    }

    // gather kept keys >= thr into LDS, pad with zeros to a power of two
    if (tid == 0) s_count = 0;
    __syncthreads();
    for (int p = tid; p < P; p += NMS_THREADS) {
        if (ld_state(st + p) != KEPT) continue;
        const unsigned long long kk = keys[p];
        if (kk < thr) continue;
        const int slot = atomicAdd(&s_count, 1);
        if (slot < SORT_CAP) sk[slot] = kk;
    }
    __syncthreads();
    const int ng = min(s_count, SORT_CAP);
    int npow = 1;
    while (npow < ng) npow <<= 1;
    for (int e = ng + tid; e < npow; e += NMS_THREADS) sk[e] = 0ull;
    __syncthreads();

    // bitonic sort, descending
    for (int size = 2; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = tid; e < npow; e += NMS_THREADS) {
                const int partner = e ^ stride;
                if (partner > e) {
                    const bool desc = (e & size) == 0;
                    const unsigned long long a = sk[e], b = sk[partner];
                    if ((a < b) == desc) { sk[e] = b; sk[partner] = a; }
                }
            }
            __syncthreads();
        }
    }

    const int nout = min(ng, cap);
    for (int e = tid; e < nout; e += NMS_THREADS) {
        const unsigned long long kk = sk[e];
        const unsigned int pk = ~(unsigned int)(kk & 0xffffffffu);
        const int f = pk >> 27, k = (pk >> 22) & 31, r = (pk >> 11) & 2047, c = pk & 2047;
        const Box b = window_box(T.L[k], boxes, r, c);
        hog_det d;
        d.frame = frame; d.filter = f; d.level = k; d.row = r; d.col = c;
        d.x0 = b.x0; d.y0 = b.y0; d.x1 = b.x1; d.y1 = b.y1;
        d.score = score_from_order((unsigned int)(kk >> 32));
        dets[(long long)frame * cap + e] = d;
    }
    if (tid == 0) n_dets[frame] = nkept;
}

hipError_t launch_nms(const LevelTable& T, int n, const unsigned long long* poskey, int* state, const int2* boxes,
                      long long iou_num, long long iou_den, void* dets, int cap, int* n_dets, hipStream_t s) {
    hipLaunchKernelGGL(hog_nms_kernel, dim3(n), dim3(NMS_THREADS), 0, s, T, poskey, state, boxes, iou_num,
                       iou_den, (hog_det*)dets, cap, n_dets);
    return hipGetLastError();
}

}  // namespace hog
