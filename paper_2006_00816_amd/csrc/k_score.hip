// Linear window scoring on the matrix cores (Sec. IV-A linear
// classification; Sec. V-A classifier and detection kernels), one launch
// over all frames, filter groups and levels.
#include "stage_score.h"

namespace hog {

// Work item = (frame, filter group, 16 window rows of the frame's list of
// rows).  Neighbouring rows read 9 of their 10 feature rows in common, so
// the items of a frame are placed on one XCD (one L2): the launch is 1-D,
// and block b runs item (b mod 8) * (blocks / 8) + b / 8.
__global__ __launch_bounds__(SCORE_THREADS) void hog_score_kernel(
    LevelTable T, int groups, int items, const float* __restrict__ feat, const float4* __restrict__ bpack,
    const float* __restrict__ bias, int nf, float thresh, float* __restrict__ dense,
    unsigned long long* __restrict__ poskey, int atomic_key) {
    __shared__ ScoreSmem sm;
    const int per = (int)(gridDim.x >> 3);
    const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (item >= items) return;
    const int it = item % T.ts_total;
    const int grp = (item / T.ts_total) % groups;
    const int frame = item / (T.ts_total * groups);
    const int tid = threadIdx.x;
    load_bpack(sm, bpack, grp, tid);
    __syncthreads();
    score_item(T, frame, grp, it, sm, sm.P[tid >> 6], feat, nf, bias, thresh, dense, poskey, atomic_key, tid);
}

hipError_t launch_score(const LevelTable& T, int n, const float* feat, const float4* bpack, const float* bias,
                        int nf, float thresh, float* dense, unsigned long long* poskey, bool atomic_key,
                        hipStream_t s) {
    const int groups = (nf + FGROUP - 1) / FGROUP;
    const long long items = (long long)T.ts_total * n * groups;
    if (items <= 0) return hipSuccess;
    if (items > 0x7fffff00LL) return hipErrorInvalidValue;
    const int blocks = (int)((items + 7) / 8 * 8);
    hipLaunchKernelGGL(hog_score_kernel, dim3(blocks), dim3(SCORE_THREADS), 0, s, T, groups, (int)items, feat,
                       bpack, bias, nf, thresh, dense, poskey, atomic_key ? 1 : 0);
    return hipGetLastError();
}

}  // namespace hog
