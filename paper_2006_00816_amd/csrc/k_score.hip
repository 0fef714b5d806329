// Linear window scoring on the matrix cores (Sec. IV-A linear
// classification; Sec. V-A classifier and detection kernels), one launch
// over all frames, filter groups and levels.
#include "stage_score.h"

namespace hog {

// Work item = (frame, filter group, ROWS window rows of the frame's list
// of rows; 16, or 4 for small batches, which then spread over more
// compute units).  Neighbouring rows read 9 of their 10 feature rows in
// common, so the items of a frame are placed on one XCD (one L2): the
// launch is 1-D, and block b runs item (b mod 8) * (blocks / 8) + b / 8.
template <int ROWS>
__global__ __launch_bounds__(ROWS * 64) void hog_score_kernel(
    LevelTable T, int groups, int per_frame, int items, const float* __restrict__ feat,
    const float4* __restrict__ bpack, const float* __restrict__ bias, int nf, float thresh,
    float* __restrict__ dense, unsigned long long* __restrict__ poskey, int atomic_key) {
    __shared__ ScoreSmemT<ROWS> sm;
    const int per = (int)(gridDim.x >> 3);
    const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (item >= items) return;
    const int it = item % per_frame;
    const int grp = (item / per_frame) % groups;
    const int frame = item / (per_frame * groups);
    const int tid = threadIdx.x;
    load_bpack(sm, bpack, grp, tid);
    __syncthreads();
    score_item<ROWS>(T, frame, grp, it, sm, sm.P[tid >> 6], feat, nf, bias, thresh, dense, poskey, atomic_key,
                     tid);
}

int score_rows_auto(const LevelTable& T, int n, int nf, int cus) {
    const long long items16 = (long long)T.ts_total * n * ((nf + FGROUP - 1) / FGROUP);
    return items16 < cus ? SCORE_SMALL_ROWS : ROWS_PER_ITEM;
}

hipError_t launch_score(const LevelTable& T, int n, const float* feat, const float4* bpack, const float* bias,
                        int nf, float thresh, float* dense, unsigned long long* poskey, bool atomic_key, int rows,
                        hipStream_t s) {
    const int groups = (nf + FGROUP - 1) / FGROUP;
    const int per_frame = (T.rows_total + rows - 1) / rows;
    const long long items = (long long)per_frame * n * groups;
    if (items <= 0) return hipSuccess;
    if (items > 0x7fffff00LL) return hipErrorInvalidValue;
    const int blocks = (int)((items + 7) / 8 * 8);
    if (rows == SCORE_SMALL_ROWS)
        hipLaunchKernelGGL(hog_score_kernel<SCORE_SMALL_ROWS>, dim3(blocks), dim3(SCORE_SMALL_ROWS * 64), 0, s, T,
                           groups, per_frame, (int)items, feat, bpack, bias, nf, thresh, dense, poskey,
                           atomic_key ? 1 : 0);
    else if (rows == ROWS_PER_ITEM)
        hipLaunchKernelGGL(hog_score_kernel<ROWS_PER_ITEM>, dim3(blocks), dim3(ROWS_PER_ITEM * 64), 0, s, T, groups,
                           per_frame, (int)items, feat, bpack, bias, nf, thresh, dense, poskey, atomic_key ? 1 : 0);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace hog
