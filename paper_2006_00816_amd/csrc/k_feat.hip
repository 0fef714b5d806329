// Block normalisation and the 31-d cell features (Sec. IV-A normalisation
// and feature computation; Sec. V-A feature kernel).
#include "stage_feat.h"

namespace hog {

// F16: the feature maps hold the scorer's split fp16 operands
// (HOG_ARITH_F16X3; see feat_cell).
template <bool F16>
__global__ __launch_bounds__(FEAT_THREADS) void hog_feat_kernel(
    LevelTable T, const float* __restrict__ hist, float* __restrict__ feat, float* __restrict__ packed) {
    __shared__ uint4 stage[FEAT_THREADS * FPAD / 4];
    feat_cell<F16>(T, hist, feat, packed, (int)blockIdx.y, (int)blockIdx.x, (int)threadIdx.x, stage);
}

hipError_t launch_feat(const LevelTable& T, int n, const float* hist, float* feat, float* packed,
                       hipStream_t s, bool f16x3) {
    if (f16x3)
        hipLaunchKernelGGL(hog_feat_kernel<true>, dim3(T.tf_total, n), dim3(FEAT_THREADS), 0, s, T, hist, feat,
                           packed);
    else
        hipLaunchKernelGGL(hog_feat_kernel<false>, dim3(T.tf_total, n), dim3(FEAT_THREADS), 0, s, T, hist, feat,
                           packed);
    return hipGetLastError();
}

}  // namespace hog
