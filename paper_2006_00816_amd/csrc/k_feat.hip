// Block normalisation and the 31-d cell features (Sec. IV-A normalisation
// and feature computation; Sec. V-A feature kernel).
#include "stage_feat.h"

namespace hog {

__global__ __launch_bounds__(FEAT_THREADS) void hog_feat_kernel(
    LevelTable T, const float* __restrict__ hist, float* __restrict__ feat, float* __restrict__ packed) {
    feat_cell(T, hist, feat, packed, (int)blockIdx.y, (int)blockIdx.x, (int)threadIdx.x);
}

hipError_t launch_feat(const LevelTable& T, int n, const float* hist, float* feat, float* packed,
                       hipStream_t s) {
    hipLaunchKernelGGL(hog_feat_kernel, dim3(T.tf_total, n), dim3(FEAT_THREADS), 0, s, T, hist, feat, packed);
    return hipGetLastError();
}

}  // namespace hog
