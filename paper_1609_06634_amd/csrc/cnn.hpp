// Launchers of the proposal-network kernels (internal, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bioem {
namespace cnn {

// C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C(m, n) with element strides;
// bf16 products, FP32 accumulation.  scratch (may be null) lets a long K be
// split over workgroups (partials summed in a fixed order).
hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, long sam, long sak, const float* B,
                long sbk, long sbn, float* C, long scm, long scn, float alpha, float beta, float* scratch,
                size_t scratch_floats);
hipError_t im2col(hipStream_t s, const float* x, int C, int B, int H, int W, float* cols);
hipError_t col2im(hipStream_t s, const float* dcols, int C, int B, int H, int W, float* dx);
hipError_t standardize(hipStream_t s, const float* imgs, int B, int npix, float* out);
hipError_t bias_relu(hipStream_t s, float* y, const float* bias, int C, long L, bool relu);
hipError_t bias_cols(hipStream_t s, float* y, const float* bias, int R, int Cn);
hipError_t relu_bwd(hipStream_t s, float* dy, const float* y, long n);
hipError_t row_sum(hipStream_t s, const float* in, int R, long sr, long sj, long L, float scale, float* out);
// [C][B][P] activation <-> [C*P][B] feature matrix.
hipError_t flatten(hipStream_t s, const float* in, int C, int B, int P, bool inverse, float* out);
hipError_t softmax_xent(hipStream_t s, const float* z, int B, int nq, const int32_t* tidx, const float* tp, int T,
                        float* dz, float* loss);
hipError_t adam(hipStream_t s, float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                float eps, int step);
hipError_t topk(hipStream_t s, const float* z, int B, int nq, int K, int32_t* out, float* mass);

}  // namespace cnn
}  // namespace bioem
