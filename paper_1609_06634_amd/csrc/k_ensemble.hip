// Posterior of a model ensemble, Eq. (pb2) of Section 2.
//
// Per image i the ensemble's posterior is the weighted sum over models of the
// per-model posteriors, so in logs
//   e_i = ln sum_m w_m exp(logp[m][i]) = M_i + ln sum_m w_m exp(logp[m][i] - M_i)
// with M_i the largest logp[m][i] among the models of positive weight (the
// posteriors of a 224^2 box are near -2.3e5 nat, far below where exp
// underflows).  The images are independent, so the ensemble's log posterior
// over the set is sum_i e_i.  FP64 throughout.  The per-image kernel reads
// logp[m][i] with consecutive threads on consecutive images (coalesced); the
// sum over images is one workgroup with a fixed strided order and a fixed
// tree, so the total does not depend on anything but the inputs.
#include "common.hpp"

namespace bioem {

namespace {

constexpr int kImgThreads = 256;
constexpr int kSumThreads = 1024;

__global__ __launch_bounds__(kImgThreads) void k_ensemble_images(const double* __restrict__ logp, int nm,
                                                                 int ni, const double* __restrict__ w,
                                                                 double* __restrict__ per) {
  const int i = blockIdx.x * kImgThreads + threadIdx.x;
  if (i >= ni) return;
  double M = -INFINITY;
  bool nan = false;
  for (int m = 0; m < nm; ++m) {
    if (!(w[m] > 0.0)) continue;
    const double v = logp[(size_t)m * ni + i];
    nan |= isnan(v);
    M = fmax(M, v);
  }
  if (nan) {
    per[i] = NAN;
    return;
  }
  if (isinf(M)) {   // every weighted term -inf, or one of them +inf
    per[i] = M;
    return;
  }
  double s = 0.0;
  for (int m = 0; m < nm; ++m) {
    const double wm = w[m];
    if (wm > 0.0) s += wm * exp(logp[(size_t)m * ni + i] - M);
  }
  per[i] = M + log(s);
}

__global__ __launch_bounds__(kSumThreads) void k_ensemble_total(const double* __restrict__ per, int ni,
                                                                double* __restrict__ total) {
  __shared__ double part[kSumThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < ni; i += kSumThreads) acc += per[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kSumThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = part[0];
}

}  // namespace

hipError_t launch_ensemble(hipStream_t s, const double* logp, int nm, int ni, const double* w, double* per,
                           double* total) {
  if (ni > 0) {
    hipLaunchKernelGGL(k_ensemble_images, dim3((ni + kImgThreads - 1) / kImgThreads), dim3(kImgThreads), 0, s,
                       logp, nm, ni, w, per);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ensemble_total, dim3(1), dim3(kSumThreads), 0, s, per, ni, total);
  return hipGetLastError();
}

}  // namespace bioem
