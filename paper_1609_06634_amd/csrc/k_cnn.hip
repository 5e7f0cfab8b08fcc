// Kernels of the orientation-proposal network: a BF16 matrix-core GEMM with
// FP32 accumulation, the im2col / col2im pair of the 3x3 stride-2 pad-1
// convolutions, and the elementwise, reduction, loss, optimiser and top-K
// kernels around them.  Activations are stored FP32 in channel-major
// [C][B][H][W] order, so a whole convolution layer over a batch is one GEMM:
//   Y [Cout][B*Ho*Wo] = W [Cout][Cin*9] x cols [Cin*9][B*Ho*Wo].
// The GEMM rounds its FP32 operands to bf16 (round to nearest even) as it
// stages them in LDS and accumulates in FP32 on v_mfma_f32_16x16x32_bf16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "common.hpp"
#include "cnn.hpp"

namespace bioem {
namespace cnn {

namespace {

typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kTK = 32;   // workgroup tile of C and K step
constexpr int kLdk = kTK + 8;                 // padded LDS row (bf16): conflict-free 16 B reads

__device__ __forceinline__ uint16_t to_bf16(float x) {
  const __bf16 h = (__bf16)x;   // round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}

// C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C(m, n), element (m, k) of A at
// A[m*sam + k*sak] (likewise B, C).  grid: (ceil(N/64), ceil(M/64), splits);
// block 256.  Each wave owns a 32x32 quarter of the 64x64 tile (2x2 MFMA
// tiles).  With splits > 1, workgroup z sums the K range
// [z*kchunk, (z+1)*kchunk) and writes alpha * partial to part[z][M][N]
// (row-major); k_splitk_reduce then adds the partials in order.
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, long sam,
                                              long sak, const float* __restrict__ B, long sbk, long sbn,
                                              float* __restrict__ C, long scm, long scn, float alpha,
                                              float beta, int kchunk, float* __restrict__ part) {
  __shared__ __align__(16) uint16_t As[kTM][kLdk];
  __shared__ __align__(16) uint16_t Bs[kTN][kLdk];   // transposed: Bs[n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const bool a_mfast = sam == 1, b_nfast = sbn == 1;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  for (int k0 = kb; k0 < ke; k0 += kTK) {
    // stage the A and B tiles (64 x 32 each), consecutive threads along the
    // operand's contiguous index
#pragma unroll
    for (int r = 0; r < (kTM * kTK) / 256; ++r) {
      const int e = tid + 256 * r;
      const int mm = a_mfast ? e % kTM : e / kTK, kk = a_mfast ? e / kTM : e % kTK;
      const int m = m0 + mm, k = k0 + kk;
      const float v = (m < M && k < ke) ? A[(long)m * sam + (long)k * sak] : 0.0f;
      As[mm][kk] = to_bf16(v);
    }
#pragma unroll
    for (int r = 0; r < (kTN * kTK) / 256; ++r) {
      const int e = tid + 256 * r;
      const int nn = b_nfast ? e % kTN : e / kTK, kk = b_nfast ? e / kTN : e % kTK;
      const int n = n0 + nn, k = k0 + kk;
      const float v = (n < N && k < ke) ? B[(long)k * sbk + (long)n * sbn] : 0.0f;
      Bs[nn][kk] = to_bf16(v);
    }
    __syncthreads();
    // fragments: lane (i = lane % 16, g = lane / 16) holds row i, k = 8g..8g+7
    const int i = lane & 15, g = lane >> 4;
    b8 af[2], bf[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) af[a] = *reinterpret_cast<const b8*>(&As[wm + 16 * a + i][8 * g]);
#pragma unroll
    for (int b = 0; b < 2; ++b) bf[b] = *reinterpret_cast<const b8*>(&Bs[wn + 16 * b + i][8 * g]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bf[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  // D[i][j] of a 16x16 tile: lane j + 16 (i / 4), element i % 4
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * a + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * b + (lane & 15);
        if (m < M && n < N) {
          if (part) {
            part[((long)blockIdx.z * M + m) * N + n] = alpha * acc[a][b][r];
          } else {
            float* c = C + (long)m * scm + (long)n * scn;
            *c = beta == 0.0f ? alpha * acc[a][b][r] : fmaf(alpha, acc[a][b][r], beta * *c);
          }
        }
      }
}

// C(m, n) = sum_z part[z][m][n] + beta C(m, n), z in increasing order.
__global__ void k_splitk_reduce(int M, int N, int splits, const float* __restrict__ part, float* __restrict__ C,
                                long scm, long scn, float beta) {
  const long total = (long)M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    float acc = 0.0f;
    for (int z = 0; z < splits; ++z) acc += part[z * total + e];
    const long m = e / N, n = e - m * N;
    float* c = C + m * scm + n * scn;
    *c = beta == 0.0f ? acc : acc + beta * *c;
  }
}

// cols[(c*9 + u*3 + v)][(b*Ho + r)*Wo + s] = x[c][b][2r+u-1][2s+v-1] (0 outside).
__global__ void k_im2col(const float* __restrict__ x, int C, int B, int H, int W, float* __restrict__ cols) {
  const int Ho = H / 2, Wo = W / 2;
  const long P = (long)B * Ho * Wo, total = (long)C * 9 * P;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / P, col = e - row * P;
    const int c = (int)(row / 9), uv = (int)(row - 9L * c), u = uv / 3, v = uv - 3 * u;
    const int s = (int)(col % Wo);
    const long t = col / Wo;
    const int r = (int)(t % Ho), b = (int)(t / Ho);
    const int y = 2 * r + u - 1, xx = 2 * s + v - 1;
    cols[e] = (y >= 0 && y < H && xx >= 0 && xx < W) ? x[(((long)c * B + b) * H + y) * W + xx] : 0.0f;
  }
}

// Adjoint of k_im2col, as a gather (each input pixel sums the entries that
// read it, in a fixed order): dx[c][b][y][x] = sum over (u, v) with
// y = 2r+u-1, x = 2s+v-1 of dcols[(c, u, v)][(b, r, s)].
__global__ void k_col2im(const float* __restrict__ dcols, int C, int B, int H, int W, float* __restrict__ dx) {
  const int Ho = H / 2, Wo = W / 2;
  const long P = (long)B * Ho * Wo, total = (long)C * B * H * W;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int xx = (int)(e % W);
    long t = e / W;
    const int y = (int)(t % H);
    t /= H;
    const int b = (int)(t % B), c = (int)(t / B);
    float acc = 0.0f;
    for (int u = 0; u < 3; ++u) {
      const int yy = y + 1 - u;
      if (yy < 0 || (yy & 1) || (yy >> 1) >= Ho) continue;
      for (int v = 0; v < 3; ++v) {
        const int xv = xx + 1 - v;
        if (xv < 0 || (xv & 1) || (xv >> 1) >= Wo) continue;
        acc += dcols[((long)c * 9 + 3 * u + v) * P + ((long)b * Ho + (yy >> 1)) * Wo + (xv >> 1)];
      }
    }
    dx[e] = acc;
  }
}

// Per image: x = (I - mean) / sqrt(var + 1e-12), written as channel 0 of a
// [1][B][H][W] activation (FP64 sums).  grid: B; block 256.
__global__ __launch_bounds__(256) void k_standardize(const float* __restrict__ imgs, int npix,
                                                     float* __restrict__ out) {
  __shared__ double red[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* im = imgs + (long)b * npix;
  double s = 0.0;
  for (int p = tid; p < npix; p += 256) s += im[p];
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double mean = red[0] / npix;
  __syncthreads();
  double q = 0.0;
  for (int p = tid; p < npix; p += 256) {
    const double d = im[p] - mean;
    q += d * d;
  }
  red[tid] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0] / npix + 1e-12);
  for (int p = tid; p < npix; p += 256) out[(long)b * npix + p] = (float)((im[p] - mean) * inv);
}

// y[c][j] = relu(y[c][j] + bias[c]) over a [C][L] activation.
__global__ void k_bias_relu(float* __restrict__ y, const float* __restrict__ bias, int C, long L, int relu) {
  const long total = (long)C * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const float v = y[e] + bias[e / L];
    y[e] = relu ? fmaxf(v, 0.0f) : v;
  }
}

// Column bias for a row-major [R][Cn] matrix: y[r][c] += bias[c].
__global__ void k_bias_cols(float* __restrict__ y, const float* __restrict__ bias, int R, int Cn) {
  const long total = (long)R * Cn;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    y[e] += bias[e % Cn];
}

// dy *= (y > 0).
__global__ void k_relu_bwd(float* __restrict__ dy, const float* __restrict__ y, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    if (!(y[e] > 0.0f)) dy[e] = 0.0f;
}

// out[r] = scale * sum_j in[r*sr + j*sj], j < L; one block per row, fixed order.
__global__ __launch_bounds__(256) void k_row_sum(const float* __restrict__ in, long sr, long sj, long L,
                                                 float scale, float* __restrict__ out) {
  __shared__ float red[256];
  const int r = blockIdx.x, tid = threadIdx.x;
  float s = 0.0f;
  for (long j = tid; j < L; j += 256) s += in[r * sr + j * sj];
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[r] = scale * red[0];
}

// Flattened features of a [C][B][P] activation: f[(c*P + p)*B + b] =
// y[(c*B + b)*P + p] (inverse = 1 gives the adjoint, the gradient scatter).
__global__ void k_flatten(const float* __restrict__ in, int C, int B, int P, int inverse, float* __restrict__ out) {
  const long total = (long)C * B * P;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    // e indexes the [C][P][B] feature matrix
    const int b = (int)(e % B);
    const long t = e / B;
    const int pp = (int)(t % P), c = (int)(t / P);
    const long y = ((long)c * B + b) * P + pp;
    if (inverse) out[y] = in[e];
    else out[e] = in[y];
  }
}

// Soft-label cross entropy of logits z [B][nq] (row-major) against sparse
// targets (idx, p) [B][T]: loss_b = logsumexp(z_b) - sum_t p_t z_{b,i_t};
// dz = (softmax(z_b) - target_b) / B.  grid: B; block 256.
__global__ __launch_bounds__(256) void k_softmax_xent(const float* __restrict__ z, int nq, const int32_t* __restrict__ tidx,
                                                      const float* __restrict__ tp, int T, int B,
                                                      float* __restrict__ dz, float* __restrict__ loss) {
  __shared__ float redf[256];
  __shared__ double redd[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* zb = z + (long)b * nq;
  float m = -INFINITY;
  for (int q = tid; q < nq; q += 256) m = fmaxf(m, zb[q]);
  redf[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) redf[tid] = fmaxf(redf[tid], redf[tid + w]);
    __syncthreads();
  }
  const float mx = redf[0];
  double s = 0.0;
  for (int q = tid; q < nq; q += 256) s += exp((double)(zb[q] - mx));
  redd[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) redd[tid] += redd[tid + w];
    __syncthreads();
  }
  const double sum = redd[0];
  const float inv = (float)(1.0 / (sum * B));
  if (dz)
    for (int q = tid; q < nq; q += 256) dz[(long)b * nq + q] = (float)exp((double)(zb[q] - mx)) * inv;
  __syncthreads();
  if (tid == 0) {
    double dot = 0.0;
    for (int t = 0; t < T; ++t) {
      const int q = tidx[(long)b * T + t];
      dot += (double)tp[(long)b * T + t] * zb[q];
      if (dz) dz[(long)b * nq + q] -= tp[(long)b * T + t] / (float)B;
    }
    if (loss) loss[b] = (float)((double)mx + log(sum) - dot);
  }
}

// Adam with bias correction on FP32 master weights.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// Order-preserving key of a float (larger float -> larger key).
__device__ __forceinline__ uint32_t fkey(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Per image: the K largest logits (ties to the lower index), written in
// increasing index order, and their softmax mass.  The K-th largest key is
// found by a bitwise search over the key; indices are then compacted in
// index order with a block scan.  grid: B; block 256.
__global__ __launch_bounds__(256) void k_topk(const float* __restrict__ z, int nq, int K, int32_t* __restrict__ out,
                                              float* __restrict__ mass) {
  __shared__ int cnt[256];
  __shared__ double redd[256];
  __shared__ float redf[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* zb = z + (long)b * nq;
  // the largest threshold t with #{key >= t} >= K, one bit at a time
  uint32_t thr = 0;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t t = thr | (1u << bit);
    int c = 0;
    for (int q = tid; q < nq; q += 256) c += fkey(zb[q]) >= t;
    cnt[tid] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) cnt[tid] += cnt[tid + w];
      __syncthreads();
    }
    if (cnt[0] >= K) thr = t;
    __syncthreads();
  }
  // contiguous chunk per thread, so the compaction follows index order
  const int chunk = (nq + 255) / 256, q0 = tid * chunk, q1 = min(nq, q0 + chunk);
  int above = 0, equal = 0;
  for (int q = q0; q < q1; ++q) {
    const uint32_t k = fkey(zb[q]);
    above += k > thr;
    equal += k == thr;
  }
  // exclusive scans of the two counts
  cnt[tid] = above;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int v = tid >= o ? cnt[tid - o] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  const int above_total = cnt[255];
  __syncthreads();
  cnt[tid] = equal;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int v = tid >= o ? cnt[tid - o] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  const int rank_e = cnt[tid] - equal;      // ties at the threshold before this chunk
  const int take_equal = K - above_total;   // ties taken, lowest indices first
  // selected-before count per thread: its selected above + its selected equal
  int sel_mine = 0;
  {
    int e = rank_e;
    for (int q = q0; q < q1; ++q) {
      const uint32_t k = fkey(zb[q]);
      if (k > thr) ++sel_mine;
      else if (k == thr && e < take_equal) { ++sel_mine; ++e; }
    }
  }
  __syncthreads();
  cnt[tid] = sel_mine;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int v = tid >= o ? cnt[tid - o] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  int pos = cnt[tid] - sel_mine;
  {
    int e = rank_e;
    for (int q = q0; q < q1; ++q) {
      const uint32_t k = fkey(zb[q]);
      bool sel = false;
      if (k > thr) sel = true;
      else if (k == thr && e < take_equal) { sel = true; ++e; }
      if (sel) out[(long)b * K + pos++] = q;
    }
  }
  // softmax mass of the selection (FP64 sums)
  float m = -INFINITY;
  for (int q = tid; q < nq; q += 256) m = fmaxf(m, zb[q]);
  redf[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) redf[tid] = fmaxf(redf[tid], redf[tid + w]);
    __syncthreads();
  }
  const float mx = redf[0];
  double all = 0.0, sel = 0.0;
  {
    int e = rank_e;
    for (int q = q0; q < q1; ++q) {
      const uint32_t k = fkey(zb[q]);
      const double x = exp((double)(zb[q] - mx));
      all += x;
      if (k > thr) sel += x;
      else if (k == thr && e < take_equal) { sel += x; ++e; }
    }
  }
  __syncthreads();
  redd[tid] = all;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) redd[tid] += redd[tid + w];
    __syncthreads();
  }
  const double tot = redd[0];
  __syncthreads();
  redd[tid] = sel;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) redd[tid] += redd[tid + w];
    __syncthreads();
  }
  if (tid == 0 && mass) mass[b] = (float)(redd[0] / tot);
}

int blocks_for(long n) { return (int)std::min<long>((n + 255) / 256, 65536L); }

}  // namespace

hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, long sam, long sak, const float* B,
                long sbk, long sbn, float* C, long scm, long scn, float alpha, float beta, float* scratch,
                size_t scratch_floats) {
  if (M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  const long tiles = (long)((N + kTN - 1) / kTN) * ((M + kTM - 1) / kTM);
  // split long reductions over several workgroups when the tile grid is small
  long splits = 1;
  if (scratch && tiles < 512 && K > 2 * 4096) {
    splits = std::min<long>((K + 4095) / 4096, (512 + tiles - 1) / tiles);
    splits = std::min<long>(splits, (long)(scratch_floats / ((size_t)M * N)));
    splits = std::max<long>(splits, 1);
  }
  const int kchunk = (int)(((K + splits - 1) / splits + kTK - 1) / kTK * kTK);
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid((N + kTN - 1) / kTN, (M + kTM - 1) / kTM, (unsigned)splits);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, alpha, beta,
                     kchunk, splits > 1 ? scratch : nullptr);
  if (splits > 1)
    hipLaunchKernelGGL(k_splitk_reduce, dim3(blocks_for((long)M * N)), dim3(256), 0, s, M, N, (int)splits, scratch,
                       C, scm, scn, beta);
  return hipGetLastError();
}

hipError_t im2col(hipStream_t s, const float* x, int C, int B, int H, int W, float* cols) {
  hipLaunchKernelGGL(k_im2col, dim3(blocks_for((long)C * 9 * B * (H / 2) * (W / 2))), dim3(256), 0, s, x, C, B, H,
                     W, cols);
  return hipGetLastError();
}

hipError_t col2im(hipStream_t s, const float* dcols, int C, int B, int H, int W, float* dx) {
  hipLaunchKernelGGL(k_col2im, dim3(blocks_for((long)C * B * H * W)), dim3(256), 0, s, dcols, C, B, H, W, dx);
  return hipGetLastError();
}

hipError_t standardize(hipStream_t s, const float* imgs, int B, int npix, float* out) {
  hipLaunchKernelGGL(k_standardize, dim3(B), dim3(256), 0, s, imgs, npix, out);
  return hipGetLastError();
}

hipError_t bias_relu(hipStream_t s, float* y, const float* bias, int C, long L, bool relu) {
  hipLaunchKernelGGL(k_bias_relu, dim3(blocks_for((long)C * L)), dim3(256), 0, s, y, bias, C, L, relu ? 1 : 0);
  return hipGetLastError();
}

hipError_t bias_cols(hipStream_t s, float* y, const float* bias, int R, int Cn) {
  hipLaunchKernelGGL(k_bias_cols, dim3(blocks_for((long)R * Cn)), dim3(256), 0, s, y, bias, R, Cn);
  return hipGetLastError();
}

hipError_t relu_bwd(hipStream_t s, float* dy, const float* y, long n) {
  hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(n)), dim3(256), 0, s, dy, y, n);
  return hipGetLastError();
}

hipError_t row_sum(hipStream_t s, const float* in, int R, long sr, long sj, long L, float scale, float* out) {
  hipLaunchKernelGGL(k_row_sum, dim3(R), dim3(256), 0, s, in, sr, sj, L, scale, out);
  return hipGetLastError();
}

hipError_t flatten(hipStream_t s, const float* in, int C, int B, int P, bool inverse, float* out) {
  hipLaunchKernelGGL(k_flatten, dim3(blocks_for((long)C * B * P)), dim3(256), 0, s, in, C, B, P, inverse ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t softmax_xent(hipStream_t s, const float* z, int B, int nq, const int32_t* tidx, const float* tp, int T,
                        float* dz, float* loss) {
  hipLaunchKernelGGL(k_softmax_xent, dim3(B), dim3(256), 0, s, z, nq, tidx, tp, T, B, dz, loss);
  return hipGetLastError();
}

hipError_t adam(hipStream_t s, float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                float eps, int step) {
  const float c1 = 1.0f / (1.0f - powf(b1, (float)step)), c2 = 1.0f / (1.0f - powf(b2, (float)step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t topk(hipStream_t s, const float* z, int B, int nq, int K, int32_t* out, float* mass) {
  hipLaunchKernelGGL(k_topk, dim3(B), dim3(256), 0, s, z, nq, K, out, mass);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace bioem
