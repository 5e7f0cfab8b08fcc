// Real-space variant of the displacement sum with border cropping (Section 3,
// Center displacement).
//
// The calculated image moved by d is I1(r + d) where r + d lies in the box
// and 0 elsewhere: nothing wraps in, so unlike the Fourier variant the
// calculated image's centred sum of squares B depends on d.  For each image
// i, calculated image p (one per orientation and CTF set) and d in the
// (2S+1)^2 window:
//   X(d) = sum_r (I_o(r) - C_o/n) p(r + d)           (over r with r + d inside)
//   B(d) = sum p(r')^2 - (sum p(r'))^2 / n            (over the moved-in part)
//   l(d) = lgamma(n/2-1) - ln 2 - ln(n)/2 + (1-n/2) ln(pi A) - ln(B(d))/2
//          + (1-n/2) log1p(-X(d)^2 / (A B(d)))
// (Eq. likeli integrated over offset, scale and noise).  This is the direct
// correlation: W = (2S+1)^2 multiply-adds per pixel and evaluation, so it
// only pays for small windows.
//
// k_crop_xcorr: a workgroup takes 32 images x 8 calculated images (32 with
// S = 0, 16 with S = 1, four or two per thread); row by
// row it stages the images' centred rows in LDS and keeps the calculated
// images' 2S+1 rows around it in an LDS ring (one new row per step; zero
// outside the box, S zero columns on each side), and each thread forms one
// pair's W correlations of that row in FP32 from a register window, added
// to FP64 accumulators once per row.  Then the FP64 likelihood per d,
// and one record per evaluation: the window maximum l_max, the relative sum
// sum_d exp(l(d) - l_max) and the argmax (lowest (dy, dx) on ties).
#include "common.hpp"

namespace bioem {

namespace {

constexpr int kTileI = 32;         // images per workgroup
constexpr int kTileP = 8;          // threads along calculated images per workgroup
constexpr int kXThreads = kTileI * kTileP;
// Calculated images per thread: small windows have few accumulators, so each
// thread takes several calculated images and every staged image row serves
// more of them.
__host__ __device__ constexpr int crop_ppt(int S) { return S == 0 ? 4 : (S == 1 ? 2 : 1); }
constexpr int kSumThreads = 256;

BIOEM_DEV double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = kSumThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// B(d) of every calculated image: one workgroup per image, fixed-order sums.
__global__ __launch_bounds__(kSumThreads) void k_crop_norms(const float* __restrict__ p, int np, int nx, int ny,
                                                            int S, double* __restrict__ Bd) {
  __shared__ double red[kSumThreads];
  const int W1 = 2 * S + 1;
  const float* x = p + (size_t)blockIdx.x * nx * ny;
  const double n = (double)nx * ny;
  for (int w = 0; w < W1 * W1; ++w) {
    const int dy = w / W1 - S, dx = w % W1 - S;
    // the moved-in part: source rows [max(0,dy), ny+min(0,dy)), columns likewise
    const int k0 = max(0, dy), k1 = ny + min(0, dy), j0 = max(0, dx), j1 = nx + min(0, dx);
    const int cols = j1 - j0, cnt = (k1 - k0) * cols;
    double s = 0.0, s2 = 0.0;
    for (int e = threadIdx.x; e < cnt; e += kSumThreads) {
      const double v = x[(size_t)(k0 + e / cols) * nx + j0 + e % cols];
      s += v;
      s2 = fma(v, v, s2);
    }
    const double cs = block_sum(s, red);
    const double css = block_sum(s2, red);
    if (threadIdx.x == 0) Bd[(size_t)blockIdx.x * W1 * W1 + w] = css - cs * cs / n;
  }
}

template <int S>
__global__ __launch_bounds__(kXThreads) void k_crop_xcorr(CropArgs a) {
  constexpr int W1 = 2 * S + 1, W = W1 * W1, PPT = crop_ppt(S), TP = kTileP * PPT;
  extern __shared__ float lds[];
  const int nx = a.nx, ny = a.ny, pw = nx + 2 * S, iw = nx + 1;
  float* Li = lds;                           // [kTileI][nx + 1]: centred image rows
  float* Lp = lds + kTileI * iw;             // [TP][W1][nx + 2S]: ring of calculated rows
  // thread (ti, tq) takes image i0 + ti and calculated images p0 + tq + kTileP m, m < PPT
  const int t = threadIdx.x, tq = t % kTileP, ti = t / kTileP;
  const int i0 = blockIdx.y * kTileI, p0 = blockIdx.x * TP;
  const double n = (double)nx * ny;
  // calculated row kk (-S <= kk < ny + S) lives in ring slot (kk + S) mod W1;
  // columns 0..S-1 and S+nx.. of every slot stay zero
  auto load_prow = [&](int kk) {
    const int slot = (kk + S) % W1;
    for (int e = t; e < TP * nx; e += kXThreads) {
      const int b = e / nx, j = e % nx, pi = p0 + b;
      float v = 0.0f;
      if (pi < a.np && kk >= 0 && kk < ny) v = a.p[((size_t)pi * ny + kk) * nx + j];
      Lp[(b * W1 + slot) * pw + S + j] = v;
    }
  };
  for (int e = t; e < TP * W1; e += kXThreads)
    for (int c = 0; c < S; ++c) {
      Lp[e * pw + c] = 0.0f;
      Lp[e * pw + S + nx + c] = 0.0f;
    }
  for (int kk = -S; kk < S; ++kk) load_prow(kk);
  double acc[PPT][W];
#pragma unroll
  for (int m = 0; m < PPT; ++m)
#pragma unroll
    for (int w = 0; w < W; ++w) acc[m][w] = 0.0;
  for (int k = 0; k < ny; ++k) {
    __syncthreads();   // the previous row's reads are done (and the pads and first rows are set)
    for (int e = t; e < kTileI * nx; e += kXThreads) {
      const int b = e / nx, j = e % nx, i = i0 + b;
      float v = 0.0f;
      if (i < a.ni) v = (float)((double)a.imgs[((size_t)i * ny + k) * nx + j] - a.stats[3 * i] / n);
      Li[b * iw + j] = v;
    }
    load_prow(k + S);
    __syncthreads();
    float row[PPT][W];
#pragma unroll
    for (int m = 0; m < PPT; ++m)
#pragma unroll
      for (int w = 0; w < W; ++w) row[m][w] = 0.0f;
    const float* li = Li + ti * iw;
    // rows k - S .. k + S of this thread's calculated images
    const float* lp[PPT][W1];
#pragma unroll
    for (int m = 0; m < PPT; ++m)
#pragma unroll
      for (int dy = 0; dy < W1; ++dy) lp[m][dy] = Lp + ((tq + kTileP * m) * W1 + (k + dy) % W1) * pw;
    // win[m][dy][slot]: a sliding window of 2S+1 columns per calculated row
    // in registers; at column j, column j + dx sits in slot (j + dx) mod W1,
    // so with j unrolled by W1 every slot index is a constant and the window
    // advances by one LDS read per row instead of W1
    float win[PPT][W1][W1];
#pragma unroll
    for (int m = 0; m < PPT; ++m)
#pragma unroll
      for (int dy = 0; dy < W1; ++dy)
#pragma unroll
        for (int dx = 0; dx < W1; ++dx) win[m][dy][dx] = lp[m][dy][dx];
    for (int jb = 0; jb < nx; jb += W1) {
#pragma unroll
      for (int u = 0; u < W1; ++u) {
        const int j = jb + u;
        if (j < nx) {
          const float ic = li[j];
          const int nxt = min(j + W1, pw - 1);   // column j + 2S + 1 (unused past the row's end)
#pragma unroll
          for (int m = 0; m < PPT; ++m)
#pragma unroll
            for (int dy = 0; dy < W1; ++dy) {
#pragma unroll
              for (int dx = 0; dx < W1; ++dx)
                row[m][dy * W1 + dx] = fmaf(ic, win[m][dy][(u + dx) % W1], row[m][dy * W1 + dx]);
              win[m][dy][u] = lp[m][dy][nxt];
            }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m)
#pragma unroll
      for (int w = 0; w < W; ++w) acc[m][w] += (double)row[m][w];
  }
  const int i = i0 + ti;
  if (i >= a.ni) return;
  const double A = a.stats[3 * i + 2], h = 0.5 * n;
  const double kn = A > 0.0 ? lgamma(h - 1.0) - log(2.0) - 0.5 * log(n) + (1.0 - h) * log(M_PI * A) : 0.0;
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    const int pi = p0 + tq + kTileP * m;
    if (pi >= a.np) continue;
    bioem_crec rec{-INFINITY, 0.0, -1, 0};
    if (A > 0.0) {
      const double* B = a.Bd + (size_t)pi * W;
      auto ll = [&](int w) -> double {
        if (!(B[w] > 0.0)) return -INFINITY;
        const double rho2 = fmin(acc[m][w] * acc[m][w] / (A * B[w]), 1.0 - 0x1p-52);
        return kn - 0.5 * log(B[w]) + (1.0 - h) * log1p(-rho2);
      };
      double lmax = -INFINITY;
      int dmax = -1;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const double v = ll(w);
        if (v > lmax) {
          lmax = v;
          dmax = w;
        }
      }
      double sum = 0.0;
      if (dmax >= 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) sum += exp(ll(w) - lmax);
      }
      rec = bioem_crec{lmax, sum, dmax, 0};
    }
    a.rec[(size_t)i * a.np + pi] = rec;
  }
}

// Per image: log-sum-exp over calculated images of l_max + ln(relative sum),
// plus the uniform grid prior; the best grid point by (l, q, c, d), ties to
// the lowest (q, c, dy, dx).  Calculated image pi holds CTF set pi / nq and
// orientation pi % nq.
struct Best {
  double l;
  int q, c, d;
};

BIOEM_DEV bool better(const Best& x, const Best& y) {
  if (x.l != y.l) return x.l > y.l;
  if (x.q != y.q) return x.q < y.q;
  if (x.c != y.c) return x.c < y.c;
  return x.d < y.d;
}

__global__ __launch_bounds__(kSumThreads) void k_crop_finalize(CropArgs a, double log_prior, double* logp,
                                                               bioem_best* best) {
  __shared__ double rm[kSumThreads], rs[kSumThreads];
  __shared__ Best rb[kSumThreads];
  const int i = blockIdx.x, t = threadIdx.x;
  double m = -INFINITY, s = 0.0;
  Best bt{-INFINITY, 0x7fffffff, 0x7fffffff, 0x7fffffff};
  for (int pi = t; pi < a.np; pi += kSumThreads) {
    const bioem_crec r = a.rec[(size_t)i * a.np + pi];
    if (r.d < 0) continue;
    const double v = r.lmax + log(r.rel);
    if (v > m) {
      s = s * exp(m - v) + 1.0;
      m = v;
    } else {
      s += exp(v - m);
    }
    const Best c{r.lmax, pi % a.nq, pi / a.nq, r.d};
    if (better(c, bt)) bt = c;
  }
  rm[t] = m;
  rs[t] = s;
  rb[t] = bt;
  __syncthreads();
  for (int h = kSumThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double m1 = rm[t], m2 = rm[t + h];
      if (m2 != -INFINITY) {
        if (m1 == -INFINITY) {
          rm[t] = m2;
          rs[t] = rs[t + h];
        } else if (m1 >= m2) {
          rs[t] = rs[t] + rs[t + h] * exp(m2 - m1);
        } else {
          rs[t] = rs[t + h] + rs[t] * exp(m1 - m2);
          rm[t] = m2;
        }
      }
      if (better(rb[t + h], rb[t])) rb[t] = rb[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const bool bad = !(a.stats[3 * i + 2] > 0.0) || rm[0] == -INFINITY;
    logp[i] = bad ? NAN : rm[0] + log(rs[0]) + log_prior;
    bioem_best b;
    b.status = bad ? 1 : 0;
    if (bad) {
      b.logl = NAN;
      b.q = b.c = -1;
      b.dx = b.dy = 0;
    } else {
      const int W1 = 2 * a.S + 1;
      b.logl = rb[0].l;
      b.q = rb[0].q;
      b.c = rb[0].c;
      b.dy = rb[0].d / W1 - a.S;
      b.dx = rb[0].d % W1 - a.S;
    }
    best[i] = b;
  }
}

}  // namespace

size_t crop_smem_bytes(int nx, int S) {
  return sizeof(float) * ((size_t)kTileI * (nx + 1) + (size_t)kTileP * crop_ppt(S) * (2 * S + 1) * (nx + 2 * S));
}

hipError_t launch_crop_norms(hipStream_t s, const CropArgs& a) {
  hipLaunchKernelGGL(k_crop_norms, dim3(a.np), dim3(kSumThreads), 0, s, a.p, a.np, a.nx, a.ny, a.S, a.Bd);
  return hipGetLastError();
}

hipError_t launch_crop_xcorr(hipStream_t s, const CropArgs& a) {
  const int tp = kTileP * crop_ppt(a.S);
  const dim3 grid((a.np + tp - 1) / tp, (a.ni + kTileI - 1) / kTileI);
  const size_t smem = crop_smem_bytes(a.nx, a.S);
  if (smem > kMaxSmem) return hipErrorInvalidValue;
  const void* fn = nullptr;
  switch (a.S) {
    case 0: fn = reinterpret_cast<const void*>(k_crop_xcorr<0>); break;
    case 1: fn = reinterpret_cast<const void*>(k_crop_xcorr<1>); break;
    case 2: fn = reinterpret_cast<const void*>(k_crop_xcorr<2>); break;
    case 3: fn = reinterpret_cast<const void*>(k_crop_xcorr<3>); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  switch (a.S) {
    case 0: hipLaunchKernelGGL(k_crop_xcorr<0>, grid, dim3(kXThreads), smem, s, a); break;
    case 1: hipLaunchKernelGGL(k_crop_xcorr<1>, grid, dim3(kXThreads), smem, s, a); break;
    case 2: hipLaunchKernelGGL(k_crop_xcorr<2>, grid, dim3(kXThreads), smem, s, a); break;
    default: hipLaunchKernelGGL(k_crop_xcorr<3>, grid, dim3(kXThreads), smem, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_crop_finalize(hipStream_t s, const CropArgs& a, double log_prior, double* logp,
                                bioem_best* best) {
  hipLaunchKernelGGL(k_crop_finalize, dim3(a.ni), dim3(kSumThreads), 0, s, a, log_prior, logp, best);
  return hipGetLastError();
}

}  // namespace bioem
