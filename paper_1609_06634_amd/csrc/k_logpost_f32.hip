// FP32 vector-ALU form of the posterior kernel.
//
// One workgroup scores one (image, orientation) pair against every CTF set
// (Listing 1 with the image loop mapped to the grid).  Per CTF set c:
//   Z(s)   = conj(F(I_o)(s)) F(I0_q)(s) CTF_c(s) Env_c(s),  Z(0) := 0
//            (the product of Eq. fourier; zeroing the DC term removes the
//            mean, i.e. the offset mu, exactly),
//   Y(dy,m)= sum_l Z(l,m) e^{+2 pi i l dy/ny}        (pruned inverse along y)
//   X(d)   = sum_m w_m Re[Y(dy,m) e^{+2 pi i m dx/nx}] (pruned c2r along x)
// for |dx|, |dy| <= S only: Eq. (fourier_explicit) evaluated at the window of
// displacements (the paper notes only some coefficients are needed).
// Each evaluation leaves the window maximum of X^2, its position, and
//   srel = sum_d exp(l(d) - l(d_max)),
//   l(d) - l(d_max) = (1 - n/2) [log1p(-rho^2(d)) - log1p(-rho^2_max)],
// taken in FP64; the per-image FP64 constants are added at finalisation.
// Reductions use a fixed thread order, so results are deterministic.
#include "common.hpp"

namespace bioem {

namespace {

constexpr int kThreads = 256;
constexpr int kColBlock = 8;   // spectrum columns staged per step

struct Smem {
  float2 *twy, *twx, *zb, *Y;
  float* X2;
  double* rd;
  float* rv;
  int* ri;
};

__device__ Smem carve(unsigned char* smem, int nx, int ny, int S) {
  const int W = 2 * S + 1, mh = nx / 2 + 1;
  Smem m;
  m.twy = reinterpret_cast<float2*>(smem);            // e^{+2 pi i t/ny}
  m.twx = m.twy + ny;                                  // e^{+2 pi i t/nx}
  m.zb = m.twx + nx;                                   // [kColBlock][ny]
  m.Y = m.zb + kColBlock * ny;                         // [W][mh]
  m.X2 = reinterpret_cast<float*>(m.Y + W * mh);       // [W*W]
  m.rd = reinterpret_cast<double*>(m.X2 + ((W * W + 1) & ~1));
  m.rv = reinterpret_cast<float*>(m.rd + kThreads);
  m.ri = reinterpret_cast<int*>(m.rv + kThreads);
  return m;
}

__device__ void load_twiddles(const Smem& m, int nx, int ny) {
  for (int t = threadIdx.x; t < ny; t += kThreads) {
    const double2 v = twiddle64(t, ny);
    m.twy[t] = make_float2((float)v.x, (float)v.y);
  }
  for (int t = threadIdx.x; t < nx; t += kThreads) {
    const double2 v = twiddle64(t, nx);
    m.twx[t] = make_float2((float)v.x, (float)v.y);
  }
}

// X(d)^2 over the window for one (image, orientation, CTF set) into m.X2,
// and its maximum with the lowest index on ties.  Called by the whole block.
__device__ void eval_window(const Smem& m, const float2* __restrict__ O, const float2* __restrict__ P,
                            const float* __restrict__ T, int nx, int ny, int ldy, int S, float& x2max,
                            int& dmax) {
  const int W = 2 * S + 1, mh = nx / 2 + 1, tid = threadIdx.x;
  for (int m0 = 0; m0 < mh; m0 += kColBlock) {
    __syncthreads();
    for (int e = tid; e < kColBlock * ny; e += kThreads) {
      const int mm = e / ny, l = e - mm * ny, col = m0 + mm;
      float2 z = make_float2(0.f, 0.f);
      if (col < mh && (col | l) != 0) {
        const float2 o = O[col * ldy + l], p = P[col * ldy + l];
        const float t = T[col * ldy + l];
        z = make_float2((o.x * p.x + o.y * p.y) * t, (o.x * p.y - o.y * p.x) * t);
      }
      m.zb[e] = z;
    }
    __syncthreads();
    for (int o = tid; o < W * kColBlock; o += kThreads) {
      const int dyi = o / kColBlock, mm = o - dyi * kColBlock, col = m0 + mm;
      if (col >= mh) continue;
      const int step = ((dyi - S) % ny + ny) % ny;
      const float2* zc = m.zb + mm * ny;
      float re = 0.f, im = 0.f;
      int t = 0;
      for (int l = 0; l < ny; ++l) {
        const float2 w = m.twy[t], z = zc[l];
        re = fmaf(w.x, z.x, fmaf(-w.y, z.y, re));
        im = fmaf(w.x, z.y, fmaf(w.y, z.x, im));
        t += step;
        if (t >= ny) t -= ny;
      }
      m.Y[dyi * mh + col] = make_float2(re, im);
    }
  }
  __syncthreads();
  float bv = -1.0f;
  int bi = 0x7fffffff;
  for (int o = tid; o < W * W; o += kThreads) {
    const int dyi = o / W, dxi = o - dyi * W;
    const int step = ((dxi - S) % nx + nx) % nx;
    const float2* yr = m.Y + dyi * mh;
    float x = 0.f;
    int t = 0;
    for (int col = 0; col < mh; ++col) {
      const float w = (col == 0 || 2 * col == nx) ? 1.f : 2.f;
      const float2 y = yr[col], e = m.twx[t];
      x = fmaf(w, y.x * e.x - y.y * e.y, x);
      t += step;
      if (t >= nx) t -= nx;
    }
    const float x2 = x * x;
    m.X2[o] = x2;
    if (x2 > bv) { bv = x2; bi = o; }
  }
  m.rv[tid] = bv;
  m.ri[tid] = bi;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      if (m.rv[tid + w] > m.rv[tid] || (m.rv[tid + w] == m.rv[tid] && m.ri[tid + w] < m.ri[tid])) {
        m.rv[tid] = m.rv[tid + w];
        m.ri[tid] = m.ri[tid + w];
      }
    }
    __syncthreads();
  }
  x2max = m.rv[0];
  dmax = m.ri[0];
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_logpost_f32(LogpostArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx, ny = a.ny, S = a.S, W = 2 * S + 1, mh = nx / 2 + 1;
  const int ldy = a.ldy, len = mh * ldy;
  const Smem m = carve(smem, nx, ny, S);
  const int slot = blockIdx.x, i = blockIdx.y, tid = threadIdx.x;
  const int nslots = a.cand ? a.k : a.nq;
  const int q = a.cand ? a.cand[(size_t)i * a.k + slot] : slot;
  bioem_erec* out = a.rec + ((size_t)i * nslots + slot) * a.nc;
  load_twiddles(m, nx, ny);

  const double A = a.istats[3 * i + 2];
  const float2* O = a.ispec + (size_t)i * len;
  const float2* P = a.pspec + (size_t)q * len;
  const double h = 0.5 * (double)nx * ny;
  const int escale = 2 * (a.iexpo[i] + a.pexpo[q]);

  for (int c = 0; c < a.nc; ++c) {
    const double B = a.B[(size_t)q * a.nc + c];
    if (!(B > 0.0) || !(A > 0.0)) {   // uniform across the block
      if (tid == 0) out[c] = bioem_erec{-1.0f, 0.0f, -1, 0};
      continue;
    }
    float x2max;
    int dmax;
    eval_window(m, O, P, a.table + (size_t)c * len, nx, ny, ldy, S, x2max, dmax);
    const double kappa = ldexp(a.kscale / (A * B), escale);
    const double r2max = fmin((double)x2max * kappa, 1.0 - 0x1p-52);
    const double lmax = log1p(-r2max);
    double sum = 0.0;
    for (int o = tid; o < W * W; o += kThreads) {
      const double r2 = fmin((double)m.X2[o] * kappa, 1.0 - 0x1p-52);
      sum += exp((1.0 - h) * (log1p(-r2) - lmax));
    }
    m.rd[tid] = sum;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) m.rd[tid] += m.rd[tid + w];
      __syncthreads();
    }
    if (tid == 0) out[c] = bioem_erec{x2max, (float)m.rd[0], dmax, 0};
  }
}

// Best displacement of each image's maximising (orientation, CTF set), for
// forms whose main kernel does not track the argmax.  grid: ni; block: 256.
__global__ __launch_bounds__(kThreads) void k_best_shift(LogpostArgs a, bioem_best* __restrict__ best) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx, ny = a.ny, S = a.S, W = 2 * S + 1, mh = nx / 2 + 1;
  const int ldy = a.ldy, len = mh * ldy;
  const int i = blockIdx.x;
  const bioem_best b = best[i];
  if (b.status != 0 || b.q < 0) return;   // uniform across the block
  const Smem m = carve(smem, nx, ny, S);
  load_twiddles(m, nx, ny);
  float x2max;
  int dmax;
  eval_window(m, a.ispec + (size_t)i * len, a.pspec + (size_t)b.q * len, a.table + (size_t)b.c * len, nx,
              ny, ldy, S, x2max, dmax);
  if (threadIdx.x == 0) {
    best[i].dy = dmax / W - S;
    best[i].dx = dmax % W - S;
  }
}

}  // namespace

size_t f32_smem_bytes(int nx, int ny, int S) {
  const int W = 2 * S + 1, mh = nx / 2 + 1;
  return sizeof(float2) * (size_t)(ny + nx + kColBlock * ny + W * mh) + sizeof(float) * ((W * W + 1) & ~1) +
         kThreads * (8 + 4 + 4) + 16;
}

hipError_t launch_best_shift(hipStream_t s, const LogpostArgs& a, bioem_best* best) {
  const size_t smem = f32_smem_bytes(a.nx, a.ny, a.S);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_best_shift),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_best_shift, dim3(a.ni), dim3(kThreads), smem, s, a, best);
  return hipGetLastError();
}

hipError_t launch_logpost_f32(hipStream_t s, const LogpostArgs& a) {
  const size_t smem = f32_smem_bytes(a.nx, a.ny, a.S);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_logpost_f32),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  dim3 grid(a.cand ? a.k : a.nq, a.ni);
  hipLaunchKernelGGL(k_logpost_f32, grid, dim3(kThreads), smem, s, a);
  return hipGetLastError();
}

}  // namespace bioem
