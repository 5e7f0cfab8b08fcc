// FP32 vector-ALU form of the posterior kernel, plus the per-image finalisation
// shared by every form.
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
// The likelihood at every d is then evaluated in FP64 and log-sum-exp reduced
// with a fixed thread order, so results are deterministic.
#include "common.hpp"

namespace bioem {

namespace {

constexpr int kThreads = 256;
constexpr int kColBlock = 8;   // spectrum columns staged per step

struct Lse {
  double m, s;   // running max and sum of exp(v - m)
};

BIOEM_DEV void lse_add(Lse& a, double v) {
  if (v == -INFINITY) return;
  if (v > a.m) {
    a.s = a.s * exp(a.m - v) + 1.0;
    a.m = v;
  } else {
    a.s += exp(v - a.m);
  }
}

BIOEM_DEV Lse lse_merge(Lse a, Lse b) {
  if (a.m == -INFINITY) return b;
  if (b.m == -INFINITY) return a;
  if (a.m >= b.m) return {a.m, a.s + b.s * exp(b.m - a.m)};
  return {b.m, b.s + a.s * exp(a.m - b.m)};
}

// (value, flat index) with ties to the lower index.
BIOEM_DEV bool better(double v, int idx, double bv, int bidx) {
  return v > bv || (v == bv && idx < bidx);
}

__global__ __launch_bounds__(kThreads) void k_logpost_f32(LogpostArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = a.nx, ny = a.ny, S = a.S, W = 2 * S + 1, mh = nx / 2 + 1;
  const int len = mh * ny;
  float2* twy = reinterpret_cast<float2*>(smem);      // e^{+2 pi i t/ny}
  float2* twx = twy + ny;                              // e^{+2 pi i t/nx}
  float2* zb = twx + nx;                               // [kColBlock][ny]
  float2* Y = zb + kColBlock * ny;                     // [W][mh]
  double* rm = reinterpret_cast<double*>(Y + W * mh);  // reduction scratch
  double* rs = rm + kThreads;
  double* rb = rs + kThreads;
  int* ri = reinterpret_cast<int*>(rb + kThreads);

  const int slot = blockIdx.x, i = blockIdx.y, tid = threadIdx.x;
  const int nslots = a.cand ? a.k : a.nq;
  const int q = a.cand ? a.cand[(size_t)i * a.k + slot] : slot;
  bioem_rec* out = a.rec + (size_t)i * nslots + slot;

  for (int t = tid; t < ny; t += kThreads) {
    const double2 v = twiddle64(t, ny);
    twy[t] = make_float2((float)v.x, (float)v.y);
  }
  for (int t = tid; t < nx; t += kThreads) {
    const double2 v = twiddle64(t, nx);
    twx[t] = make_float2((float)v.x, (float)v.y);
  }

  const double A = a.istats[3 * i + 2];
  const float2* O = a.ispec + (size_t)i * len;
  const float2* P = a.pspec + (size_t)q * len;
  const double n = (double)nx * ny, h = 0.5 * n;
  const double kn = lgamma(h - 1.0) - log(2.0) - 0.5 * log(n) + (1.0 - h) * log(M_PI * A);
  const int escale = 2 * (a.iexpo[i] + a.pexpo[q]);

  Lse acc{-INFINITY, 0.0};
  double bv = -INFINITY;
  int bidx = 0x7fffffff;

  for (int c = 0; c < a.nc; ++c) {
    const double B = a.B[(size_t)q * a.nc + c];
    if (!(B > 0.0) || !(A > 0.0)) continue;   // uniform across the block
    const float* T = a.table + (size_t)c * len;
    for (int m0 = 0; m0 < mh; m0 += kColBlock) {
      __syncthreads();
      for (int e = tid; e < kColBlock * ny; e += kThreads) {
        const int mm = e / ny, l = e - mm * ny, m = m0 + mm;
        float2 z = make_float2(0.f, 0.f);
        if (m < mh && (m | l) != 0) {
          const float2 o = O[m * ny + l], p = P[m * ny + l];
          const float t = T[m * ny + l];
          z = make_float2((o.x * p.x + o.y * p.y) * t, (o.x * p.y - o.y * p.x) * t);
        }
        zb[e] = z;
      }
      __syncthreads();
      for (int o = tid; o < W * kColBlock; o += kThreads) {
        const int dyi = o / kColBlock, mm = o - dyi * kColBlock, m = m0 + mm;
        if (m >= mh) continue;
        const int step = ((dyi - S) % ny + ny) % ny;
        const float2* zc = zb + mm * ny;
        float re = 0.f, im = 0.f;
        int t = 0;
        for (int l = 0; l < ny; ++l) {
          const float2 w = twy[t], z = zc[l];
          re = fmaf(w.x, z.x, fmaf(-w.y, z.y, re));
          im = fmaf(w.x, z.y, fmaf(w.y, z.x, im));
          t += step;
          if (t >= ny) t -= ny;
        }
        Y[dyi * mh + m] = make_float2(re, im);
      }
    }
    __syncthreads();
    const double kappa = ldexp(1.0, escale) / (n * n * A * B);
    const double kc = kn - 0.5 * log(B);
    for (int o = tid; o < W * W; o += kThreads) {
      const int dyi = o / W, dxi = o - dyi * W;
      const int step = ((dxi - S) % nx + nx) % nx;
      const float2* yr = Y + dyi * mh;
      float x = 0.f;
      int t = 0;
      for (int m = 0; m < mh; ++m) {
        const float w = (m == 0 || 2 * m == nx) ? 1.f : 2.f;
        const float2 y = yr[m], e = twx[t];
        x = fmaf(w, y.x * e.x - y.y * e.y, x);
        t += step;
        if (t >= nx) t -= nx;
      }
      const double rho2 = fmin((double)x * (double)x * kappa, 1.0 - 0x1p-52);
      const double l = kc + (1.0 - h) * log1p(-rho2);
      lse_add(acc, l);
      const int idx = c * W * W + o;
      if (better(l, idx, bv, bidx)) { bv = l; bidx = idx; }
    }
  }

  // Deterministic block reduction of (LSE, best).
  __syncthreads();
  rm[tid] = acc.m; rs[tid] = acc.s; rb[tid] = bv; ri[tid] = bidx;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const Lse x = lse_merge({rm[tid], rs[tid]}, {rm[tid + w], rs[tid + w]});
      rm[tid] = x.m; rs[tid] = x.s;
      if (better(rb[tid + w], ri[tid + w], rb[tid], ri[tid])) { rb[tid] = rb[tid + w]; ri[tid] = ri[tid + w]; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    bioem_rec r;
    r.lse = rm[0] == -INFINITY ? -INFINITY : rm[0] + log(rs[0]);
    r.bestl = rb[0];
    r.q = q;
    const int wd = W * W;
    r.c = ri[0] == 0x7fffffff ? -1 : ri[0] / wd;
    r.d = ri[0] == 0x7fffffff ? -1 : ri[0] - r.c * wd;
    r.pad = 0;
    *out = r;
  }
}

// Per image: LSE over evaluated orientations, best grid point, optional
// per-orientation posteriors.  grid: ni; block: 256.
__global__ __launch_bounds__(kThreads) void k_finalize(const bioem_rec* __restrict__ rec, int nslots,
                                                       int nq_total, const double* __restrict__ istats,
                                                       double log_prior, double* __restrict__ logp,
                                                       bioem_best* __restrict__ best,
                                                       double* __restrict__ orient) {
  __shared__ double rm[kThreads], rs[kThreads], rb[kThreads];
  __shared__ int ri[kThreads];
  const int i = blockIdx.x, tid = threadIdx.x;
  const bioem_rec* r = rec + (size_t)i * nslots;
  if (orient && nslots != nq_total)
    for (int q = tid; q < nq_total; q += kThreads) orient[(size_t)i * nq_total + q] = -INFINITY;
  __syncthreads();
  Lse acc{-INFINITY, 0.0};
  double bv = -INFINITY;
  int bslot = 0x7fffffff;
  for (int s = tid; s < nslots; s += kThreads) {
    const bioem_rec x = r[s];
    lse_add(acc, x.lse);
    if (x.c >= 0) {
      // order by (q, c, d): the record already holds its lowest (c, d)
      const bool take = x.bestl > bv ||
                        (x.bestl == bv && bslot != 0x7fffffff && x.q < r[bslot].q);
      if (take) { bv = x.bestl; bslot = s; }
    }
    if (orient) orient[(size_t)i * nq_total + x.q] = x.lse + log_prior;
  }
  rm[tid] = acc.m; rs[tid] = acc.s; rb[tid] = bv; ri[tid] = bslot;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const Lse x = lse_merge({rm[tid], rs[tid]}, {rm[tid + w], rs[tid + w]});
      rm[tid] = x.m; rs[tid] = x.s;
      const int so = ri[tid + w], sm = ri[tid];
      bool take = false;
      if (so != 0x7fffffff) {
        if (sm == 0x7fffffff) take = true;
        else if (rb[tid + w] > rb[tid]) take = true;
        else if (rb[tid + w] == rb[tid] && r[so].q < r[sm].q) take = true;
      }
      if (take) { rb[tid] = rb[tid + w]; ri[tid] = so; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double A = istats[3 * i + 2];
    const bool bad = !(A > 0.0) || rm[0] == -INFINITY || ri[0] == 0x7fffffff;
    if (logp) logp[i] = bad ? NAN : rm[0] + log(rs[0]) + log_prior;
    if (best) {
      bioem_best b;
      b.status = bad ? 1 : 0;
      if (bad) {
        b.logl = NAN; b.q = b.c = -1; b.dx = b.dy = 0;
      } else {
        const bioem_rec x = r[ri[0]];
        b.logl = x.bestl; b.q = x.q; b.c = x.c;
        // d encodes (dy + S) * W + (dx + S); W is recovered by the caller's S
        b.dx = x.d; b.dy = 0;
      }
      best[i] = b;
    }
  }
}

// Decode the packed displacement now that S is known.
__global__ void k_best_decode(bioem_best* best, int ni, int S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  bioem_best b = best[i];
  if (b.status == 0) {
    const int W = 2 * S + 1, d = b.dx;
    b.dy = d / W - S;
    b.dx = d - (d / W) * W - S;
    best[i] = b;
  }
}

}  // namespace

size_t f32_smem_bytes(int nx, int ny, int S) {
  const int W = 2 * S + 1, mh = nx / 2 + 1;
  return sizeof(float2) * (size_t)(ny + nx + kColBlock * ny + W * mh) + kThreads * (3 * 8 + 4) + 16;
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

hipError_t launch_finalize(hipStream_t s, const bioem_rec* rec, int ni, int nq_eval, int nq_total,
                           const double* istats, double log_prior, double* logp, bioem_best* best,
                           double* logp_orient) {
  hipLaunchKernelGGL(k_finalize, dim3(ni), dim3(kThreads), 0, s, rec, nq_eval, nq_total, istats,
                     log_prior, logp, best, logp_orient);
  return hipGetLastError();
}

hipError_t launch_best_decode(hipStream_t s, bioem_best* best, int ni, int S) {
  hipLaunchKernelGGL(k_best_decode, dim3((ni + 255) / 256), dim3(256), 0, s, best, ni, S);
  return hipGetLastError();
}

}  // namespace bioem
