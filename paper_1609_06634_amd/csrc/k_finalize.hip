// Per-image finalisation shared by every form of the posterior kernel.
//
// From each evaluation's window maximum of X^2 and its relative shift sum,
// the FP64 log-likelihood at the maximum is (Eq. likeli integrated over the
// offset, the scale and the noise, then Eq. Pmom on the grid)
//   l_max = lgamma(n/2-1) - ln 2 - ln(n)/2 + (1-n/2) ln(pi A) - ln(B)/2
//           + (1-n/2) log1p(-rho^2_max),   rho^2_max = X^2_max / (A B),
// and its contribution to the posterior is l_max + ln srel.  The image's log
// posterior is the log-sum-exp over orientations and CTF sets plus the
// uniform grid prior -ln(Nq Nc Nd); the per-orientation value is the same sum
// restricted to one orientation.  The maximising grid point is the largest
// l_max, ties to the lowest (q, c, dy, dx).  Every reduction runs in a fixed
// order (per-thread strided loops, then a tree), so results are
// deterministic.
#include "common.hpp"

namespace bioem {

namespace {

constexpr int kThreads = 256;

struct Lse {
  double m, s;   // running max and sum of exp(v - m)
};

BIOEM_DEV void lse_add(Lse& a, double v) {
  if (!(v > -INFINITY)) return;
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

struct Cand {
  double l;
  int q, c, d;
};

BIOEM_DEV bool cand_better(const Cand& x, const Cand& y) {
  if (x.l != y.l) return x.l > y.l;
  if (x.q != y.q) return x.q < y.q;
  if (x.c != y.c) return x.c < y.c;
  return x.d < y.d;
}

__global__ __launch_bounds__(kThreads) void k_finalize(FinalizeArgs f) {
  __shared__ double rm[kThreads], rs[kThreads];
  __shared__ Cand rb[kThreads];
  const int i = blockIdx.x, tid = threadIdx.x;
  const double n = (double)f.nx * f.ny, h = 0.5 * n;
  const double A = f.istats[3 * i + 2];
  const bool img_ok = A > 0.0;
  const double kn = img_ok ? lgamma(h - 1.0) - log(2.0) - 0.5 * log(n) + (1.0 - h) * log(M_PI * A) : 0.0;
  const int ei = f.iexpo[i];
  const bioem_erec* r = f.rec + (size_t)i * f.nslots * f.nc;
  if (f.orient && f.nslots != f.nq_total)
    for (int q = tid; q < f.nq_total; q += kThreads) f.orient[(size_t)i * f.nq_total + q] = -INFINITY;
  __syncthreads();
  Lse acc{-INFINITY, 0.0};
  Cand bt{-INFINITY, 0x7fffffff, 0x7fffffff, 0x7fffffff};
  for (int s = tid; s < f.nslots; s += kThreads) {
    const int q = f.cand ? f.cand[(size_t)i * f.k + s] : s;
    const int esc = 2 * (ei + f.pexpo[q]);
    Lse qs{-INFINITY, 0.0};
    for (int c = 0; c < f.nc && img_ok; ++c) {
      const bioem_erec x = r[(size_t)s * f.nc + c];
      const double B = f.B[(size_t)q * f.nc + c];
      if (!(x.x2max >= 0.0f) || !(B > 0.0)) continue;
      const double kappa = ldexp(1.0 / (n * n * A * B), esc);
      const double rho2 = fmin((double)x.x2max * kappa, 1.0 - 0x1p-52);
      const double lmax = kn - 0.5 * log(B) + (1.0 - h) * log1p(-rho2);
      lse_add(qs, lmax + log((double)x.srel));
      const Cand cd{lmax, q, c, x.d};
      if (cand_better(cd, bt)) bt = cd;
    }
    const double lq = qs.m == -INFINITY ? -INFINITY : qs.m + log(qs.s);
    lse_add(acc, lq);
    if (f.orient) f.orient[(size_t)i * f.nq_total + q] = lq + f.log_prior;
  }
  rm[tid] = acc.m;
  rs[tid] = acc.s;
  rb[tid] = bt;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const Lse x = lse_merge({rm[tid], rs[tid]}, {rm[tid + w], rs[tid + w]});
      rm[tid] = x.m;
      rs[tid] = x.s;
      if (cand_better(rb[tid + w], rb[tid])) rb[tid] = rb[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const bool bad = !img_ok || rm[0] == -INFINITY || rb[0].q == 0x7fffffff;
    if (f.logp) f.logp[i] = bad ? NAN : rm[0] + log(rs[0]) + f.log_prior;
    if (f.best) {
      bioem_best b;
      b.status = bad ? 1 : 0;
      if (bad) {
        b.logl = NAN; b.q = b.c = -1; b.dx = b.dy = 0;
      } else {
        const int W = 2 * f.S + 1;
        b.logl = rb[0].l; b.q = rb[0].q; b.c = rb[0].c;
        // forms that do not track the argmax leave d < 0; their best shift
        // is recovered by a separate pass
        b.dy = rb[0].d >= 0 ? rb[0].d / W - f.S : 0;
        b.dx = rb[0].d >= 0 ? rb[0].d % W - f.S : 0;
      }
      f.best[i] = b;
    }
  }
}

}  // namespace

hipError_t launch_finalize(hipStream_t s, const FinalizeArgs& f) {
  hipLaunchKernelGGL(k_finalize, dim3(f.ni), dim3(kThreads), 0, s, f);
  return hipGetLastError();
}

}  // namespace bioem
