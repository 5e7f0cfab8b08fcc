// Split-precision (matrix-core) form of the posterior kernel.
//
// The pruned inverse transform of Eq. (fourier_explicit) restricted to the
// shift window |dx|, |dy| <= S is computed as two chained DFT-GEMMs on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulation):
//
//   stage 1 (along y, every spectrum column m):
//     Y(dy, m) = sum_l e^{+2 pi i l dy/ny} Z(l, m),  Z = conj(F I_o) F I0 CTF Env
//   The +dy and -dy rows share cos/sin rows:  with P = sum_l cos(.) Z and
//   Q = sum_l sin(.) Z (dy' = |dy|), Y(+-dy') = P +- iQ, so only 2S+1 real
//   DFT rows are needed.  Columns m = 0 and m = nx/2 are both Hermitian along
//   l, so they share one slot as Z(l,0) + i Z(l,nx/2); nx/2 slots remain.
//
//   stage 2 (c2r along x):
//     X(+-dy', dx) = E(dy', dx) -+ O(dy', dx),
//     E = sum_m [Re P G_re + Im P G_im],  O = sum_m [Im Q G_re - Re Q G_im],
//     G_re = w_m cos(2 pi m dx/nx), G_im = -w_m sin(2 pi m dx/nx)  (w_m = 2),
//     and for the packed slot G_re = 1, G_im = (-1)^dx.
//   O has the form of E after (Re Q, Im Q) -> (Im Q, -Re Q), a per-lane swap
//   on the stage-1 accumulators, so one G matrix serves both.
//
// Every FP32 operand x is split as hi = round(x), lo = round(x - hi) in
// fp16 (or bf16) and each product uses hi*hi + hi*lo + lo*hi, giving about
// 22 (16) significant bits with FP32 accumulation.  Spectra are stored
// scaled so |value| <= 1 (fp16 range); the scale returns in the FP64 terms.
//
// Likelihood epilogue (per image, orientation, CTF set): with rho^2(d) =
// X(d)^2 kappa, the reference value at the window maximum
//   l_ref = lgamma(n/2-1) - ln 2 - ln(n)/2 + (1-n/2) ln(pi A) - ln(B)/2
//           + (1-n/2) log1p(-rho^2_max)
// is FP64, and the shift sum is taken relative to it,
//   sum_d exp(l(d) - l_ref) = sum_d (1 + u_d)^-(n/2-1),
//   u_d = (rho^2_max - rho^2(d)) / (1 - rho^2_max) >= 0,
// where every term lies in (0, 1] and the maximum term is exactly 1, so the
// sum needs only FP32.  LSE merges across CTF sets are FP64.
//
// Work decomposition: a wave owns one (image, orientation) pair and loops
// over CTF sets in groups of EW, sharing the image/projection loads and the
// stage-1 DFT fragments (LDS) across the group.  Waves are persistent and
// walk a tiled (image, orientation) order so that concurrently running
// waves share spectra in L2 and the last-level cache.
#include <algorithm>

#include "common.hpp"

namespace bioem {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool BF> struct Prec;
template <> struct Prec<false> {
  using E = _Float16;
  using V = h8;
  static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Prec<true> {
  using E = __bf16;
  using V = b8;
  static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kTileImages = 16;     // item tiling for cache reuse
constexpr int kTileSlots = 128;

struct SplitArgs {
  LogpostArgs a;
  const uint4* F;       // stage-1 DFT fragments  [KS][NT][2][64]
  const uint4* G;       // stage-2 DFT fragments  [MT][NT][2][64]
  const float2* u;      // [nc][nx/2+1]  kappa e^{i phi_m} env_m
  const float2* v;      // [nc][ny]      e^{i phi_l} env_l
  int KS, MT;
  int n_ti, n_ts;       // item tiles along images and slots
};

template <bool BF>
__device__ __forceinline__ void split8(const float (&x)[8], typename Prec<BF>::V& hi,
                                       typename Prec<BF>::V& lo) {
  using E = typename Prec<BF>::E;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const E h = (E)x[r];
    hi[r] = h;
    lo[r] = (E)(x[r] - (float)h);
  }
}

// Eight consecutive complex values of one spectrum column, zero past ny.
__device__ __forceinline__ void load8(const float2* __restrict__ col, int l0, int ny, float2 (&o)[8]) {
  if (l0 + 8 <= ny) {
    const float4* p = reinterpret_cast<const float4*>(col + l0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float4 t = p[r];
      o[2 * r] = make_float2(t.x, t.y);
      o[2 * r + 1] = make_float2(t.z, t.w);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) o[r] = (l0 + r < ny) ? col[l0 + r] : make_float2(0.f, 0.f);
  }
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// log(1 + u) for u >= 0 with relative accuracy near FP32 epsilon (the
// rounding of 1 + u is compensated by u / ((1 + u) - 1)).
__device__ __forceinline__ float log1p_acc(float u) {
  const float w = 1.0f + u;
  const float d = w - 1.0f;
  return d == 0.0f ? u : __logf(w) * (u / d);
}

template <bool BF, int NT, int EW>
__global__ __launch_bounds__(kThreads, 1) void k_logpost_split(SplitArgs sa) {
  using P = Prec<BF>;
  using V = typename P::V;
  extern __shared__ uint4 lds[];
  const LogpostArgs& a = sa.a;
  const int KS = sa.KS, MT = sa.MT;
  const int nF = KS * NT * 2 * 64, nG = MT * NT * 2 * 64;
  for (int e = threadIdx.x; e < nF + nG; e += kThreads) lds[e] = e < nF ? sa.F[e] : sa.G[e - nF];
  __syncthreads();
  const uint4* Fs = lds;
  const uint4* Gs = lds + nF;

  const int nx = a.nx, ny = a.ny, S = a.S, W = 2 * S + 1;
  const int mh = nx / 2 + 1, half = nx / 2;
  const size_t len = (size_t)mh * ny;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * kWaves;
  const int nslots = a.cand ? a.k : a.nq;
  const int tile_items = kTileImages * kTileSlots;
  const int n_items = sa.n_ti * sa.n_ts * tile_items;
  const double n = (double)nx * ny, h = 0.5 * n;
  const float c2 = (float)(h - 1.0);
  const bool fr = li < 8;   // Fr (cos) column of a stage-1 tile; else Fi (sin)

  for (int item = wave; item < n_items; item += nwaves) {
    const int tile = item / tile_items, rr = item - tile * tile_items;
    const int ti = tile / sa.n_ts, ts = tile - ti * sa.n_ts;
    const int i = ti * kTileImages + rr / kTileSlots;
    const int slot = ts * kTileSlots + rr % kTileSlots;
    if (i >= a.ni || slot >= nslots) continue;   // uniform across the wave
    const int q = a.cand ? a.cand[(size_t)i * a.k + slot] : slot;
    const float2* O = a.ispec + (size_t)i * len;
    const float2* Pq = a.pspec + (size_t)q * len;
    const double A = a.istats[3 * i + 2];
    const int esc = 2 * (a.iexpo[i] + a.pexpo[q]);
    const double kn = lgamma(h - 1.0) - log(2.0) - 0.5 * log(n) + (1.0 - h) * log(M_PI * A);

    double lm = -INFINITY, ls = 0.0, bestv = -INFINITY;
    int bestc = -1, bestd = -1;

    for (int cg = 0; cg < a.nc && A > 0.0; cg += EW) {
      f4 acc2[EW][NT][NT];
#pragma unroll
      for (int e = 0; e < EW; ++e)
#pragma unroll
        for (int x = 0; x < NT; ++x)
#pragma unroll
          for (int y = 0; y < NT; ++y) acc2[e][x][y] = f4{0.f, 0.f, 0.f, 0.f};

      for (int mt = 0; mt < MT; ++mt) {
        f4 acc1[EW][NT][2];
#pragma unroll
        for (int e = 0; e < EW; ++e)
#pragma unroll
          for (int x = 0; x < NT; ++x) acc1[e][x][0] = acc1[e][x][1] = f4{0.f, 0.f, 0.f, 0.f};
        const int s = 16 * mt + li;          // stage-1 row: spectrum slot
        const bool live = s < half;
        const bool packed = s == 0;          // slot 0 carries columns 0 and nx/2
        const float2* Oc = O + (size_t)(live ? s : 0) * ny;
        const float2* Pc = Pq + (size_t)(live ? s : 0) * ny;
        for (int ks = 0; ks < KS; ++ks) {
          const int l0 = 32 * ks + 8 * lg;
          float2 w0[8], wn[8];
          {
            float2 o[8], p[8];
            load8(Oc, l0, ny, o);
            load8(Pc, l0, ny, p);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              const float re = o[r].x * p[r].x + o[r].y * p[r].y;
              const float im = o[r].x * p[r].y - o[r].y * p[r].x;
              w0[r] = live ? make_float2(re, im) : make_float2(0.f, 0.f);
            }
            if (packed && l0 == 0) w0[0] = make_float2(0.f, 0.f);   // Z(0,0) := 0
          }
          if (packed) {
            float2 o[8], p[8];
            load8(O + (size_t)half * ny, l0, ny, o);
            load8(Pq + (size_t)half * ny, l0, ny, p);
#pragma unroll
            for (int r = 0; r < 8; ++r)
              wn[r] = make_float2(o[r].x * p[r].x + o[r].y * p[r].y, o[r].x * p[r].y - o[r].y * p[r].x);
          }
          V fh[NT], fl[NT];
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            const uint4 th = Fs[((ks * NT + ct) * 2 + 0) * 64 + lane];
            const uint4 tl = Fs[((ks * NT + ct) * 2 + 1) * 64 + lane];
            fh[ct] = __builtin_bit_cast(V, th);
            fl[ct] = __builtin_bit_cast(V, tl);
          }
#pragma unroll
          for (int e = 0; e < EW; ++e) {
            const int c = cg + e;
            if (c >= a.nc) break;
            const float2* vc = sa.v + (size_t)c * ny;
            const float2 u0 = sa.u[(size_t)c * mh + (live ? s : 0)];
            float zr[8], zi[8];
            float2 vv[8];
            load8(vc, l0, ny, vv);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              const float t = u0.x * vv[r].x - u0.y * vv[r].y;
              zr[r] = w0[r].x * t;
              zi[r] = w0[r].y * t;
            }
            if (packed) {
              const float2 un = sa.u[(size_t)c * mh + half];
#pragma unroll
              for (int r = 0; r < 8; ++r) {
                const float t = un.x * vv[r].x - un.y * vv[r].y;
                // Z0 + i Zn
                zr[r] -= wn[r].y * t;
                zi[r] += wn[r].x * t;
              }
            }
            V zrh, zrl, zih, zil;
            split8<BF>(zr, zrh, zrl);
            split8<BF>(zi, zih, zil);
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
              acc1[e][ct][0] = P::mma(zrh, fh[ct], acc1[e][ct][0]);
              acc1[e][ct][0] = P::mma(zrh, fl[ct], acc1[e][ct][0]);
              acc1[e][ct][0] = P::mma(zrl, fh[ct], acc1[e][ct][0]);
              acc1[e][ct][1] = P::mma(zih, fh[ct], acc1[e][ct][1]);
              acc1[e][ct][1] = P::mma(zih, fl[ct], acc1[e][ct][1]);
              acc1[e][ct][1] = P::mma(zil, fh[ct], acc1[e][ct][1]);
            }
          }
        }
        // stage 2: this m-tile is one K-step of the c2r GEMM
        V gh[NT], gl[NT];
#pragma unroll
        for (int dt = 0; dt < NT; ++dt) {
          gh[dt] = __builtin_bit_cast(V, Gs[((mt * NT + dt) * 2 + 0) * 64 + lane]);
          gl[dt] = __builtin_bit_cast(V, Gs[((mt * NT + dt) * 2 + 1) * 64 + lane]);
        }
#pragma unroll
        for (int e = 0; e < EW; ++e) {
          if (cg + e >= a.nc) break;
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            float b[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float re = acc1[e][ct][0][r], im = acc1[e][ct][1][r];
              b[r] = fr ? re : im;
              b[4 + r] = fr ? im : -re;
            }
            V bh, bl;
            split8<BF>(b, bh, bl);
#pragma unroll
            for (int dt = 0; dt < NT; ++dt) {
              acc2[e][dt][ct] = P::mma(gh[dt], bh, acc2[e][dt][ct]);
              acc2[e][dt][ct] = P::mma(gh[dt], bl, acc2[e][dt][ct]);
              acc2[e][dt][ct] = P::mma(gl[dt], bh, acc2[e][dt][ct]);
            }
          }
        }
      }

      // likelihood epilogue per CTF set of the group
#pragma unroll
      for (int e = 0; e < EW; ++e) {
        const int c = cg + e;
        if (c >= a.nc) break;
        const double B = a.B[(size_t)q * a.nc + c];
        if (!(B > 0.0)) continue;
        float x2v[NT * NT * 4];
        float x2max = -1.0f;
        int dbest = 0x7fffffff;
#pragma unroll
        for (int dt = 0; dt < NT; ++dt)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float mine = acc2[e][dt][ct][r];
              const float other = __shfl_xor(mine, 8, 64);
              const float X = fr ? (mine - other) : (other + mine);
              const int dyp = 8 * ct + (li & 7);
              const int dxi = 16 * dt + 4 * lg + r;
              const bool ok = dyp <= S && (fr || dyp > 0) && dxi < W;
              const int d = ((fr ? dyp : -dyp) + S) * W + dxi;
              const float x2 = ok ? X * X : -1.0f;
              x2v[(dt * NT + ct) * 4 + r] = x2;
              if (ok && (x2 > x2max || (x2 == x2max && d < dbest))) { x2max = x2; dbest = d; }
            }
        const float wmax = wave_max_f(x2max);
        const int dmax = wave_min_i(x2max == wmax ? dbest : 0x7fffffff);
        const double kappa = ldexp(1.0, esc) / (n * n * A * B);
        const double rho2 = fmin((double)wmax * kappa, 1.0 - 0x1p-52);
        const double lref = kn - 0.5 * log(B) + (1.0 - h) * log1p(-rho2);
        const float cu = (float)(kappa / (1.0 - rho2));
        float sum = 0.0f;
#pragma unroll
        for (int k = 0; k < NT * NT * 4; ++k) {
          if (x2v[k] >= 0.0f) {
            const float uu = (wmax - x2v[k]) * cu;
            sum += __expf(-c2 * log1p_acc(uu));
          }
        }
        const double tot = wave_sum_d((double)sum);
        const double le = lref + log(tot);
        if (le > lm) {
          ls = ls * exp(lm - le) + 1.0;
          lm = le;
        } else {
          ls += exp(le - lm);
        }
        if (lref > bestv) { bestv = lref; bestc = c; bestd = dmax; }
      }
    }
    if (lane == 0) {
      bioem_rec rec;
      rec.lse = lm == -INFINITY ? -INFINITY : lm + log(ls);
      rec.bestl = bestv;
      rec.q = q;
      rec.c = bestc;
      rec.d = bestd;
      rec.pad = 0;
      a.rec[(size_t)i * nslots + slot] = rec;
    }
  }
}

// Fragment tables of the two DFT matrices, split into hi/lo parts.
template <bool BF>
__global__ void k_split_tables(int nx, int ny, int S, int NT, int KS, int MT, uint4* __restrict__ F,
                               uint4* __restrict__ G) {
  using E = typename Prec<BF>::E;
  const int nF = KS * NT * 2 * 64, nG = MT * NT * 2 * 64;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nF + nG) return;
  const int W = 2 * S + 1, half = nx / 2;
  double val[8];
  int hl, lane;
  if (idx < nF) {
    lane = idx & 63;
    hl = (idx >> 6) & 1;
    const int rest = idx >> 7;
    const int ct = rest % NT, ks = rest / NT;
    const int j = lane & 15, g = lane >> 4;
    const bool fr = j < 8;
    const int dyp = 8 * ct + (j & 7);
    for (int r = 0; r < 8; ++r) {
      const int l = 32 * ks + 8 * g + r;
      double x = 0.0;
      if (l < ny && dyp <= S) {
        const double2 t = twiddle64(((long)l * dyp) % ny, ny);
        x = fr ? t.x : t.y;
      }
      val[r] = x;
    }
  } else {
    const int k = idx - nF;
    lane = k & 63;
    hl = (k >> 6) & 1;
    const int rest = k >> 7;
    const int dt = rest % NT, mt = rest / NT;
    const int row = lane & 15, g = lane >> 4;
    const int dxi = 16 * dt + row, dx = dxi - S;
    for (int r = 0; r < 8; ++r) {
      const bool re = r < 4;
      const int s = 16 * mt + 4 * g + (r & 3);
      double x = 0.0;
      if (dxi < W && s < half) {
        if (s == 0) {
          x = re ? 1.0 : ((dx & 1) ? -1.0 : 1.0);
        } else {
          const long t = (((long)s * dx) % nx + nx) % nx;
          const double2 w = twiddle64(t, nx);
          x = re ? 2.0 * w.x : -2.0 * w.y;
        }
      }
      val[r] = x;
    }
  }
  union { uint4 u; E e[8]; } pack;
  for (int r = 0; r < 8; ++r) {
    const E hi = (E)(float)val[r];
    pack.e[r] = hl == 0 ? hi : (E)(float)(val[r] - (double)(float)hi);
  }
  (idx < nF ? F[idx] : G[idx - nF]) = pack.u;
}

// Separable CTF factors: CTF(s) Env(s) = Re(u_m v_l) with
// u_m = kappa e^{i phi_m} env_m, v_l = e^{i phi_l} env_l, kappa = -A + i sqrt(1-A^2),
// phi = a s^2 / 2 split into its x and y parts, env = exp(-b s^2/2) likewise.
__global__ void k_ctf_factors(const double* __restrict__ ctf, int nc, int nx, int ny, double pixel,
                              float2* __restrict__ u, float2* __restrict__ v) {
  const int mh = nx / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nc * (mh + ny)) return;
  const int c = idx / (mh + ny), k = idx - c * (mh + ny);
  const double a = ctf[3 * c], amp = ctf[3 * c + 1], b = ctf[3 * c + 2];
  if (k < mh) {
    const double f = 2.0 * M_PI * k / (nx * pixel);
    const double s2 = f * f;
    double sn, cs;
    sincos(0.5 * a * s2, &sn, &cs);
    const double env = exp(-0.5 * b * s2);
    const double kr = -amp, ki = sqrt(1.0 - amp * amp);
    u[(size_t)c * mh + k] = make_float2((float)((kr * cs - ki * sn) * env), (float)((kr * sn + ki * cs) * env));
  } else {
    const int l = k - mh;
    const int ls = (l <= ny / 2) ? l : l - ny;
    const double f = 2.0 * M_PI * ls / (ny * pixel);
    const double s2 = f * f;
    double sn, cs;
    sincos(0.5 * a * s2, &sn, &cs);
    const double env = exp(-0.5 * b * s2);
    v[(size_t)c * ny + l] = make_float2((float)(cs * env), (float)(sn * env));
  }
}

int nt_for(int S) { return (S + 8) / 8; }   // ceil((S+1)/8) column tiles == ceil((2S+1)/16) dx tiles

size_t split_smem(int nx, int ny, int S) {
  const int NT = nt_for(S);
  const int KS = (ny + 31) / 32, MT = (nx / 2 + 15) / 16;
  return (size_t)(KS + MT) * NT * 2 * 64 * sizeof(uint4);
}

template <bool BF, int NT>
hipError_t launch_nt(hipStream_t s, const SplitArgs& sa, size_t smem, int grid) {
  constexpr int EW = 2;
  auto kern = k_logpost_split<BF, NT, EW>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), smem, s, sa);
  return hipGetLastError();
}

}  // namespace

bool split_supported(int nx, int ny, int S) {
  const int NT = nt_for(S);
  return NT >= 1 && NT <= 3 && split_smem(nx, ny, S) <= kMaxSmem;
}

hipError_t launch_logpost_split(hipStream_t s, const LogpostArgs& a, bool bf16) {
  const int NT = nt_for(a.S);
  const int KS = (a.ny + 31) / 32, MT = (a.nx / 2 + 15) / 16;
  const int nF = KS * NT * 2 * 64, nG = MT * NT * 2 * 64;
  const int mh = a.nx / 2 + 1;
  uint4* tabs = nullptr;
  float2* fac = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&tabs), sizeof(uint4) * (nF + nG), s);
  if (e != hipSuccess) return e;
  e = hipMallocAsync(reinterpret_cast<void**>(&fac), sizeof(float2) * (size_t)a.nc * (mh + a.ny), s);
  if (e != hipSuccess) { hipFreeAsync(tabs, s); return e; }
  const int nt = nF + nG;
  if (bf16)
    hipLaunchKernelGGL(k_split_tables<true>, dim3((nt + 255) / 256), dim3(256), 0, s, a.nx, a.ny, a.S, NT, KS, MT,
                       tabs, tabs + nF);
  else
    hipLaunchKernelGGL(k_split_tables<false>, dim3((nt + 255) / 256), dim3(256), 0, s, a.nx, a.ny, a.S, NT, KS, MT,
                       tabs, tabs + nF);
  const int nfac = a.nc * (mh + a.ny);
  hipLaunchKernelGGL(k_ctf_factors, dim3((nfac + 255) / 256), dim3(256), 0, s, a.ctf, a.nc, a.nx, a.ny,
                     a.pixel, fac, fac + (size_t)a.nc * mh);
  SplitArgs sa;
  sa.a = a;
  sa.F = tabs;
  sa.G = tabs + nF;
  sa.u = fac;
  sa.v = fac + (size_t)a.nc * mh;
  sa.KS = KS;
  sa.MT = MT;
  const int nslots = a.cand ? a.k : a.nq;
  sa.n_ti = (a.ni + kTileImages - 1) / kTileImages;
  sa.n_ts = (nslots + kTileSlots - 1) / kTileSlots;
  const long n_items = (long)sa.n_ti * sa.n_ts * kTileImages * kTileSlots;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  const long want = (n_items + kWaves - 1) / kWaves;
  const int grid = (int)std::min<long>(want, (long)ncu);
  const size_t smem = split_smem(a.nx, a.ny, a.S);
  if (NT == 1) e = bf16 ? launch_nt<true, 1>(s, sa, smem, grid) : launch_nt<false, 1>(s, sa, smem, grid);
  else if (NT == 2) e = bf16 ? launch_nt<true, 2>(s, sa, smem, grid) : launch_nt<false, 2>(s, sa, smem, grid);
  else e = bf16 ? launch_nt<true, 3>(s, sa, smem, grid) : launch_nt<false, 3>(s, sa, smem, grid);
  hipFreeAsync(fac, s);
  hipFreeAsync(tabs, s);
  return e;
}

}  // namespace bioem
