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
// Shift-window epilogue (per image, orientation, CTF set): with rho^2(d) =
// X(d)^2 kappa and the window maximum rho^2_max, the shift sum relative to
// the maximising shift is
//   sum_d exp(l(d) - l_max) = sum_d (1 + u_d)^-(n/2-1),
//   u_d = (rho^2_max - rho^2(d)) / (1 - rho^2_max) >= 0,
// where every term lies in (0, 1] and the maximum term is exactly 1, so FP32
// suffices.  When c = n/2-1 >= 1024, terms with u >= 0.05 are below e^-50
// and log1p(u) is its degree-3 series on [0, 0.05]: the exponent error c u^4/4
// changes a term t = e^{-c log1p(u)} by at most about t c u^4/4 <= 1.2 / c^3
// (the product peaks at u = 4/c), below 2e-9 of the sum at c = 1024.  Each
// evaluation leaves (max X^2, relative sum); the FP64 likelihood constants,
// log-sum-exp merges and the best grid point are taken at finalisation, and
// the best displacement of each image is recovered afterwards.
//
// Work decomposition: a wave owns one (image, orientation, group of EW CTF
// sets) item and shares the image/projection loads and the stage-1 DFT
// fragments (LDS) across the group.  Consecutive waves take the other CTF
// groups of the same (image, orientation), so their spectrum loads meet in
// L1; items walk a tiled (image, orientation) order so that concurrently
// running waves share spectra in L2 and the last-level cache.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "split_common.hpp"

namespace bioem {

namespace {

constexpr int kTileImages = 32;     // default item tile (images x slots) for cache reuse
constexpr int kTileSlots = 128;

using namespace split;

struct SplitArgs {
  LogpostArgs a;
  const uint4* F;       // stage-1 DFT fragments  [KS][NT][2][64]
  const uint4* G;       // stage-2 DFT fragments  [MT][NT][2][64]
  int KS, MT;
  int ncg;              // CTF groups per (image, orientation)
  int ti, ts;           // item tile: images x slots
  int n_ti, n_ts;       // item tiles along images and slots
  int xcd;              // 1: tiles dealt to XCDs, images fastest within a tile
};

// Per-lane operands of one stage-1 K-step: the image and projection values of
// this lane's slot column and the CTF values of each CTF set of the group.
template <int EW>
struct Step {
  float2 o[8], p[8];
  float t[EW][8];
};

// K-step `step` (= mt * KS + ks) of this lane from the fragment-order copies:
// four contiguous 1 KB pieces per spectrum and two per CTF table.
template <int EW>
__device__ __forceinline__ void load_spectra(Step<EW>& st, const float4* __restrict__ Ot,
                                             const float4* __restrict__ Pt, int step, int lane) {
  const size_t c = (size_t)step * 256 + lane;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float4 v = Ot[c + 64 * r], w = Pt[c + 64 * r];
    st.o[2 * r] = make_float2(v.x, v.y);
    st.o[2 * r + 1] = make_float2(v.z, v.w);
    st.p[2 * r] = make_float2(w.x, w.y);
    st.p[2 * r + 1] = make_float2(w.z, w.w);
  }
}

template <int EW>
__device__ __forceinline__ void load_tables(Step<EW>& st, const float4* const (&Tt)[EW], int step, int lane) {
  const size_t ct = (size_t)step * 128 + lane;
#pragma unroll
  for (int e = 0; e < EW; ++e) {
    const float4 v = Tt[e][ct], w = Tt[e][ct + 64];
    st.t[e][0] = v.x; st.t[e][1] = v.y; st.t[e][2] = v.z; st.t[e][3] = v.w;
    st.t[e][4] = w.x; st.t[e][5] = w.y; st.t[e][6] = w.z; st.t[e][7] = w.w;
  }
}

template <int EW>
__device__ __forceinline__ void load_step(Step<EW>& st, const float4* __restrict__ Ot, const float4* __restrict__ Pt,
                                          const float4* const (&Tt)[EW], int step, int lane) {
  load_spectra<EW>(st, Ot, Pt, step, lane);
  load_tables<EW>(st, Tt, step, lane);
}

// One work item: image i, orientation slot, CTF group cg (EW CTF sets).
// Fs/Gs: the DFT fragments of this item's box, already in LDS.
// Load schedules of the stage-1 K loop.
constexpr int kLoadNext = 0;   // one register set, next step loaded once consumed
constexpr int kLoadPing = 1;   // two register sets in ping-pong
constexpr int kLoadNone = 2;   // each step loaded just before use

template <bool BF, int NT, int EW, int LM, bool PRIO = false>
__device__ __forceinline__ void split_item(const SplitArgs& sa, const uint4* __restrict__ Fs,
                                           const uint4* __restrict__ Gs, int item) {
  using P = Prec<BF>;
  using V = typename P::V;
  const LogpostArgs& a = sa.a;
  const int KS = sa.KS, MT = sa.MT;
  const int nx = a.nx, ny = a.ny, S = a.S, W = 2 * S + 1;
  const int mh = nx / 2 + 1, half = nx / 2, ldy = a.ldy;
  const size_t len = (size_t)mh * ldy;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int nslots = a.cand ? a.k : a.nq;
  const int ncg = sa.ncg;
  const int tile_items = sa.ti * sa.ts * ncg;
  const double n = (double)nx * ny, h = 0.5 * n;
  const float c2 = (float)(h - 1.0);
  const float c2l2e = c2 * 1.4426950408889634f;
  const bool series = c2 >= 1024.0f;
  const bool fr = li < 8;   // Fr (cos) column of a stage-1 tile; else Fi (sin)
  // epilogue constants: X = E - O on cosine lanes, E + O on sine lanes
  const float sgn = fr ? -1.0f : 1.0f;
  const bool ct_last_ok = (li & 7) <= S - 8 * (NT - 1);
  const bool ct0_ok = fr || (li & 7) != 0;
  const int lg4 = 4 * lg, wlast = W - 16 * (NT - 1);
  // -(n/2-1) log2(e) times the series of log1p: u - u^2/2 + u^3/3
  const float p1 = -c2l2e, p2 = 0.5f * c2l2e, p3 = -c2l2e / 3.0f;

  {
    const int tile = item / tile_items, rr = item - tile * tile_items;
    const int ti = tile / sa.n_ts, ts = tile - ti * sa.n_ts;
    const int cg = rr % ncg, pr = rr / ncg;
    const int i = ti * sa.ti + (sa.xcd ? pr % sa.ti : pr / sa.ts);
    const int slot = ts * sa.ts + (sa.xcd ? pr / sa.ti : pr % sa.ts);
    if (i >= a.ni || slot >= nslots) return;   // uniform across the wave
    const int q = a.cand ? a.cand[(size_t)i * a.k + slot] : slot;
    const float2* O = a.ispec + (size_t)i * len;
    const float2* Pq = a.pspec + (size_t)q * len;
    const size_t tlen = tile_spec_len(nx, ny), ttlen = tile_table_len(nx, ny);
    const float4* Ot = a.itile + (size_t)i * tlen;
    const float4* Pt = a.ptile + (size_t)q * tlen;
    const double A = a.istats[3 * i + 2];
    // X carries the operand scale 2^zs of the CTF values: kappa takes it off
    const int esc = 2 * (a.iexpo[i] + a.pexpo[q]) - 2 * a.zs;
    const int c0 = cg * EW;
    bioem_erec* out = a.rec + ((size_t)i * nslots + slot) * a.nc;

    if (!(A > 0.0)) {   // degenerate image: every evaluation is void
      if (lane < EW && c0 + lane < a.nc) out[c0 + lane] = bioem_erec{-1.0f, 0.0f, -1, 0};
    } else {
      f4 acc2[EW][NT][NT];
#pragma unroll
      for (int e = 0; e < EW; ++e)
#pragma unroll
        for (int x = 0; x < NT; ++x)
#pragma unroll
          for (int y = 0; y < NT; ++y) acc2[e][x][y] = f4{0.f, 0.f, 0.f, 0.f};

      // CTF tables of the group in fragment order (slots past nx/2 hold
      // zeros in every copy, so their products vanish)
      const float4* Tt[EW];
#pragma unroll
      for (int e = 0; e < EW; ++e) Tt[e] = a.ttile + (size_t)min(c0 + e, a.nc - 1) * ttlen;
      // with the in-place schedule the loaded step carries across m-tiles:
      // the first step of the next tile is in flight during stage 2
      Step<EW> st;
      if constexpr (LM == kLoadNext) load_step<EW>(st, Ot, Pt, Tt, 0, lane);
      for (int mt = 0; mt < MT; ++mt) {
        f4 acc1[EW][NT][2];
#pragma unroll
        for (int e = 0; e < EW; ++e)
#pragma unroll
          for (int x = 0; x < NT; ++x) acc1[e][x][0] = acc1[e][x][1] = f4{0.f, 0.f, 0.f, 0.f};
        const int st0 = mt * KS;             // flat index of the tile's first K-step
        const bool pk = mt == 0;             // slot 0 of this tile carries columns 0 and nx/2
        // prep: the K-step's conjugate products, CTF-weighted and split
        // into hi/lo operands (consumes the loaded step); mma: its products
        auto prep = [&](const Step<EW>& cur, int ks, V (&zrh)[EW], V (&zrl)[EW], V (&zih)[EW], V (&zil)[EW]) {
          const int l0 = 32 * ks + 8 * lg;
          float2 w0[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const float2 o = cur.o[r], p = cur.p[r];
            w0[r] = make_float2(o.x * p.x + o.y * p.y, o.x * p.y - o.y * p.x);
          }
          float zr[EW][8], zi[EW][8];
#pragma unroll
          for (int e = 0; e < EW; ++e)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              zr[e][r] = w0[r].x * cur.t[e][r];
              zi[e][r] = w0[r].y * cur.t[e][r];
            }
          if (pk) {
            if (li == 0) {
              if (l0 == 0) {   // Z(0,0) := 0
#pragma unroll
                for (int e = 0; e < EW; ++e) zr[e][0] = zi[e][0] = 0.f;
              }
              float2 o[8], p[8];
              load8c(O + (size_t)half * ldy, l0, o);
              load8c(Pq + (size_t)half * ldy, l0, p);
#pragma unroll
              for (int e = 0; e < EW; ++e) {
                float t[8];
                load8r(a.table + (size_t)min(c0 + e, a.nc - 1) * len + (size_t)half * ldy, l0, t);
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                  const float wr = o[r].x * p[r].x + o[r].y * p[r].y;
                  const float wi = o[r].x * p[r].y - o[r].y * p[r].x;
                  // Z0 + i Zn
                  zr[e][r] -= wi * t[r];
                  zi[e][r] += wr * t[r];
                }
              }
            }
          }
#pragma unroll
          for (int e = 0; e < EW; ++e) {
            split8<BF>(zr[e], zrh[e], zrl[e]);
            split8<BF>(zi[e], zih[e], zil[e]);
          }
        };
        auto mma = [&](int ks, const V (&zrh)[EW], const V (&zrl)[EW], const V (&zih)[EW], const V (&zil)[EW]) {
          // with two waves per SIMD, the wave in its matrix phase goes first
          // so the other wave's vector work fills the matrix pipe's cycles
          if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
          V fh[NT], fl[NT];
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            fh[ct] = __builtin_bit_cast(V, Fs[((ks * NT + ct) * 2 + 0) * 64 + lane]);
            fl[ct] = __builtin_bit_cast(V, Fs[((ks * NT + ct) * 2 + 1) * 64 + lane]);
          }
          // three split products, ordered so that no two consecutive MFMAs
          // update the same accumulator
#pragma unroll
          for (int e = 0; e < EW; ++e)
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
              acc1[e][ct][0] = P::mma(zrh[e], fh[ct], acc1[e][ct][0]);
              acc1[e][ct][1] = P::mma(zih[e], fh[ct], acc1[e][ct][1]);
            }
#pragma unroll
          for (int e = 0; e < EW; ++e)
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
              acc1[e][ct][0] = P::mma(zrh[e], fl[ct], acc1[e][ct][0]);
              acc1[e][ct][1] = P::mma(zih[e], fl[ct], acc1[e][ct][1]);
            }
#pragma unroll
          for (int e = 0; e < EW; ++e)
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
              acc1[e][ct][0] = P::mma(zrl[e], fh[ct], acc1[e][ct][0]);
              acc1[e][ct][1] = P::mma(zil[e], fh[ct], acc1[e][ct][1]);
            }
          if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        };
        auto body = [&](const Step<EW>& cur, int ks) {
          V zrh[EW], zrl[EW], zih[EW], zil[EW];
          prep(cur, ks, zrh, zrl, zih, zil);
          mma(ks, zrh, zrl, zih, zil);
        };
        if constexpr (LM == kLoadPing) {
          // two register sets in ping-pong: the loads of the next K-step are
          // in flight while this one computes, with no copies between sets
          Step<EW> sa0, sa1;
          load_step<EW>(sa0, Ot, Pt, Tt, st0, lane);
          for (int ks = 0; ks < KS; ks += 2) {
            if (ks + 1 < KS) load_step<EW>(sa1, Ot, Pt, Tt, st0 + ks + 1, lane);
            body(sa0, ks);
            if (ks + 1 < KS) {
              if (ks + 2 < KS) load_step<EW>(sa0, Ot, Pt, Tt, st0 + ks + 2, lane);
              body(sa1, ks + 1);
            }
          }
        } else if constexpr (LM == kLoadNone) {
          for (int ks = 0; ks < KS; ++ks) {
            Step<EW> st;
            load_step<EW>(st, Ot, Pt, Tt, st0 + ks, lane);
            body(st, ks);
          }
        } else {
          // one register set: once a step's loads are consumed by prep, the
          // same registers take the next step's loads, which stay in flight
          // during this step's matrix products
          for (int ks = 0; ks < KS; ++ks) {
            V zrh[EW], zrl[EW], zih[EW], zil[EW];
            prep(st, ks, zrh, zrl, zih, zil);
            // the next K-step in flat order (the next tile's first after the last)
            if (st0 + ks + 1 < MT * KS) load_step<EW>(st, Ot, Pt, Tt, st0 + ks + 1, lane);
            mma(ks, zrh, zrl, zih, zil);
          }
        }
        // stage 2: this m-tile is one K-step of the c2r GEMM
        V gh[NT], gl[NT];
#pragma unroll
        for (int dt = 0; dt < NT; ++dt) {
          gh[dt] = __builtin_bit_cast(V, Gs[((mt * NT + dt) * 2 + 0) * 64 + lane]);
          gl[dt] = __builtin_bit_cast(V, Gs[((mt * NT + dt) * 2 + 1) * 64 + lane]);
        }
        V bh[EW][NT], bl[EW][NT];
#pragma unroll
        for (int e = 0; e < EW; ++e)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            float b[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float re = acc1[e][ct][0][r], im = acc1[e][ct][1][r];
              b[r] = fr ? re : im;
              b[4 + r] = fr ? im : -re;
            }
            split8<BF>(b, bh[e][ct], bl[e][ct]);
          }
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int e = 0; e < EW; ++e)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int dt = 0; dt < NT; ++dt) acc2[e][dt][ct] = P::mma(gh[dt], bh[e][ct], acc2[e][dt][ct]);
#pragma unroll
        for (int e = 0; e < EW; ++e)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int dt = 0; dt < NT; ++dt) acc2[e][dt][ct] = P::mma(gh[dt], bl[e][ct], acc2[e][dt][ct]);
#pragma unroll
        for (int e = 0; e < EW; ++e)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int dt = 0; dt < NT; ++dt) acc2[e][dt][ct] = P::mma(gl[dt], bh[e][ct], acc2[e][dt][ct]);
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
      }

      // shift-window epilogue per CTF set of the group (FP32; the FP64
      // likelihood terms are added at finalisation)
#pragma unroll
      for (int e = 0; e < EW; ++e) {
        const int c = c0 + e;
        if (c >= a.nc) continue;   // uniform
        const double B = a.B[(size_t)q * a.nc + c];
        if (!(B > 0.0)) {
          if (lane == 0) out[c] = bioem_erec{-1.0f, 0.0f, -1, 0};
          continue;
        }
        // Pass 1: X = E -+ O from the partner lane, squared in place; only
        // the last column tile (dy' > S), the dy' = 0 sine column and the
        // last dx tile (dx > S) hold slots outside the window.
        float x2max = 0.0f;
#pragma unroll
        for (int dt = 0; dt < NT; ++dt)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float mine = acc2[e][dt][ct][r];
              const float X = fmaf(sgn, lane_xor8(mine), mine);
              float x2 = X * X;
              bool ok = true;
              if (ct == NT - 1) ok = ok && ct_last_ok;
              if (ct == 0) ok = ok && ct0_ok;
              if (dt == NT - 1) ok = ok && (lg4 + r < wlast);
              if (ct == NT - 1 || ct == 0 || dt == NT - 1) x2 = ok ? x2 : -1.0f;
              acc2[e][dt][ct][r] = x2;
              x2max = fmaxf(x2max, x2);
            }
        const float wmax = wave_max_f(x2max);
        const double kappa = ldexp(a.kscale / (A * B), esc);
        const double rho2 = fmin((double)wmax * kappa, 1.0 - 0x1p-52);
        const float cu = (float)(kappa / (1.0 - rho2));
        // Pass 2: sum of (1 + u)^-(n/2-1) over the window, u = (max X^2 - X^2) c_u
        // (exactly 0 at the maximum: no rounding of max X^2 c_u enters every term).
        float sum = 0.0f;
        if (series) {
#pragma unroll
          for (int k = 0; k < NT * NT * 4; ++k) {
            const float x2 = acc2[e][k / (4 * NT)][(k / 4) % NT][k % 4];
            const float u = fminf((wmax - x2) * cu, 0.05f);
            // slots outside the window are marked x2 = -1 and left out
            const float t = __builtin_amdgcn_exp2f(u * (p1 + u * (p2 + u * p3)));
            sum += x2 >= 0.0f ? t : 0.0f;
          }
        } else {
#pragma unroll
          for (int k = 0; k < NT * NT * 4; ++k) {
            const float x2 = acc2[e][k / (4 * NT)][(k / 4) % NT][k % 4];
            const float u = (wmax - x2) * cu;
            const float t = __expf(-c2 * log1p_acc(u));
            sum += x2 >= 0.0f ? t : 0.0f;
          }
        }
        const float tot = wave_sum_f(sum);
        if (lane == 0) out[c] = bioem_erec{ldexpf(wmax, -2 * a.zs), tot, -1, 0};   // max X^2 without the scale
      }
    }
  }
}

template <bool BF, int NT, int EW, int WAVES, int LM, bool XCD, bool PRIO>
__global__ __launch_bounds__(64 * WAVES, 1) void k_logpost_split(SplitArgs sa) {
  extern __shared__ uint4 lds[];
  const int nF = sa.KS * NT * 2 * 64, nG = sa.MT * NT * 2 * 64;
  for (int e = threadIdx.x; e < nF + nG; e += 64 * WAVES) lds[e] = e < nF ? sa.F[e] : sa.G[e - nF];
  __syncthreads();
  const int n_items = sa.n_ti * sa.n_ts * sa.ti * sa.ts * sa.ncg;
  if constexpr (XCD) {
    // Workgroups are dealt to the 8 XCDs round-robin (each with its own L2):
    // XCD x takes tiles x, x + 8, ... and its waves sweep one tile together,
    // images fastest, so the tile's images stay in that L2 while its
    // orientations stream through.
    const int kx = min(8, (int)gridDim.x);   // groups present (every one has a workgroup)
    const int x = blockIdx.x % kx;
    const int nwg = (gridDim.x - x + kx - 1) / kx;
    const int lw = (blockIdx.x / kx) * WAVES + (threadIdx.x >> 6), nw = nwg * WAVES;
    const int tile_items = sa.ti * sa.ts * sa.ncg, n_tiles = sa.n_ti * sa.n_ts;
    for (int t = x; t < n_tiles; t += kx)
      for (int r = lw; r < tile_items; r += nw) split_item<BF, NT, EW, LM, PRIO>(sa, lds, lds + nF, t * tile_items + r);
  } else {
    const int wave = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * WAVES;
    for (int item = wave; item < n_items; item += nwaves) split_item<BF, NT, EW, LM, PRIO>(sa, lds, lds + nF, item);
  }
}

// Persistent form over several jobs (boxes, shift windows, grids) in one
// launch.  The work list is the concatenation of every job's items in blocks
// of WAVES consecutive items; workgroup b takes blocks b, b + G, b + 2G, ...
// so all workgroups sweep the jobs together (the spectra of the current
// tiles stay shared in the caches) and each receives a near-equal share of
// every job.  A workgroup reloads the DFT fragments into LDS when it moves
// on to the next job.
struct JobDesc {
  SplitArgs sa;
  int nt, ew;
  int block0;   // first work block of the job
};

template <bool BF, int EW, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 1) void k_logpost_batch(const JobDesc* __restrict__ jobs, int njobs,
                                                                 int total_blocks) {
  extern __shared__ uint4 lds[];
  int cur = -1, nF = 0;
  for (int blk = blockIdx.x; blk < total_blocks; blk += gridDim.x) {
    int j = cur < 0 ? 0 : cur;   // blocks only increase, so the job index only advances
    while (j + 1 < njobs && jobs[j + 1].block0 <= blk) ++j;
    const JobDesc& jd = jobs[j];
    if (j != cur) {
      nF = jd.sa.KS * jd.nt * 128;
      const int nG = jd.sa.MT * jd.nt * 128;
      __syncthreads();   // every wave is done with the previous job's fragments
      for (int e = threadIdx.x; e < nF + nG; e += 64 * WAVES) lds[e] = e < nF ? jd.sa.F[e] : jd.sa.G[e - nF];
      __syncthreads();
      cur = j;
    }
    const int item = (blk - jd.block0) * WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the job's arguments as a value (scalar registers), not re-read from the table
    const SplitArgs sa = jd.sa;
    // two waves per SIMD: each K-step loaded just before use, the matrix
    // phase at raised priority (as the default single-job variant)
    constexpr int LM = kLoadNone;
    switch (jd.nt) {   // uniform across the workgroup
      case 1: split_item<BF, 1, EW, LM, true>(sa, lds, lds + nF, item); break;
      case 2: split_item<BF, 2, EW, LM, true>(sa, lds, lds + nF, item); break;
      default: split_item<BF, 3, EW, LM, true>(sa, lds, lds + nF, item); break;
    }
  }
}

// Fragment tables of the two DFT matrices, split into hi/lo parts.
template <bool BF>
__global__ void k_split_tables(int nx, int ny, int S, int NT, int KS, int MT, uint4* __restrict__ F,
                               uint4* __restrict__ G) {
  const int nF = KS * NT * 2 * 64, nG = MT * NT * 2 * 64;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nF + nG) return;
  const int W = 2 * S + 1, half = nx / 2;
  float val[8];
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
      val[r] = (float)x;
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
      val[r] = (float)x;
    }
  }
  uint32_t hi[4], lo[4];
  for (int r = 0; r < 4; ++r) Prec<BF>::split2(val[2 * r], val[2 * r + 1], hi[r], lo[r]);
  const uint4 out = hl == 0 ? make_uint4(hi[0], hi[1], hi[2], hi[3]) : make_uint4(lo[0], lo[1], lo[2], lo[3]);
  (idx < nF ? F[idx] : G[idx - nF]) = out;
}

int nt_for(int S) { return (S + 8) / 8; }   // ceil((S+1)/8) column tiles == ceil((2S+1)/16) dx tiles

size_t split_smem(int nx, int ny, int S) {
  const int NT = nt_for(S);
  const int KS = (ny + 31) / 32, MT = (nx / 2 + 15) / 16;
  return (size_t)(KS + MT) * NT * 2 * 64 * sizeof(uint4);
}

// Launch shapes of the split kernel: CTF sets per wave item, waves per
// workgroup (4 = one wave per SIMD with up to 512 registers, 8 = two per SIMD
// with up to 256) and the load schedule of the K loop.
struct Shape {
  int ew, waves, lm, xcd;
};
constexpr Shape kShapes[] = {{2, 4, kLoadPing, 0}, {2, 8, kLoadNone, 0}, {1, 8, kLoadNext, 0},
                             {4, 4, kLoadNext, 0}, {2, 4, kLoadNext, 0}, {4, 4, kLoadNone, 0},
                             {2, 4, kLoadNone, 0}, {4, 4, kLoadNext, 1}, {2, 4, kLoadNext, 1},
                             {2, 8, kLoadNext, 0}, {2, 8, kLoadNone, 1}, {2, 8, kLoadNone, 0}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

template <bool BF, int NT, int EW, int WAVES, int LM, bool XCD = false, bool PRIO = false>
hipError_t launch_shape(hipStream_t s, const SplitArgs& sa, size_t smem, int ncu) {
  auto kern = k_logpost_split<BF, NT, EW, WAVES, LM, XCD, PRIO>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const long n_items = (long)sa.n_ti * sa.n_ts * sa.ti * sa.ts * sa.ncg;
  const long want = (n_items + WAVES - 1) / WAVES;
  const int grid = (int)std::min<long>(want, (long)ncu);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WAVES), smem, s, sa);
  return hipGetLastError();
}

template <bool BF, int NT>
hipError_t launch_nt(hipStream_t s, const SplitArgs& sa, size_t smem, int ncu, int shape) {
  switch (shape) {
    case 0: return launch_shape<BF, NT, 2, 4, kLoadPing>(s, sa, smem, ncu);
    case 1: return launch_shape<BF, NT, 2, 8, kLoadNone>(s, sa, smem, ncu);
    case 2: return launch_shape<BF, NT, 1, 8, kLoadNext>(s, sa, smem, ncu);
    case 3: return launch_shape<BF, NT, 4, 4, kLoadNext>(s, sa, smem, ncu);
    case 4: return launch_shape<BF, NT, 2, 4, kLoadNext>(s, sa, smem, ncu);
    case 5: return launch_shape<BF, NT, 4, 4, kLoadNone>(s, sa, smem, ncu);
    case 6: return launch_shape<BF, NT, 2, 4, kLoadNone>(s, sa, smem, ncu);
    case 7: return launch_shape<BF, NT, 4, 4, kLoadNext, true>(s, sa, smem, ncu);
    case 8: return launch_shape<BF, NT, 2, 4, kLoadNext, true>(s, sa, smem, ncu);
    case 9: return launch_shape<BF, NT, 2, 8, kLoadNext>(s, sa, smem, ncu);
    case 10: return launch_shape<BF, NT, 2, 8, kLoadNone, true>(s, sa, smem, ncu);
    default: return launch_shape<BF, NT, 2, 8, kLoadNone, false, true>(s, sa, smem, ncu);
  }
}

}  // namespace

bool split_supported(int nx, int ny, int S) {
  const int NT = nt_for(S);
  return NT >= 1 && NT <= 3 && split_smem(nx, ny, S) <= kMaxSmem;
}

int split_num_shapes() { return kNumShapes; }

static int split_ctf_groups(int nc, int ew) { return (nc + ew - 1) / ew; }

static int device_cus() {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  return ncu;
}

// Fragment tables (stream-ordered allocation, freed by the caller with
// hipFreeAsync) and the argument block of one job.
static hipError_t make_split_args(hipStream_t s, const LogpostArgs& a, bool bf16, int ew, int ti, int ts,
                                  SplitArgs& sa, uint4*& tabs) {
  const int NT = nt_for(a.S);
  const int KS = (a.ny + 31) / 32, MT = (a.nx / 2 + 15) / 16;
  const int nF = KS * NT * 2 * 64, nG = MT * NT * 2 * 64;
  tabs = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&tabs), sizeof(uint4) * (nF + nG), s);
  if (e != hipSuccess) return e;
  const int nt = nF + nG;
  if (bf16)
    hipLaunchKernelGGL(k_split_tables<true>, dim3((nt + 255) / 256), dim3(256), 0, s, a.nx, a.ny, a.S, NT, KS, MT,
                       tabs, tabs + nF);
  else
    hipLaunchKernelGGL(k_split_tables<false>, dim3((nt + 255) / 256), dim3(256), 0, s, a.nx, a.ny, a.S, NT, KS, MT,
                       tabs, tabs + nF);
  sa = SplitArgs{};
  sa.a = a;
  sa.F = tabs;
  sa.G = tabs + nF;
  sa.KS = KS;
  sa.MT = MT;
  sa.ncg = split_ctf_groups(a.nc, ew);
  const int nslots = a.cand ? a.k : a.nq;
  sa.ti = ti > 0 ? ti : kTileImages;
  sa.ts = ts > 0 ? ts : kTileSlots;
  sa.n_ti = (a.ni + sa.ti - 1) / sa.ti;
  sa.n_ts = (nslots + sa.ts - 1) / sa.ts;
  return hipGetLastError();
}

hipError_t launch_logpost_split(hipStream_t s, const LogpostArgs& a, bool bf16, int shape, int ti, int ts) {
  if (shape < 0 || shape >= kNumShapes) return hipErrorInvalidValue;
  SplitArgs sa;
  uint4* tabs = nullptr;
  hipError_t e = make_split_args(s, a, bf16, kShapes[shape].ew, ti, ts, sa, tabs);
  sa.xcd = kShapes[shape].xcd;
  if (e == hipSuccess) {
    const int NT = nt_for(a.S), ncu = device_cus();
    const size_t smem = split_smem(a.nx, a.ny, a.S);
    if (NT == 1) e = bf16 ? launch_nt<true, 1>(s, sa, smem, ncu, shape) : launch_nt<false, 1>(s, sa, smem, ncu, shape);
    else if (NT == 2) e = bf16 ? launch_nt<true, 2>(s, sa, smem, ncu, shape) : launch_nt<false, 2>(s, sa, smem, ncu, shape);
    else e = bf16 ? launch_nt<true, 3>(s, sa, smem, ncu, shape) : launch_nt<false, 3>(s, sa, smem, ncu, shape);
  }
  const hipError_t f = tabs ? hipFreeAsync(tabs, s) : hipSuccess;
  return e != hipSuccess ? e : f;
}

int split_shape_for_ew(int ew, bool bf16) {
  // two CTF sets: two waves per SIMD (the other wave covers load latency),
  // the wave in its matrix phase at raised priority; four: one wave per
  // SIMD with every register, where the bf16 split spills under next-step
  // loads
  if (ew == 2) return 11;
  return bf16 ? 5 : 3;
}

int split_shape_ew(int shape) { return shape >= 0 && shape < kNumShapes ? kShapes[shape].ew : 4; }

hipError_t launch_logpost_batch(hipStream_t s, const BatchJob* jobs, int njobs, bool bf16) {
  constexpr int kWaves = 8;     // two waves per SIMD, as the default single-job variant
  constexpr int kBatchEW = 2;
  if (njobs < 1) return hipErrorInvalidValue;
  // The work list takes the jobs with the costliest items first: with the
  // cheap ones first the launch measured up to a quarter slower than one
  // launch per job, with the costly ones first within 2%.  The order of the
  // list does not change any job's results.
  std::vector<int> order(njobs);
  for (int j = 0; j < njobs; ++j) order[j] = j;
  auto cost = [&](int j) { return (long)jobs[j].a.nx * jobs[j].a.ny * (2 * jobs[j].a.S + 1); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<JobDesc> desc(njobs);
  std::vector<uint4*> tabs(njobs, nullptr);
  hipError_t e = hipSuccess;
  long blocks = 0;
  size_t smem = 0;
  for (int k = 0; k < njobs && e == hipSuccess; ++k) {
    const int j = order[k];
    const int ew = kBatchEW;   // one item width for the whole launch
    e = make_split_args(s, jobs[j].a, bf16, ew, jobs[j].ti, jobs[j].ts, desc[k].sa, tabs[k]);
    desc[k].nt = nt_for(jobs[j].a.S);
    desc[k].ew = ew;
    desc[k].block0 = (int)blocks;
    const SplitArgs& sa = desc[k].sa;
    const long items = (long)sa.n_ti * sa.n_ts * sa.ti * sa.ts * sa.ncg;
    blocks += (items + kWaves - 1) / kWaves;
    smem = std::max(smem, split_smem(jobs[j].a.nx, jobs[j].a.ny, jobs[j].a.S));
  }
  JobDesc* djobs = nullptr;
  if (e == hipSuccess && blocks > 0x7fffffffL) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&djobs), sizeof(JobDesc) * njobs, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(djobs, desc.data(), sizeof(JobDesc) * njobs, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    auto kern = bf16 ? k_logpost_batch<true, kBatchEW, kWaves> : k_logpost_batch<false, kBatchEW, kWaves>;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)smem);
    if (e == hipSuccess) {
      const int grid = (int)std::min<long>(blocks, (long)device_cus());
      hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kWaves), smem, s, djobs, njobs, (int)blocks);
      e = hipGetLastError();
    }
  }
  // the host descriptor copy must not be reused before the copy has run
  const hipError_t sy = hipStreamSynchronize(s);
  if (djobs) (void)hipFreeAsync(djobs, s);
  for (uint4* t : tabs)
    if (t) (void)hipFreeAsync(t, s);
  return e != hipSuccess ? e : sy;
}

}  // namespace bioem
