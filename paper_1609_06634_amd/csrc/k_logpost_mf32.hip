// Plain FP32 posterior kernel on the FP32 matrix cores (v_mfma_f32_16x16x4f32:
// FP32 operands, FP32 accumulation).
//
// The pruned inverse transform of Eq. (fourier_explicit) over the shift window
// |dx|, |dy| <= S is factored so that each matrix product works on a quarter
// of a spectrum column instead of all of it (the paper notes that only the
// window's coefficients are needed, Section 3, Margin for improvements):
//
// Stage 1 (along y, length N = ny, every spectrum column).  Split the window
// rows k by parity (one radix-2 step), then pair l with H - l (H = N/2):
//   z0(l) = Z(l) + Z(l+H),  z1(l) = Z(l) - Z(l+H),   l in [0, H)
//   u0 = z0(j) + z0(H-j), v0 = z0(j) - z0(H-j)      (even k)
//   u1 = z1(j) - z1(H-j), v1 = z1(j) + z1(H-j)      (odd k)
//   Y(+-k) = U(k) +- i V(k),  U = sum_j u cos(2 pi j k/N),  V = sum_j v sin(..)
// for j in [1, ceil(N/4) - 1]; each of the four blocks (u0, v0, u1, v1) is a
// real-coefficient product over about N/4 points with at most 16 output rows
// (k = 2p or 2p+1, p < 16, so S <= 31).  The points 0, H (and N/4, 3N/4 when
// 4 | N) share one slot: Z(0) +- Z(H) enter U with weight 1, Z(N/4) - Z(3N/4)
// enters V of the odd rows with sign (-1)^p, and Z(N/4) + Z(3N/4) is added to
// U of the even rows with sign (-1)^p after the products.
//
// Stage 2 (c2r along x, half spectrum m in [0, M], M = nx/2), split by the
// parity of dx and paired m <-> M - m, using Y(k, -m) = conj(Y(k, m)):
//   a(m) = Y(m) + conj(Y(M-m)),  b(m) = Y(m) - conj(Y(M-m))
//   X(+-2u)      = a(0) + sum_m 2 [Re a cos(4 pi m u/nx) -+ Im a sin(..)]
//   X(+-(2u+1))  = b(0) + sum_m 2 [Re b cos(2 pi m (2u+1)/nx) -+ Im b sin(..)]
// with the self-paired column M/2 weighted 1/2.  Columns 0 and M are Hermitian
// along y (their Y are real), so they share one slot as Z(l,0) + i Z(l,M).
// Every term is linear in the stage-1 outputs (Re U, Im U, Re V, Im V), so the
// stage-1 accumulators feed the stage-2 products directly as operands: the
// 16x16x4 accumulator layout (lane = column, 4 rows per lane) is the operand
// layout of the next product with the 4 rows as its K index.
//
// Work per evaluation at 224^2, S = 20: 784 stage-1 and 224 stage-2 products
// (16x16x4), against 3600 for the unfactored real-coefficient transform.
//
// Inputs are orbit-order copies: for each (half group h, K-step, lane) the
// four values Z(j), Z(H-j), Z(H+j), Z(N-j) of the lane's column, for the
// projections (one copy per orientation) and for the products
// conj(F I_o) x CTF x Env (one copy per image and CTF set, DC set to zero),
// so Z is one complex product per value and each wave load is 2 KB in one
// piece.  The shift-window epilogue is the one of the split-precision kernel:
// window maximum of X^2 and the FP32 sum of (1 + u)^-(n/2-1) relative to it;
// the FP64 likelihood terms are added at finalisation.
#include <algorithm>

#include "common.hpp"

namespace bioem {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

struct MfGeom {
  int nx, ny, H, hasQ, Q, J1, KS1, Mx, hasQx, Qx, nreg, nHG;
};

__host__ __device__ inline MfGeom mf_geom(int nx, int ny) {
  MfGeom G;
  G.nx = nx; G.ny = ny;
  G.H = ny / 2;
  G.hasQ = ny % 4 == 0;
  G.Q = ny / 4;
  G.J1 = G.hasQ ? ny / 4 - 1 : (ny - 2) / 4;
  G.KS1 = (G.J1 + 1 + 3) / 4;
  G.Mx = nx / 2;
  G.hasQx = nx % 4 == 0;
  G.Qx = nx / 4;
  G.nreg = G.hasQx ? G.Mx / 2 - 1 : (G.Mx - 1) / 2;
  G.nHG = (1 + G.nreg + 7) / 8;
  return G;
}

__host__ __device__ inline size_t mf_main_len(const MfGeom& G) { return (size_t)G.nHG * G.KS1 * 128; }
// float4 per item of an orbit-order copy: the main part and the packed slot's
// second column [KS1][4][2]
__host__ __device__ inline size_t mf_item_len(const MfGeom& G) { return mf_main_len(G) + (size_t)G.KS1 * 8; }

// Column of data row p of half group h: -2 the packed slot (columns 0 and M),
// -1 none, else the column m.
__device__ inline int mf_col(const MfGeom& G, int h, int p) {
  const int u = 8 * h + (p >> 1), mu = p & 1;
  if (u == 0) return mu == 0 ? -2 : (G.hasQx ? G.Qx : -1);
  if (u <= G.nreg) return mu == 0 ? u : G.Mx - u;
  return -1;
}

// Row l of element e of orbit slot j (-1 none).
__device__ inline int mf_row(const MfGeom& G, int j, int e) {
  if (j == 0) {
    if (e == 0) return 0;
    if (e == 2) return G.H;
    if (!G.hasQ) return -1;
    return e == 1 ? G.Q : 3 * G.Q;
  }
  if (j > G.J1) return -1;
  switch (e) {
    case 0: return j;
    case 1: return G.H - j;
    case 2: return G.H + j;
    default: return G.ny - j;
  }
}

// Element (col, row) of an orbit-order copy: (item, index w within the item)
// -> column and the two rows of the float4 at w (-1 none).
__device__ inline void mf_where(const MfGeom& G, int w, int& col, int& r0, int& r1) {
  const int ml = (int)mf_main_len(G);
  int j, half;
  if (w < ml) {
    half = w & 1;
    const int lane = (w >> 1) & 63, step = w >> 7;
    const int h = step / G.KS1, s1 = step - h * G.KS1;
    col = mf_col(G, h, lane & 15);
    j = 4 * s1 + (lane >> 4);
    if (col == -2) col = 0;
  } else {
    const int w2 = w - ml;
    half = w2 & 1;
    const int g = (w2 >> 1) & 3, s1 = w2 >> 3;
    col = G.Mx;   // second column of the packed slot
    j = 4 * s1 + g;
  }
  r0 = col < 0 ? -1 : mf_row(G, j, 2 * half);
  r1 = col < 0 ? -1 : mf_row(G, j, 2 * half + 1);
}

__global__ __launch_bounds__(256) void k_mf_copy_spec(const float2* __restrict__ spec, long total, int nx, int ny,
                                                      float4* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const MfGeom G = mf_geom(nx, ny);
  const long per = (long)mf_item_len(G);
  const long item = idx / per;
  int col, r0, r1;
  mf_where(G, (int)(idx - item * per), col, r0, r1);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (col >= 0) {
    const float2* c = spec + (size_t)item * (nx / 2 + 1) * spec_ld(ny) + (size_t)col * spec_ld(ny);
    if (r0 >= 0) { v.x = c[r0].x; v.y = c[r0].y; }
    if (r1 >= 0) { v.z = c[r1].x; v.w = c[r1].y; }
  }
  out[idx] = v;
}

// conj(F I_o) x CTF table for images [0, ni) x CTF sets [0, nc), item i * nc + c;
// the (0, 0) coefficient is set to zero (the offset mu is integrated out).
__global__ __launch_bounds__(256) void k_mf_copy_at(const float2* __restrict__ ispec, const float* __restrict__ table,
                                                    long total, int nc, int nx, int ny, float4* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const MfGeom G = mf_geom(nx, ny);
  const long per = (long)mf_item_len(G);
  const long item = idx / per;
  const long i = item / nc, c = item - i * nc;
  int col, r0, r1;
  mf_where(G, (int)(idx - item * per), col, r0, r1);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (col >= 0) {
    const size_t ld = spec_ld(ny), clen = (size_t)(nx / 2 + 1) * ld;
    const float2* o = ispec + (size_t)i * clen + (size_t)col * ld;
    const float* t = table + (size_t)c * clen + (size_t)col * ld;
    if (r0 >= 0 && !(col == 0 && r0 == 0)) { v.x = o[r0].x * t[r0]; v.y = -o[r0].y * t[r0]; }
    if (r1 >= 0 && !(col == 0 && r1 == 0)) { v.z = o[r1].x * t[r1]; v.w = -o[r1].y * t[r1]; }
  }
  out[idx] = v;
}

// Matrix-core operand tables, built in FP64 and rounded once:
//   F1[step][lane] = (u0, v0, u1, v1) coefficients of slot j = 4 step + lane/16
//                    for output row p = lane % 16 (k = 2p, 2p, 2p+1, 2p+1);
//   F2[h][h2][lane] = (Ea, Oa, Eb, Ob) coefficients of pair 8h + 2(lane/16) + h2
//                    for output row r = lane % 16 (dx = 2r or 2r+1).
__global__ __launch_bounds__(256) void k_mf_tables(int nx, int ny, int S, float4* __restrict__ F1,
                                                   float4* __restrict__ F2) {
  const MfGeom G = mf_geom(nx, ny);
  const int n1 = G.KS1 * 64, n2 = G.nHG * 128;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n1 + n2) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (idx < n1) {
    const int lane = idx & 63, s1 = idx >> 6;
    const int p = lane & 15, j = 4 * s1 + (lane >> 4);
    const int k0 = 2 * p, k1 = 2 * p + 1;
    if (j == 0) {
      v[0] = k0 <= S ? 1.0 : 0.0;
      v[2] = k1 <= S ? 1.0 : 0.0;
      v[3] = (G.hasQ && k1 <= S) ? ((p & 1) ? -1.0 : 1.0) : 0.0;
    } else if (j <= G.J1) {
      if (k0 <= S) {
        const double2 t = twiddle64(((long)j * k0) % ny, ny);
        v[0] = t.x; v[1] = t.y;
      }
      if (k1 <= S) {
        const double2 t = twiddle64(((long)j * k1) % ny, ny);
        v[2] = t.x; v[3] = t.y;
      }
    }
    F1[idx] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  } else {
    const int w = idx - n1;
    const int lane = w & 63, h2 = (w >> 6) & 1, h = w >> 7;
    const int r = lane & 15, u = 8 * h + 2 * (lane >> 4) + h2;
    const bool ea = 2 * r <= S, eb = 2 * r + 1 <= S;
    if (u == 0) {
      if (G.hasQx && ea) v[0] = 2.0 * twiddle64(((long)2 * G.Qx * r) % nx, nx).x;
      v[2] = eb ? 1.0 : 0.0;
      if (G.hasQx && eb) v[3] = 2.0 * twiddle64(((long)G.Qx * (2 * r + 1)) % nx, nx).y;
    } else if (u <= G.nreg) {
      if (ea) {
        const double2 t = twiddle64(((long)2 * u * r) % nx, nx);
        v[0] = 2.0 * t.x; v[1] = 2.0 * t.y;
      }
      if (eb) {
        const double2 t = twiddle64(((long)u * (2 * r + 1)) % nx, nx);
        v[2] = 2.0 * t.x; v[3] = 2.0 * t.y;
      }
    }
    F2[w] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  }
}

struct MfArgs {
  LogpostArgs a;
  const float4* at;   // [ni][nc][len] image x CTF products (chunk-relative images)
  const float4* pm;   // [nq][len] projections
  const float4* F1;   // [KS1][64]
  const float4* F2;   // [nHG][2][64]
  int KS1, nHG;
  long len;           // float4 per item
  int ti, ts, n_ti, n_ts;   // item tile: images x orientation slots
};

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float2 cmul(float ar, float ai, float br, float bi) {
  return make_float2(fmaf(ar, br, -ai * bi), fmaf(ar, bi, ai * br));
}

__device__ __forceinline__ float wmax_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ float wsum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// log(1 + u) for u >= 0 with relative accuracy near FP32 epsilon.
__device__ __forceinline__ float log1p_f(float u) {
  const float w = 1.0f + u;
  const float d = w - 1.0f;
  return d == 0.0f ? u : __logf(w) * (u / d);
}

struct Step {
  float4 a0, a1, p0, p1;
};

__device__ __forceinline__ void load_step(Step& st, const float4* __restrict__ A, const float4* __restrict__ P,
                                          int t, int lane) {
  const size_t o = ((size_t)t * 64 + lane) * 2;
  st.a0 = A[o];
  st.a1 = A[o + 1];
  st.p0 = P[o];
  st.p1 = P[o + 1];
}

// One evaluation (image i, orientation slot, CTF set c) by one wave.
__device__ __forceinline__ void mf_item(const MfArgs& ma, const float4* __restrict__ F1s,
                                        const float4* __restrict__ F2s, int item) {
  const LogpostArgs& a = ma.a;
  const int lane = threadIdx.x & 63, p = lane & 15, g = lane >> 4;
  const int nslots = a.cand ? a.k : a.nq, nc = a.nc;
  const int tile_items = ma.ti * ma.ts * nc;
  const int tile = item / tile_items, rr = item - tile * tile_items;
  const int ti = tile / ma.n_ts, ts = tile - ti * ma.n_ts;
  const int c = rr % nc, pr = rr / nc;
  const int i = ti * ma.ti + pr / ma.ts;
  const int slot = ts * ma.ts + pr % ma.ts;
  if (i >= a.ni || slot >= nslots) return;   // uniform across the wave
  const int q = a.cand ? a.cand[(size_t)i * a.k + slot] : slot;
  bioem_erec* out = a.rec + ((size_t)i * nslots + slot) * nc + c;
  const double A = a.istats[3 * i + 2];
  const double B = a.B[(size_t)q * nc + c];
  if (!(A > 0.0) || !(B > 0.0)) {   // degenerate image or projection: void evaluation
    if (lane == 0) *out = bioem_erec{-1.0f, 0.0f, -1, 0};
    return;
  }
  const int S = a.S;
  const int KS1 = ma.KS1, nHG = ma.nHG, nsteps = KS1 * nHG;
  const float4* Ab = ma.at + ((size_t)i * nc + c) * ma.len;
  const float4* Pb = ma.pm + (size_t)q * ma.len;
  const size_t side = (size_t)nHG * KS1 * 128;

  f4 d2[2][8];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 8; ++t) d2[s][t] = f4{0.f, 0.f, 0.f, 0.f};

  Step cur;
  load_step(cur, Ab, Pb, 0, lane);
  for (int h = 0; h < nHG; ++h) {
    f4 d1[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int b = 0; b < 4; ++b) d1[t][b] = f4{0.f, 0.f, 0.f, 0.f};
    float cre = 0.f, cim = 0.f;   // Z(N/4) + Z(3N/4) of this lane's column (slot 0)
    for (int s1 = 0; s1 < KS1; ++s1) {
      const int t = h * KS1 + s1;
      Step nxt;
      if (t + 1 < nsteps) load_step(nxt, Ab, Pb, t + 1, lane);
      float2 e0 = cmul(cur.a0.x, cur.a0.y, cur.p0.x, cur.p0.y);
      float2 e1 = cmul(cur.a0.z, cur.a0.w, cur.p0.z, cur.p0.w);
      float2 e2 = cmul(cur.a1.x, cur.a1.y, cur.p1.x, cur.p1.y);
      float2 e3 = cmul(cur.a1.z, cur.a1.w, cur.p1.z, cur.p1.w);
      if (h == 0) {      // uniform
        if (p == 0) {    // packed slot: + i Z(l, M)
          const size_t o = side + ((size_t)s1 * 4 + g) * 2;
          const float4 sa0 = Ab[o], sa1 = Ab[o + 1], sp0 = Pb[o], sp1 = Pb[o + 1];
          const float2 f0 = cmul(sa0.x, sa0.y, sp0.x, sp0.y);
          const float2 f1 = cmul(sa0.z, sa0.w, sp0.z, sp0.w);
          const float2 f2 = cmul(sa1.x, sa1.y, sp1.x, sp1.y);
          const float2 f3 = cmul(sa1.z, sa1.w, sp1.z, sp1.w);
          e0.x -= f0.y; e0.y += f0.x;
          e1.x -= f1.y; e1.y += f1.x;
          e2.x -= f2.y; e2.y += f2.x;
          e3.x -= f3.y; e3.y += f3.x;
        }
      }
      const float z0ar = e0.x + e2.x, z0ai = e0.y + e2.y, z1ar = e0.x - e2.x, z1ai = e0.y - e2.y;
      const float z0br = e1.x + e3.x, z0bi = e1.y + e3.y, z1br = e1.x - e3.x, z1bi = e1.y - e3.y;
      float u0r = z0ar + z0br, u0i = z0ai + z0bi, v0r = z0ar - z0br, v0i = z0ai - z0bi;
      float u1r = z1ar - z1br, u1i = z1ai - z1bi, v1r = z1ar + z1br, v1i = z1ai + z1bi;
      if (s1 == 0) {   // uniform: slot 0 (lanes g = 0) holds the points 0, N/4, H, 3N/4
        if (g == 0) {
          u0r = z0ar; u0i = z0ai;
          v0r = 0.f; v0i = 0.f;
          u1r = z1ar; u1i = z1ai;
          v1r = z1br; v1i = z1bi;
          cre = z0br; cim = z0bi;
        }
      }
      const float4 Bf = F1s[s1 * 64 + lane];
      d1[0][0] = mma(u0r, Bf.x, d1[0][0]);
      d1[1][0] = mma(u0i, Bf.x, d1[1][0]);
      d1[0][1] = mma(v0r, Bf.y, d1[0][1]);
      d1[1][1] = mma(v0i, Bf.y, d1[1][1]);
      d1[0][2] = mma(u1r, Bf.z, d1[0][2]);
      d1[1][2] = mma(u1i, Bf.z, d1[1][2]);
      d1[0][3] = mma(v1r, Bf.w, d1[0][3]);
      d1[1][3] = mma(v1i, Bf.w, d1[1][3]);
      if (t + 1 < nsteps) cur = nxt;
    }
    // even rows: + (-1)^p (Z(N/4) + Z(3N/4)) of each column (slot 0, lane = data row)
    {
      const float sg = (p & 1) ? -1.0f : 1.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float xr = __shfl(cre, 4 * g + r, 64), xi = __shfl(cim, 4 * g + r, 64);
        d1[0][0][r] = fmaf(sg, xr, d1[0][0][r]);
        d1[1][0][r] = fmaf(sg, xi, d1[1][0][r]);
      }
    }
    // stage 2: the accumulator rows 4g + r are (pair 2g + r/2, member r%2)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const f4 Ur = d1[0][2 * s], Ui = d1[1][2 * s], Vr = d1[0][2 * s + 1], Vi = d1[1][2 * s + 1];
      float a0u = 0.f, a0v = 0.f;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int ra = 2 * h2, rb = 2 * h2 + 1;
        float URp = Ur[ra] + Ur[rb], URm = Ur[ra] - Ur[rb], UIp = Ui[ra] + Ui[rb], UIm = Ui[ra] - Ui[rb];
        float VRp = Vr[ra] + Vr[rb], VRm = Vr[ra] - Vr[rb], VIp = Vi[ra] + Vi[rb], VIm = Vi[ra] - Vi[rb];
        if (h == 0 && h2 == 0) {   // uniform
          if (g == 0) {            // pair 0: packed slot (member 0) and column M/2 (member 1)
            a0u = Ur[ra] + Ui[ra];
            a0v = Vi[ra] - Vr[ra];
            URm = Ur[ra] - Ui[ra];
            VIm = Vi[ra] + Vr[ra];
            URp = Ur[rb];
            VIp = Vi[rb];
            UIp = Ui[rb];
            VRp = Vr[rb];
            UIm = 0.f;
            VRm = 0.f;
          }
        }
        const float4 Af = F2s[(h * 2 + h2) * 64 + lane];
        d2[s][0] = mma(Af.x, URp, d2[s][0]);
        d2[s][1] = mma(Af.x, VIp, d2[s][1]);
        d2[s][2] = mma(Af.y, UIm, d2[s][2]);
        d2[s][3] = mma(Af.y, VRm, d2[s][3]);
        d2[s][4] = mma(Af.z, URm, d2[s][4]);
        d2[s][5] = mma(Af.z, VIm, d2[s][5]);
        d2[s][6] = mma(Af.w, UIp, d2[s][6]);
        d2[s][7] = mma(Af.w, VRp, d2[s][7]);
      }
      if (h == 0) {   // a(0) = Y(0) + Y(M), weight 1 at every even dx
        const float xu = __shfl(a0u, p, 64), xv = __shfl(a0v, p, 64);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          d2[s][0][r] += xu;
          d2[s][1][r] += xv;
        }
      }
    }
  }

  // epilogue: X at (+-k, +-dx) from the eight stage-2 products, squared
  // (-1 marks slots outside the window and the duplicates of k = 0, dx = 0)
  float x2max = 0.0f;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int k = 2 * p + s;
    const bool kp = k <= S, km = kp && k > 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rho = 4 * g + r;
      const bool ap = 2 * rho <= S, am = ap && rho > 0, bp = 2 * rho + 1 <= S;
      const float Eap = d2[s][0][r] - d2[s][1][r], Eam = d2[s][0][r] + d2[s][1][r];
      const float Oap = d2[s][2][r] + d2[s][3][r], Oam = d2[s][2][r] - d2[s][3][r];
      const float Ebp = d2[s][4][r] - d2[s][5][r], Ebm = d2[s][4][r] + d2[s][5][r];
      const float Obp = d2[s][6][r] + d2[s][7][r], Obm = d2[s][6][r] - d2[s][7][r];
      float x[8];
      x[0] = Eap - Oap; x[1] = Eap + Oap; x[2] = Eam - Oam; x[3] = Eam + Oam;
      x[4] = Ebp - Obp; x[5] = Ebp + Obp; x[6] = Ebm - Obm; x[7] = Ebm + Obm;
      const bool ok[8] = {kp && ap, kp && am, km && ap, km && am, kp && bp, kp && bp, km && bp, km && bp};
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const float x2 = ok[v] ? x[v] * x[v] : -1.0f;
        d2[s][v][r] = x2;
        x2max = fmaxf(x2max, x2);
      }
    }
  }
  const float wmax = wmax_f(x2max);
  const int esc = 2 * (a.iexpo[i] + a.pexpo[q]);
  const double kappa = ldexp(a.kscale / (A * B), esc);
  const double rho2 = fmin((double)wmax * kappa, 1.0 - 0x1p-52);
  const float cu = (float)(kappa / (1.0 - rho2));
  const float base = wmax * cu;
  const double n = (double)a.nx * a.ny;
  const float c2 = (float)(0.5 * n - 1.0);
  float sum = 0.0f;
  if (c2 >= 1024.0f) {
    // log1p(u) by its degree-3 series on [0, 0.05]; terms with u >= 0.05 are
    // below e^-50 of the maximum term (1) and are left at u = 0.05
    const float c2l2e = c2 * 1.4426950408889634f;
    const float p1 = -c2l2e, p2 = 0.5f * c2l2e, p3 = -c2l2e / 3.0f;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int v = 0; v < 8; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x2 = d2[s][v][r];
          const float u = __builtin_amdgcn_fmed3f(fmaf(-x2, cu, base), 0.0f, 0.05f);
          const float t = __builtin_amdgcn_exp2f(u * (p1 + u * (p2 + u * p3)));
          sum += x2 >= 0.0f ? t : 0.0f;
        }
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int v = 0; v < 8; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x2 = d2[s][v][r];
          const float u = fmaxf(fmaf(-x2, cu, base), 0.0f);
          const float t = __expf(-c2 * log1p_f(u));
          sum += x2 >= 0.0f ? t : 0.0f;
        }
  }
  const float tot = wsum_f(sum);
  if (lane == 0) *out = bioem_erec{wmax, tot, -1, 0};
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_logpost_mf32(MfArgs ma) {
  extern __shared__ float4 lds_mf[];
  const int n1 = ma.KS1 * 64, n2 = ma.nHG * 128;
  for (int e = threadIdx.x; e < n1 + n2; e += 64 * WAVES) lds_mf[e] = e < n1 ? ma.F1[e] : ma.F2[e - n1];
  __syncthreads();
  const long n_items = (long)ma.n_ti * ma.n_ts * ma.ti * ma.ts * ma.a.nc;
  const int wave = blockIdx.x * WAVES + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * WAVES;
  for (long item = wave; item < n_items; item += nwaves) mf_item(ma, lds_mf, lds_mf + n1, (int)item);
}

constexpr int kMfWaves = 8;
constexpr int kMfTileImages = 32;
constexpr int kMfTileSlots = 128;

int mf_device_cus() {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  return ncu;
}

}  // namespace

size_t mf_len(int nx, int ny) { return mf_item_len(mf_geom(nx, ny)); }

size_t mf32_smem_bytes(int nx, int ny) {
  const MfGeom G = mf_geom(nx, ny);
  return sizeof(float4) * ((size_t)G.KS1 * 64 + (size_t)G.nHG * 128);
}

bool mf32_supported(int nx, int ny, int S) {
  return S >= 0 && S <= 31 && nx % 2 == 0 && ny % 2 == 0 && nx >= 4 && ny >= 4 &&
         mf32_smem_bytes(nx, ny) <= kMaxSmem;
}

hipError_t launch_mf_copy_spec(hipStream_t s, const float2* spec, int n, int nx, int ny, float4* out) {
  const long total = (long)n * (long)mf_len(nx, ny);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mf_copy_spec, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, spec, total, nx, ny,
                     out);
  return hipGetLastError();
}

hipError_t launch_mf_copy_at(hipStream_t s, const float2* ispec, const float* table, int ni, int nc, int nx, int ny,
                             float4* out) {
  const long total = (long)ni * nc * (long)mf_len(nx, ny);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mf_copy_at, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ispec, table, total,
                     nc, nx, ny, out);
  return hipGetLastError();
}

size_t mf32_table_len(int nx, int ny) {
  const MfGeom G = mf_geom(nx, ny);
  return (size_t)G.KS1 * 64 + (size_t)G.nHG * 128;
}

hipError_t launch_mf_tables(hipStream_t s, int nx, int ny, int S, float4* tabs) {
  const MfGeom G = mf_geom(nx, ny);
  const int n = G.KS1 * 64 + G.nHG * 128;
  hipLaunchKernelGGL(k_mf_tables, dim3((n + 255) / 256), dim3(256), 0, s, nx, ny, S, tabs, tabs + G.KS1 * 64);
  return hipGetLastError();
}

hipError_t launch_logpost_mf32(hipStream_t s, const LogpostArgs& a, const float4* at, const float4* pm,
                               const float4* tabs, int ti, int ts) {
  const MfGeom G = mf_geom(a.nx, a.ny);
  MfArgs ma{};
  ma.a = a;
  ma.at = at;
  ma.pm = pm;
  ma.F1 = tabs;
  ma.F2 = tabs + G.KS1 * 64;
  ma.KS1 = G.KS1;
  ma.nHG = G.nHG;
  ma.len = (long)mf_len(a.nx, a.ny);
  const int nslots = a.cand ? a.k : a.nq;
  ma.ti = ti > 0 ? ti : kMfTileImages;
  ma.ts = ts > 0 ? ts : kMfTileSlots;
  ma.n_ti = (a.ni + ma.ti - 1) / ma.ti;
  ma.n_ts = (nslots + ma.ts - 1) / ma.ts;
  const long n_items = (long)ma.n_ti * ma.n_ts * ma.ti * ma.ts * a.nc;
  if (n_items <= 0) return hipSuccess;
  if (n_items > 0x7fffffffL) return hipErrorInvalidValue;
  const size_t smem = mf32_smem_bytes(a.nx, a.ny);
  auto kern = k_logpost_mf32<kMfWaves>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const long want = (n_items + kMfWaves - 1) / kMfWaves;
  const int grid = (int)std::min<long>(want, (long)mf_device_cus());
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kMfWaves), smem, s, ma);
  return hipGetLastError();
}

}  // namespace bioem
