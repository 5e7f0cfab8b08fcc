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
#include <type_traits>
#include <utility>

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
  G.KS1 = ((G.J1 + 1 + 3) / 4 + 1) & ~1;   // even: the K-steps are consumed in pairs
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

// Orbit-order copy of stored spectra (images with zero_dc: the (0, 0)
// coefficient is set to zero, so the product with any projection has no DC
// term and the offset mu is integrated out exactly).
__global__ __launch_bounds__(256) void k_mf_copy_spec(const float2* __restrict__ spec, long total, int nx, int ny,
                                                      int zero_dc, float4* __restrict__ out) {
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
    if (r0 >= 0 && !(zero_dc && col == 0 && r0 == 0)) { v.x = c[r0].x; v.y = c[r0].y; }
    if (r1 >= 0 && !(zero_dc && col == 0 && r1 == 0)) { v.z = c[r1].x; v.w = c[r1].y; }
  }
  out[idx] = v;
}

// Orbit-order copy of the CTF x envelope tables: for each (half group,
// K-step, lane) the four values T(j), T(H-j), T(H+j), T(N-j) of the lane's
// column (one float4), then the packed slot's second column [KS1][4].
__host__ __device__ inline size_t mf_tab_len(const MfGeom& G) {
  return (size_t)G.nHG * G.KS1 * 64 + (size_t)G.KS1 * 4;
}

__global__ __launch_bounds__(256) void k_mf_copy_table(const float* __restrict__ table, long total, int nx, int ny,
                                                       float4* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const MfGeom G = mf_geom(nx, ny);
  const long per = (long)mf_tab_len(G);
  const long item = idx / per;
  const int w = (int)(idx - item * per), ml = G.nHG * G.KS1 * 64;
  int col, j;
  if (w < ml) {
    const int lane = w & 63, step = w >> 6;
    const int h = step / G.KS1, s1 = step - h * G.KS1;
    col = mf_col(G, h, lane & 15);
    if (col == -2) col = 0;
    j = 4 * s1 + (lane >> 4);
  } else {
    const int w2 = w - ml;
    col = G.Mx;
    j = 4 * (w2 >> 2) + (w2 & 3);
  }
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  if (col >= 0) {
    const float* c = table + (size_t)item * (nx / 2 + 1) * spec_ld(ny) + (size_t)col * spec_ld(ny);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = mf_row(G, j, e);
      if (r >= 0) v[e] = c[r];
    }
  }
  out[idx] = make_float4(v[0], v[1], v[2], v[3]);
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
  const float4* im;     // [ni][len] image spectra, orbit order (chunk-relative images)
  const float4* pm;     // [nq][len] projection spectra, orbit order
  const float4* tm;     // [nc][tlen] CTF x envelope tables, orbit order
  const float4* F1;     // [KS1][64]
  const float4* F2;     // [nHG][2][64]
  const double* istats; const int32_t* iexpo; const int32_t* pexpo; const double* B;
  const int32_t* cand;  // [ni][k] or null
  bioem_erec* rec;      // [ni][nslots][nc]
  double kscale;
  long len, tlen;
  int ni, nq, nc, k, nx, ny, S;
  int KS1, nHG;
  int G, wpp, R, passes;        // pairs per group, waves per pair, K-steps per round, CTF passes
  int ti, ts, n_ti, n_ts;       // pair tile: images x orientation slots
};

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. N - 1, unrolled
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int kMfWaves = 4;     // one wave per SIMD in a workgroup
constexpr int kMfBlocksPerCU = 3; // three workgroups per CU: three waves per SIMD (at most 168 VGPRs)
constexpr int kSlotF4 = 136;    // one produced K-step in LDS: [2][64 lanes] float4 + [2][4] (packed column)

// 16-byte load through a buffer resource: voffset per lane, soffset uniform
__device__ __forceinline__ float4 bld4(__amdgpu_buffer_rsrc_t r, int vo, int so) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
}

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
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

// conj(a) b for the complex pairs (a.xy, b.xy) and (a.zw, b.zw).
__device__ __forceinline__ float4 cjmul2(float4 a, float4 b) {
  return make_float4(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x), fmaf(a.z, b.z, a.w * b.w),
                     fmaf(a.z, b.w, -a.w * b.z));
}

// Folded products of one orbit, W_e = conj(I_e) P_e (e = 0..3 over j, H-j,
// H+j, N-j):  (W0 + W3, W0 - W3), (W1 + W2, W1 - W2); for the shared slot
// (points 0, N/4, H, 3N/4): (W0, W2), (W1 + W3, W1 - W3).
__device__ __forceinline__ void fold_w(float4 i0, float4 i1, float4 p0, float4 p1, float4& o0, float4& o1) {
  const float4 w01 = cjmul2(i0, p0), w23 = cjmul2(i1, p1);
  o0 = make_float4(w01.x + w23.z, w01.y + w23.w, w01.x - w23.z, w01.y - w23.w);
  o1 = make_float4(w01.z + w23.x, w01.w + w23.y, w01.z - w23.x, w01.w - w23.y);
}

__device__ __forceinline__ void fold_w_special(float4 i0, float4 i1, float4 p0, float4 p1, float4& o0,
                                               float4& o1) {
  const float4 w01 = cjmul2(i0, p0), w23 = cjmul2(i1, p1);
  o0 = make_float4(w01.x, w01.y, w23.x, w23.y);
  o1 = make_float4(w01.z + w23.z, w01.w + w23.w, w01.z - w23.z, w01.w - w23.w);
}

// Block operands (u0, v0, u1, v1) of one column from its folded products X
// and CTF values T of the orbit.  Regular slot: with A+- = X0, B+- = X1 and
// T(j) = T(N-j) = Ta, T(H-j) = T(H+j) = Tb (the envelope is radial):
//   u0 = Ta A+ + Tb B+,  u1 = Ta A+ - Tb B+,  v0 = Ta A- - Tb B-,  v1 = Ta A- + Tb B-.
// Shared slot: u0 = T0 W0 + TH W2, u1 = T0 W0 - TH W2, v0 = 0,
// v1 = TQ (W1 - W3), and c = TQ (W1 + W3) is added to the even rows later.
struct Ops {
  float u0r, u0i, v0r, v0i, u1r, u1i, v1r, v1i;
};

__device__ __forceinline__ Ops ops_regular(float4 x0, float4 x1, float4 t) {
  const float ta = t.x, tb = t.y;
  const float ypr = tb * x1.x, ypi = tb * x1.y, ymr = tb * x1.z, ymi = tb * x1.w;
  Ops o;
  o.u0r = fmaf(ta, x0.x, ypr); o.u0i = fmaf(ta, x0.y, ypi);
  o.u1r = fmaf(ta, x0.x, -ypr); o.u1i = fmaf(ta, x0.y, -ypi);
  o.v0r = fmaf(ta, x0.z, -ymr); o.v0i = fmaf(ta, x0.w, -ymi);
  o.v1r = fmaf(ta, x0.z, ymr); o.v1i = fmaf(ta, x0.w, ymi);
  return o;
}

__device__ __forceinline__ Ops ops_special(float4 x0, float4 x1, float4 t, float& cr, float& ci) {
  const float t0 = t.x, tq = t.y, th = t.z;
  const float yr = th * x0.z, yi = th * x0.w;
  Ops o;
  o.u0r = fmaf(t0, x0.x, yr); o.u0i = fmaf(t0, x0.y, yi);
  o.u1r = fmaf(t0, x0.x, -yr); o.u1i = fmaf(t0, x0.y, -yi);
  o.v0r = 0.f; o.v0i = 0.f;
  o.v1r = tq * x1.z; o.v1i = tq * x1.w;
  cr = tq * x1.x; ci = tq * x1.y;
  return o;
}

// One workgroup: groups of G (image, orientation) pairs; wave w scores CTF set
// pass * wpp + w % wpp of pair w / wpp.  The folded products conj(I) P of each
// K-step are made once per pair (each wave makes one K-step of a round) and
// read by the pair's waves from LDS; every wave then applies its own CTF set.
//
// The consumed steps run half group by half group, two K-steps at a time
// (KS1 is even), with the cases that differ resolved at compile time: the
// first K-step of a half group holds the shared slot (points 0, N/4, H,
// 3N/4) in its lanes g = 0, and the first half group carries the packed
// slot's second column (x = nx/2) in lanes p = 0.  The CTF values of a step
// are loaded two steps ahead into one of two register sets.
//
// kSpec: the 224 x 224 box with four or more CTF sets (KS1 = 14, seven half
// groups, rounds of four K-steps, one pair per group), with every step
// unrolled so that round boundaries, shared-slot steps and stage 2 fall at
// compile-time positions and the global loads of a boundary are unconditional
// (indices clamped): the wait counts before each step are then exact.
template <bool kSpec>
__global__ __launch_bounds__(64 * kMfWaves, kMfBlocksPerCU) void k_logpost_mf32(MfArgs ma) {
  extern __shared__ float4 lds_mf[];
  const int n1 = ma.KS1 * 64, n2 = ma.nHG * 128;
  float4* const F1s = lds_mf;
  float4* const F2s = lds_mf + n1;
  float4* const slots = F2s + n2;                          // [2][kMfWaves][kSlotF4]
  float4* const stage = slots + 2 * kMfWaves * kSlotF4;    // [kMfWaves][16]
  for (int e = threadIdx.x; e < n1 + n2; e += 64 * kMfWaves) lds_mf[e] = e < n1 ? ma.F1[e] : ma.F2[e - n1];
  __syncthreads();

  int lane = threadIdx.x & 63, p = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int KS1 = kSpec ? 14 : ma.KS1, nHG = kSpec ? 7 : ma.nHG, nsteps = KS1 * nHG;
  const int G = kSpec ? 1 : ma.G, wpp = kSpec ? kMfWaves : ma.wpp, R = kSpec ? 4 : ma.R, passes = ma.passes;
  const int lgR = kSpec ? 2 : __builtin_ctz(R);   // R is a power of two
  const int nrounds = (nsteps + R - 1) >> lgR;
  const int nslots = ma.cand ? ma.k : ma.nq;
  const int S = ma.S;
  const size_t main_len = (size_t)nHG * KS1 * 128, tmain = (size_t)nHG * KS1 * 64;
  // producer role: K-step w % R of each round for pair w / R of the group
  const int gp_p = w >> lgR, kp = w & (R - 1);
  // consumer role
  const int gi = w / wpp, cw = w - gi * wpp;

  const int tile_pairs = ma.ti * ma.ts;
  const int groups_per_tile = (tile_pairs + G - 1) / G * passes;
  const int n_tiles = ma.n_ti * ma.n_ts;
  // tiles are dealt to the XCDs (workgroups go round-robin over the 8 XCDs),
  // so one tile's images stay in one L2 while its orientations stream through
  const int kx = min(8, (int)gridDim.x);
  const int xcd = blockIdx.x % kx, lw = blockIdx.x / kx;
  const int nwx = ((int)gridDim.x - xcd + kx - 1) / kx;

  for (int t = xcd; t < n_tiles; t += kx) {
    int dnts = ma.n_ts;
    asm volatile("" : "+s"(dnts));
    const int tI = t / dnts, tS = t - tI * dnts;
    for (int gg = lw; gg < groups_per_tile; gg += nwx) {
      // the divisors and the lane index pass through an empty asm at every
      // group, so that the divisors' reciprocals and the lane-derived
      // addresses are formed per group instead of being hoisted out of the
      // loops and held (or spilled to scratch) for the whole kernel
      int dpass = passes, dti = ma.ti;
      asm volatile("" : "+s"(dpass), "+s"(dti));
      asm volatile("" : "+v"(lane), "+v"(p), "+v"(g));
      const int pass = gg % dpass, grp = gg / dpass;
      // pair (image, slot) of group member m, valid or not
      auto pair_of = [&](int m, int& i, int& slot) -> bool {
        const int pl = grp * G + m;
        i = tI * dti + pl % dti;
        slot = tS * ma.ts + pl / dti;
        return pl < tile_pairs && i < ma.ni && slot < nslots;
      };
      // the group's first valid pair stands in for its invalid members (a
      // group can begin past the last image of a tile row and still hold
      // valid pairs); a group with none is skipped (uniform)
      int i0 = 0, s0 = 0, m0 = -1;
      for (int m = 0; m < G && m0 < 0; ++m)
        if (pair_of(m, i0, s0)) m0 = m;
      if (m0 < 0) continue;
      int ip, sp, ic, sc;
      if (!pair_of(gp_p, ip, sp)) { ip = i0; sp = s0; }
      const bool cvalid_pair = pair_of(gi, ic, sc);
      if (!cvalid_pair) { ic = i0; sc = s0; }
      const int c = pass * wpp + cw;
      const bool mine = cvalid_pair && c < ma.nc;
      const int cc = min(c, ma.nc - 1);
      const int qp = ma.cand ? ma.cand[(size_t)ip * ma.k + sp] : sp;
      const int qc = ma.cand ? ma.cand[(size_t)ic * ma.k + sc] : sc;
      const float4* Ib = ma.im + (size_t)ip * ma.len;
      const float4* Pb = ma.pm + (size_t)qp * ma.len;
      const float4* Tb = ma.tm + (size_t)cc * ma.tlen;
      // buffer resources of the three items: the loads below take their
      // offsets as a lane part (a register) and a uniform part (formed on the
      // scalar unit), with no 64-bit address arithmetic per load.  Word 3 of
      // a gfx9 resource: 32-bit data format, no swizzle or stride; the range
      // is the item's length (mf32_supported bounds it far below 2^31 bytes).
      constexpr int kRsrcW3 = 0x00020000;
      auto rsrc = [](const float4* q, size_t n) {   // q is uniform: taken from lane 0
        const uint64_t a = (uint64_t)q;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
        void* u = (void*)(((uint64_t)hi << 32) | lo);
        return __builtin_amdgcn_make_buffer_rsrc(u, 0, (int)(n * 16), kRsrcW3);
      };
      const __amdgpu_buffer_rsrc_t rI = rsrc(Ib, ma.len), rP = rsrc(Pb, ma.len), rT = rsrc(Tb, ma.tlen);

      // producer: loads of one K-step (and the packed slot's second column,
      // one float4 per lane of the first 16), then its folded products
      float4 pf0, pf1, pf2, pf3, pfs;
      auto load = [&](int rr, auto PFS) {
        if constexpr (kSpec) {   // unconditional: indices past the last step are clamped
          const int st = min((rr << lgR) + kp, nsteps - 1);
          const int vo = lane * 32, so = st * 2048;
          pf0 = bld4(rI, vo, so); pf1 = bld4(rI, vo + 16, so);
          pf2 = bld4(rP, vo, so); pf3 = bld4(rP, vo + 16, so);
          if constexpr (decltype(PFS)::value) {   // a round that can hold first-half-group steps
            // lanes 0, 1 of each four take the image, lanes 2, 3 the projection: both
            // are loaded and one is kept, as a resource cannot differ between lanes
            const int gs = (lane >> 2) & 3, which = lane & 3;
            const int vs = gs * 32 + (which & 1) * 16, ss = (int)(main_len * 16) + min(st, KS1 - 1) * 128;
            const float4 si = bld4(rI, vs, ss), sp = bld4(rP, vs, ss);
            pfs = which < 2 ? si : sp;
          }
          return;
        }
        const int st = (rr << lgR) + kp;
        if (st < nsteps) {
          const int vo = lane * 32, so = st * 2048;
          pf0 = bld4(rI, vo, so); pf1 = bld4(rI, vo + 16, so);
          pf2 = bld4(rP, vo, so); pf3 = bld4(rP, vo + 16, so);
          if (st < KS1) {   // first half group: the packed slot (used by lanes 0 .. 15)
            const int gs = (lane >> 2) & 3, which = lane & 3;
            const int vs = gs * 32 + (which & 1) * 16, ss = (int)(main_len * 16) + st * 128;
            const float4 si = bld4(rI, vs, ss), sp = bld4(rP, vs, ss);
            pfs = which < 2 ? si : sp;
          }
        }
      };
      auto produce = [&](int rr) {
        const int st = (rr << lgR) + kp;
        if (!kSpec && st >= nsteps) return;   // uniform per wave (kSpec: folds into the free buffer)
        const int s1 = st % KS1;
        float4* sl = slots + ((rr & 1) * kMfWaves + w) * kSlotF4;
        float4 o0, o1;
        fold_w(pf0, pf1, pf2, pf3, o0, o1);
        if (s1 == 0) {   // uniform: lanes g = 0 hold the shared slot
          float4 q0, q1;
          fold_w_special(pf0, pf1, pf2, pf3, q0, q1);
          if (g == 0) { o0 = q0; o1 = q1; }
        }
        sl[lane] = o0;
        sl[64 + lane] = o1;
        if (st < KS1) {   // uniform: first half group, the packed slot's second column
          float4* sg = stage + w * 16;
          if (lane < 16) sg[lane] = pfs;
          if (p == 0) {
            const float4 a0 = sg[4 * g], a1 = sg[4 * g + 1], b0 = sg[4 * g + 2], b1 = sg[4 * g + 3];
            if (s1 == 0 && g == 0) fold_w_special(a0, a1, b0, b1, o0, o1);
            else fold_w(a0, a1, b0, b1, o0, o1);
            sl[128 + g] = o0;
            sl[132 + g] = o1;
          }
        }
      };
      // start of round rr >= 1: every wave has consumed round rr - 1 and made
      // round rr; make round rr + 1 in the freed buffer, load round rr + 2
      auto boundary_at = [&](int st, auto PFS) {   // kSpec: the caller knows st is a round start
        const int rr = st >> lgR;
        // the lane index passes through an empty asm at every round, so that
        // the lane-derived LDS and global addresses are formed again for each
        // round rather than held across all of them (held, they exceed the
        // 168 registers of three waves per SIMD and spill to scratch)
        asm volatile("" : "+v"(lane), "+v"(p), "+v"(g));
        __syncthreads();
        produce(rr + 1);
        load(rr + 2, PFS);
      };
      auto boundary = [&](int st) {
        if ((st & (R - 1)) == 0 && st > 0) {   // uniform
          const int rr = st >> lgR;
          __syncthreads();
          if (rr + 1 < nrounds) produce(rr + 1);
          if (rr + 2 < nrounds) load(rr + 2, std::true_type{});
        }
      };

      f4 d2[2][8];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int v = 0; v < 8; ++v) d2[s][v] = f4{0.f, 0.f, 0.f, 0.f};
      f4 d1[2][4];
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int b = 0; b < 4; ++b) d1[tt][b] = f4{0.f, 0.f, 0.f, 0.f};
      float cre = 0.f, cim = 0.f;

      // stage 2 of half group h (its stage-1 accumulators are complete);
      // FIRST: h = 0, whose pair 0 is the packed slot and the column nx/4
      auto stage2 = [&](auto FIRST, int h) {
        // even rows: + (-1)^p (W(N/4) + W(3N/4)) T(N/4) of each column (rows
        // outside the window stay exact zeros)
        const float sg = 2 * p > S ? 0.0f : ((p & 1) ? -1.0f : 1.0f);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const float xr = __shfl(cre, 4 * g + rr, 64), xi = __shfl(cim, 4 * g + rr, 64);
          d1[0][0][rr] = fmaf(sg, xr, d1[0][0][rr]);
          d1[1][0][rr] = fmaf(sg, xi, d1[1][0][rr]);
        }
        // accumulator rows 4g + r are (pair 2g + r/2, member r%2)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const f4 Ur = d1[0][2 * s], Ui = d1[1][2 * s], Vr = d1[0][2 * s + 1], Vi = d1[1][2 * s + 1];
          float a0u = 0.f, a0v = 0.f;
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) {
            const int ra = 2 * h2, rb = 2 * h2 + 1;
            float URp = Ur[ra] + Ur[rb], URm = Ur[ra] - Ur[rb], UIp = Ui[ra] + Ui[rb], UIm = Ui[ra] - Ui[rb];
            float VRp = Vr[ra] + Vr[rb], VRm = Vr[ra] - Vr[rb], VIp = Vi[ra] + Vi[rb], VIm = Vi[ra] - Vi[rb];
            if constexpr (decltype(FIRST)::value) {
              if (h2 == 0 && g == 0) {   // pair 0: packed slot (member 0) and column nx/4 (member 1)
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
          if constexpr (decltype(FIRST)::value) {   // a(0) = Y(0) + Y(nx/2), weight 1 at every even dx
            const float xu = __shfl(a0u, p, 64), xv = __shfl(a0v, p, 64);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const bool in = 2 * (4 * g + rr) <= S;
              d2[s][0][rr] += in ? xu : 0.f;
              d2[s][1][rr] += in ? xv : 0.f;
            }
          }
        }
        // d1, cre and cim are restarted by the next half group's first K-step
      };

      // one consumed K-step st (K-step s1 of its half group); tc / tsc hold
      // its CTF values and receive those of step st + 2.  PK: first half
      // group (packed slot); SP: s1 = 0 (shared slot in lanes g = 0).
      auto step = [&](auto PK, auto SP, int st, int s1, float4& tc, float4& tsc) {
        constexpr bool kPK = decltype(PK)::value, kSP = decltype(SP)::value;
        if constexpr (!kSpec) asm volatile("" : "+v"(lane), "+v"(p), "+v"(g));   // see boundary_at
        const int rr = st >> lgR;
        const float4* sl = slots + ((rr & 1) * kMfWaves + gi * R + (st & (R - 1))) * kSlotF4;
        const float4 x0 = sl[lane], x1 = sl[64 + lane], bf = F1s[s1 * 64 + lane];
        Ops o;
        if constexpr (kSP) {
          float cr = 0.f, ci = 0.f;
          const Ops a = ops_regular(x0, x1, tc), b = ops_special(x0, x1, tc, cr, ci);
          const bool spl = g == 0;
          o.u0r = spl ? b.u0r : a.u0r; o.u0i = spl ? b.u0i : a.u0i;
          o.v0r = spl ? b.v0r : a.v0r; o.v0i = spl ? b.v0i : a.v0i;
          o.u1r = spl ? b.u1r : a.u1r; o.u1i = spl ? b.u1i : a.u1i;
          o.v1r = spl ? b.v1r : a.v1r; o.v1i = spl ? b.v1i : a.v1i;
          cre = spl ? cr : 0.f;
          cim = spl ? ci : 0.f;
        } else {
          o = ops_regular(x0, x1, tc);
        }
        if constexpr (kPK) {
          if (p == 0) {  // packed slot: + i x (the column nx/2)
            const float4 y0 = sl[128 + g], y1 = sl[132 + g];
            Ops m;
            float cr = 0.f, ci = 0.f;
            if (kSP && g == 0) m = ops_special(y0, y1, tsc, cr, ci);
            else m = ops_regular(y0, y1, tsc);
            o.u0r -= m.u0i; o.u0i += m.u0r;
            o.v0r -= m.v0i; o.v0i += m.v0r;
            o.u1r -= m.u1i; o.u1i += m.u1r;
            o.v1r -= m.v1i; o.v1i += m.v1r;
            cre -= ci; cim += cr;
          }
        }
        // this register set now takes the CTF values of step st + 2 (the
        // load is unconditional, clamped to the last step, so that no copy
        // of the old values has to wait for it)
        {
          const int sn = min(st + 2, nsteps - 1);
          tc = bld4(rT, lane * 16, sn * 1024);
          if constexpr (kPK) tsc = bld4(rT, g * 16, (int)(tmain * 16) + min(st + 2, KS1 - 1) * 64);
        }
        // the first K-step of a half group starts its accumulators (a zero
        // C operand instead of clearing 32 registers)
        const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
        d1[0][0] = mma(o.u0r, bf.x, kSP ? z4 : d1[0][0]);
        d1[1][0] = mma(o.u0i, bf.x, kSP ? z4 : d1[1][0]);
        d1[0][1] = mma(o.v0r, bf.y, kSP ? z4 : d1[0][1]);
        d1[1][1] = mma(o.v0i, bf.y, kSP ? z4 : d1[1][1]);
        d1[0][2] = mma(o.u1r, bf.z, kSP ? z4 : d1[0][2]);
        d1[1][2] = mma(o.u1i, bf.z, kSP ? z4 : d1[1][2]);
        d1[0][3] = mma(o.v1r, bf.w, kSP ? z4 : d1[0][3]);
        d1[1][3] = mma(o.v1i, bf.w, kSP ? z4 : d1[1][3]);
      };

      // CTF values of steps 0 and 1 (KS1 >= 2), in the two register sets
      float4 ta = Tb[lane], tb = Tb[64 + lane];
      float4 tsa = make_float4(0.f, 0.f, 0.f, 0.f), tsb = tsa;
      if (p == 0) {
        tsa = Tb[tmain + g];
        tsb = Tb[tmain + 4 + g];
      }

      load(0, std::true_type{});
      produce(0);
      if (nrounds > 1) load(1, std::true_type{});
      __syncthreads();
      if (nrounds > 1) produce(1);
      if (nrounds > 2) load(2, std::true_type{});

      using T_ = std::integral_constant<bool, true>;
      using F_ = std::integral_constant<bool, false>;
      if constexpr (kSpec) {
        // first half group: steps 0 .. 13, boundaries at 4, 8, 12
        static_for<14>([&](auto I) {
          constexpr int o = decltype(I)::value;
          // the round loaded at o holds steps 4 (o / 4 + 2) .. + 3: first
          // half group steps (below 14) only for o = 4
          if constexpr (o > 0 && (o & 3) == 0) boundary_at(o, std::integral_constant<bool, o == 4>{});
          if constexpr (o & 1) step(T_{}, std::integral_constant<bool, o == 0>{}, o, o, tb, tsb);
          else step(T_{}, std::integral_constant<bool, o == 0>{}, o, o, ta, tsa);
        });
        stage2(T_{}, 0);
        // half groups 1 .. 6 in pairs: steps 14 + 28 hp + o, boundaries where
        // 14 + o is a multiple of 4
        for (int hp = 0; hp < 3; ++hp) {
          asm volatile("" : "+v"(lane), "+v"(p), "+v"(g));   // see boundary_at
          const int base = 14 + 28 * hp;
          static_for<28>([&](auto I) {
            constexpr int o = decltype(I)::value;
            constexpr int s1 = o % 14;
            if constexpr (((14 + o) & 3) == 0) boundary_at(base + o, std::false_type{});
            if constexpr (o & 1) step(F_{}, std::integral_constant<bool, s1 == 0>{}, base + o, s1, tb, tsb);
            else step(F_{}, std::integral_constant<bool, s1 == 0>{}, base + o, s1, ta, tsa);
            if constexpr (s1 == 13) stage2(F_{}, 1 + 2 * hp + o / 14);
          });
        }
      } else {
      const bool r1 = R == 1;   // a round boundary can fall on an odd step
      // first half group
      boundary(0);
      step(T_{}, T_{}, 0, 0, ta, tsa);
      if (r1) boundary(1);
      step(T_{}, F_{}, 1, 1, tb, tsb);
      int st = 2;
      for (int s1 = 2; s1 < KS1; s1 += 2, st += 2) {
        boundary(st);
        step(T_{}, F_{}, st, s1, ta, tsa);
        if (r1) boundary(st + 1);
        step(T_{}, F_{}, st + 1, s1 + 1, tb, tsb);
      }
      stage2(T_{}, 0);
      for (int h = 1; h < nHG; ++h) {
        boundary(st);
        step(F_{}, T_{}, st, 0, ta, tsa);
        if (r1) boundary(st + 1);
        step(F_{}, F_{}, st + 1, 1, tb, tsb);
        st += 2;
        for (int s1 = 2; s1 < KS1; s1 += 2, st += 2) {
          boundary(st);
          step(F_{}, F_{}, st, s1, ta, tsa);
          if (r1) boundary(st + 1);
          step(F_{}, F_{}, st + 1, s1 + 1, tb, tsb);
        }
        stage2(F_{}, h);
      }
      }
      __syncthreads();   // the last round's slots are read before the next group makes round 0

      // epilogue of this wave's evaluation (image ic, orientation qc, CTF c)
      const double A = ma.istats[3 * ic + 2];
      const double Bq = ma.B[(size_t)qc * ma.nc + cc];
      bioem_erec* out = ma.rec + ((size_t)ic * nslots + sc) * ma.nc + cc;
      if (!(A > 0.0) || !(Bq > 0.0)) {   // uniform: degenerate image or projection
        if (mine && lane == 0) *out = bioem_erec{-1.0f, 0.0f, -1, 0};
        continue;
      }
      // X at (+-k, +-dx) from the eight stage-2 products, squared in place.
      // Rows outside the window hold exact zeros (zero coefficients), and the
      // duplicates of k = 0 and dx = 0 are set to zero here, so every slot
      // that is not one of the (2S+1)^2 shifts holds X^2 = 0: their terms are
      // taken off the sum at the end as a count.
      float x2max = 0.0f;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const float Eap = d2[s][0][rr] - d2[s][1][rr], Eam = d2[s][0][rr] + d2[s][1][rr];
          const float Oap = d2[s][2][rr] + d2[s][3][rr], Oam = d2[s][2][rr] - d2[s][3][rr];
          const float Ebp = d2[s][4][rr] - d2[s][5][rr], Ebm = d2[s][4][rr] + d2[s][5][rr];
          const float Obp = d2[s][6][rr] + d2[s][7][rr], Obm = d2[s][6][rr] - d2[s][7][rr];
          float x[8];
          x[0] = Eap - Oap; x[1] = Eap + Oap; x[2] = Eam - Oam; x[3] = Eam + Oam;
          x[4] = Ebp - Obp; x[5] = Ebp + Obp; x[6] = Ebm - Obm; x[7] = Ebm + Obm;
          if (s == 0) {   // k = 0: -k repeats +k
            const bool k0 = p == 0;
            x[2] = k0 ? 0.f : x[2]; x[3] = k0 ? 0.f : x[3];
            x[6] = k0 ? 0.f : x[6]; x[7] = k0 ? 0.f : x[7];
          }
          if (rr == 0) {   // dx = 0: -dx repeats +dx
            const bool r0 = g == 0;
            x[1] = r0 ? 0.f : x[1]; x[3] = r0 ? 0.f : x[3];
          }
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            const float x2 = x[v] * x[v];
            d2[s][v][rr] = x2;
            x2max = fmaxf(x2max, x2);
          }
        }
      }
      const float wmax = wmax_f(x2max);
      const int esc = 2 * (ma.iexpo[ic] + ma.pexpo[qc]);
      const double kappa = ldexp(ma.kscale / (A * Bq), esc);
      const double rho2 = fmin((double)wmax * kappa, 1.0 - 0x1p-52);
      const float cu = (float)(kappa / (1.0 - rho2));
      // the box size passes through an empty asm here, so the constants below
      // are formed in the epilogue instead of being hoisted out of the group
      // loop and held (or spilled) across all K-steps
      int npix = ma.nx * ma.ny, Se = S;
      asm volatile("" : "+s"(npix), "+s"(Se));
      const double n = (double)npix;
      const float c2 = (float)(0.5 * n - 1.0);
      const float nzero = (float)(64 * 64 - (2 * Se + 1) * (2 * Se + 1));
      // u = (max X^2 - X^2) c_u: >= 0, and exactly 0 at the maximum
      float sum = 0.0f, f0;
      if (c2 >= 1024.0f) {
        // log1p(u) by its degree-3 series, which is never below log1p(u): a
        // term with u >= 0.05 is below e^-50 of the maximum term (1) and
        // stays negligible
        const float c2l2e = c2 * 1.4426950408889634f;
        const float p1 = -c2l2e, p2 = 0.5f * c2l2e, p3 = -c2l2e / 3.0f;
        auto term = [&](float x2) {
          const float u = (wmax - x2) * cu;
          return __builtin_amdgcn_exp2f(u * fmaf(u, fmaf(u, p3, p2), p1));
        };
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int v = 0; v < 8; ++v)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) sum += term(d2[s][v][rr]);
        f0 = term(0.0f);
      } else {
        auto term = [&](float x2) { return __expf(-c2 * log1p_f((wmax - x2) * cu)); };
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int v = 0; v < 8; ++v)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) sum += term(d2[s][v][rr]);
        f0 = term(0.0f);
      }
      const float tot = wsum_f(sum) - nzero * f0;
      if (mine && lane == 0) *out = bioem_erec{wmax, tot, -1, 0};
    }
  }
}

constexpr int kMfTileImages = 8;
constexpr int kMfTileSlots = 64;

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
size_t mf_table_len(int nx, int ny) { return mf_tab_len(mf_geom(nx, ny)); }

size_t mf32_smem_bytes(int nx, int ny) {
  const MfGeom G = mf_geom(nx, ny);
  return sizeof(float4) * ((size_t)G.KS1 * 64 + (size_t)G.nHG * 128 + 2 * kMfWaves * kSlotF4 + kMfWaves * 16);
}

bool mf32_supported(int nx, int ny, int S) {
  return S >= 0 && S <= 31 && nx % 2 == 0 && ny % 2 == 0 && nx >= 4 && ny >= 4 &&
         mf32_smem_bytes(nx, ny) <= kMaxSmem;
}

hipError_t launch_mf_copy_spec(hipStream_t s, const float2* spec, int n, int nx, int ny, bool zero_dc,
                               float4* out) {
  const long total = (long)n * (long)mf_len(nx, ny);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mf_copy_spec, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, spec, total, nx, ny,
                     zero_dc ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_mf_copy_table(hipStream_t s, const float* table, int nc, int nx, int ny, float4* out) {
  const long total = (long)nc * (long)mf_table_len(nx, ny);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mf_copy_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, table, total, nx,
                     ny, out);
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

hipError_t launch_logpost_mf32(hipStream_t s, const LogpostArgs& a, const float4* im, const float4* pm,
                               const float4* tm, const float4* tabs, int ti, int ts) {
  const MfGeom G = mf_geom(a.nx, a.ny);
  MfArgs ma{};
  ma.im = im; ma.pm = pm; ma.tm = tm;
  ma.F1 = tabs;
  ma.F2 = tabs + G.KS1 * 64;
  ma.istats = a.istats; ma.iexpo = a.iexpo; ma.pexpo = a.pexpo; ma.B = a.B;
  ma.cand = a.cand; ma.k = a.k;
  ma.rec = a.rec;
  ma.kscale = a.kscale;
  ma.len = (long)mf_item_len(G);
  ma.tlen = (long)mf_tab_len(G);
  ma.ni = a.ni; ma.nq = a.nq; ma.nc = a.nc; ma.nx = a.nx; ma.ny = a.ny; ma.S = a.S;
  ma.KS1 = G.KS1;
  ma.nHG = G.nHG;
  // waves per pair: the CTF sets of one pair share its products (a power of
  // two up to the workgroup's wave count, so a group of pairs fills it)
  int wpp = 1;
  while (wpp < a.nc && wpp < kMfWaves) wpp *= 2;
  ma.wpp = wpp;
  ma.G = kMfWaves / wpp;
  ma.R = kMfWaves / ma.G;            // every wave makes one K-step per round
  ma.passes = (a.nc + wpp - 1) / wpp;
  const int nslots = a.cand ? a.k : a.nq;
  ma.ti = ti > 0 ? ti : kMfTileImages;
  ma.ts = ts > 0 ? ts : kMfTileSlots;
  ma.n_ti = (a.ni + ma.ti - 1) / ma.ti;
  ma.n_ts = (nslots + ma.ts - 1) / ma.ts;
  const long groups = (long)ma.n_ti * ma.n_ts * (((long)ma.ti * ma.ts + ma.G - 1) / ma.G) * ma.passes;
  if (groups <= 0) return hipSuccess;
  if ((long)ma.n_ti * ma.n_ts > 0x7fffffffL || (long)ma.ti * ma.ts * ma.passes > 0x7fffffffL)
    return hipErrorInvalidValue;
  const size_t smem = mf32_smem_bytes(a.nx, a.ny);
  const bool spec = G.KS1 == 14 && G.nHG == 7 && wpp == kMfWaves;
  const void* fn = spec ? reinterpret_cast<const void*>(k_logpost_mf32<true>)
                        : reinterpret_cast<const void*>(k_logpost_mf32<false>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const int grid = (int)std::min<long>(groups, (long)kMfBlocksPerCU * mf_device_cus());
  if (spec)
    hipLaunchKernelGGL(k_logpost_mf32<true>, dim3(grid), dim3(64 * kMfWaves), smem, s, ma);
  else
    hipLaunchKernelGGL(k_logpost_mf32<false>, dim3(grid), dim3(64 * kMfWaves), smem, s, ma);
  return hipGetLastError();
}

}  // namespace bioem
