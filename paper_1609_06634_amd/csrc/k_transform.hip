// Projection of Gaussian-sphere models, half-spectrum DFTs, per-image sums and
// synthetic maps.  None of this is on the per-evaluation hot loop (it runs
// once per orientation or per image, Listing 1's outer loops), so it favours
// accuracy: every step computes in FP64 and only the stored spectra are FP32.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace bioem {

namespace {

constexpr int kProjWaves = 8;      // waves per projection workgroup (two per SIMD)
constexpr int kProjTiles = 13;     // 16x16 output tiles per wave
constexpr int kProjChunk = 16;     // spheres per LDS stage (four MFMA K-steps)
constexpr int kProjSeg = 63;       // pixels per wave segment (64 boundaries)
constexpr int kProjSuper = 512;    // spheres whose rotated parameters sit in LDS at once
constexpr int kDftRows = 8;        // rows per workgroup of the forward row transform
constexpr int kDftCols = 4;        // columns per workgroup of the forward column transform

typedef double d4 __attribute__((ext_vector_type(4)));

// Eq. (ideal) with each Gaussian integrated over the pixel:
//   I0[k][j] = sum_a w_a Ey_a[k] Ex_a[j],
//   Ex_a[j] = integral over pixel j of the unit 1-D Gaussian of width sigma_a
//             centred at the rotated x_a (likewise Ey),
// i.e. a [ny x ns] x [ns x nx] FP64 product per orientation, computed on the
// FP64 matrix cores (v_mfma_f64_16x16x4_f64) from factors built in LDS.
// A pixel integral is (erf(b) - erf(a))/2 over its two boundaries; each
// boundary's erfc(|z|) is evaluated once and shared with the neighbouring
// pixel, and the difference is taken on the side that avoids cancellation.
// A workgroup owns a band of whole 16-row tile rows (as many as its waves'
// accumulators hold) and builds the y factors of those rows only.
// grid: (bands, nq); block: 64 * kProjWaves.
__global__ __launch_bounds__(64 * kProjWaves, 1) void k_project(const double* __restrict__ spheres, int ns,
                                                             const double* __restrict__ quats, int nx,
                                                             int ny, double pixel, double* __restrict__ out) {
  __shared__ double ex[kProjChunk][kMaxBox];
  __shared__ double ey[kProjChunk][kMaxBox];
  __shared__ double rot[6];
  __shared__ int ext[kProjChunk][4];   // pixel ranges (x lo, x hi, y lo, y hi) of each sphere
  extern __shared__ double4 prm[];     // [kProjSuper]: rotated x, y, 1/(sqrt(2) sigma), weight
  const int q = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    double w = quats[4 * q + 0], x = quats[4 * q + 1], y = quats[4 * q + 2], z = quats[4 * q + 3];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    // first two rows of the active rotation matrix (z is integrated out)
    rot[0] = 1 - 2 * (y * y + z * z); rot[1] = 2 * (x * y - w * z); rot[2] = 2 * (x * z + w * y);
    rot[3] = 2 * (x * y + w * z); rot[4] = 1 - 2 * (x * x + z * z); rot[5] = 2 * (y * z - w * x);
  }
  const int tcols = (nx + 15) / 16, trows = (ny + 15) / 16;
  const int rb = (kProjWaves * kProjTiles) / tcols;            // tile rows per band
  const int tr0 = blockIdx.x * rb, tr1 = min(trows, tr0 + rb);
  const int band0 = tr0 * tcols, band1 = tr1 * tcols;
  const int nxp = 16 * tcols, ky0 = 16 * tr0, nyb = 16 * (tr1 - tr0);
  const int segx = (nxp + kProjSeg - 1) / kProjSeg, segy = (nyb + kProjSeg - 1) / kProjSeg;
  const int tasks = kProjChunk * (segx + segy);
  const double h = 0.5 * pixel;
  d4 acc[kProjTiles];
#pragma unroll
  for (int t = 0; t < kProjTiles; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  for (int s0 = 0; s0 < ns; s0 += kProjSuper) {
   const int sn = min(kProjSuper, ns - s0);
   // rotated centres and widths of this run of spheres, once per workgroup
   __syncthreads();
   for (int t = tid; t < sn; t += 64 * kProjWaves) {
     const double* sp = spheres + 5 * (size_t)(s0 + t);
     prm[t] = make_double4(rot[0] * sp[0] + rot[1] * sp[1] + rot[2] * sp[2],
                           rot[3] * sp[0] + rot[4] * sp[1] + rot[5] * sp[2], 1.0 / (sqrt(2.0) * sp[3]), sp[4]);
   }
   __syncthreads();
   for (int a0 = s0; a0 < s0 + sn; a0 += kProjChunk) {
    // Beyond 12 sigma plus a pixel from its centre a sphere's pixel integrals
    // are below erfc(8) ~ 1e-29 of its peak: segments and output tiles
    // outside every sphere's range take no factors and no products.
    if (tid < kProjChunk) {
      int r4[4] = {1, 0, 1, 0};   // empty
      if (a0 + tid < s0 + sn) {
        const double4 pa = prm[a0 - s0 + tid];
        const double R = (12.0 / (sqrt(2.0) * pa.z) + pixel) / pixel;   // 12 sigma + a pixel
        const double cx = pa.x / pixel + nx / 2, cy = pa.y / pixel + ny / 2;
        r4[0] = (int)fmax(floor(cx - R), -1.0); r4[1] = (int)fmin(ceil(cx + R), (double)nx);
        r4[2] = (int)fmax(floor(cy - R), -1.0); r4[3] = (int)fmin(ceil(cy + R), (double)ny);
      }
      for (int k = 0; k < 4; ++k) ext[tid][k] = r4[k];
    }
    __syncthreads();
    // factors of this chunk: one (sphere, axis, 63-pixel segment) per wave pass
    for (int task = wave; task < tasks; task += kProjWaves) {
      const int a = task / (segx + segy), r = task - a * (segx + segy);
      const bool yaxis = r >= segx;
      // pixels [lo, hi) of this axis are built; the segment starts at p0
      const int lo = yaxis ? ky0 : 0, hi = yaxis ? ky0 + nyb : nxp;
      const int p0 = lo + kProjSeg * (yaxis ? r - segx : r);
      const int n = yaxis ? ny : nx;
      double c = 0.0, inv = 0.0, wgt = 0.0;
      const bool real = a0 + a < s0 + sn;
      if (real) {
        const double4 pa = prm[a0 - s0 + a];
        c = yaxis ? pa.y : pa.x;
        inv = pa.z;
        wgt = yaxis ? pa.w : 1.0;
      }
      // boundary p0 + lane lies at the lower edge of pixel p0 + lane
      const int elo = ext[a][yaxis ? 2 : 0], ehi = ext[a][yaxis ? 3 : 1];
      const bool far = p0 + kProjSeg - 1 < elo || p0 > ehi;   // uniform across the wave
      const double zb = (((p0 + lane) - n / 2) * pixel - h - c) * inv;
      const double az = fabs(zb);
      const double eb = (!far && az < 27.3) ? erfc(az) : 0.0;   // erfc(27.3) < 2^-1074
      const double zn = __shfl_down(zb, 1, 64);
      const double en = __shfl_down(eb, 1, 64);
      const int p = p0 + lane;
      if (lane < kProjSeg && p < hi) {
        double v = 0.0;
        if (real && !far && p < n) {
          if (zb > 0.0) v = 0.5 * (eb - en);           // both boundaries above the centre
          else if (zn < 0.0) v = 0.5 * (en - eb);      // both below
          else v = 0.5 * ((1.0 - eb) + (1.0 - en));    // straddles the centre
        }
        if (yaxis) ey[a][p - ky0] = wgt * v;
        else ex[a][p] = wgt * v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kProjChunk / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4), li = lane & 15;
      // lane t decides whether some sphere of this K-step reaches the wave's
      // tile t; one ballot gives the wave a uniform mask
      bool reach = false;
      if (lane < kProjTiles) {
        const int tile = band0 + wave + kProjWaves * lane;
        if (tile < band1) {
          const int tr = tile / tcols, tc = tile - tr * tcols;
          for (int a = 4 * ks; a < 4 * ks + 4; ++a)
            reach = reach || (ext[a][0] <= 16 * tc + 15 && ext[a][1] >= 16 * tc && ext[a][2] <= 16 * tr + 15 &&
                              ext[a][3] >= 16 * tr);
        }
      }
      const uint64_t hit = __ballot(reach);
#pragma unroll
      for (int t = 0; t < kProjTiles; ++t) {
        const int tile = band0 + wave + kProjWaves * t;
        if (tile < band1 && ((hit >> t) & 1)) {   // uniform across the wave
          const int tr = tile / tcols, tc = tile - tr * tcols;
          const double av = ey[kk][16 * (tr - tr0) + li];
          const double bv = ex[kk][16 * tc + li];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
   }
  }
  // The FP64 16x16 result interleaves rows: D[i][j] sits in lane
  // j + 16 (i % 4), element i / 4 (unlike the FP32-output forms, where lane
  // groups hold consecutive rows).
  double* dst = out + (size_t)q * ny * nx;
#pragma unroll
  for (int t = 0; t < kProjTiles; ++t) {
    const int tile = band0 + wave + kProjWaves * t;
    if (tile < band1) {
      const int tr = tile / tcols, tc = tile - tr * tcols;
      const int j = 16 * tc + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * tr + (lane >> 4) + 4 * r;
        if (k < ny && j < nx) dst[(size_t)k * nx + j] = acc[t][r];
      }
    }
  }
}

// Row pass of the forward 2-D DFT: rows[i][k][m] = sum_j x[i][k][j] e^{-2 pi i m j / nx}.
// grid: ceil(n * ny / kDftRows) blocks; block: 128.
__global__ __launch_bounds__(128) void k_rdft_rows(const double* __restrict__ in64,
                                                   const float* __restrict__ in32, int nx, long nrows,
                                                   double2* __restrict__ rows) {
  // kDftRows rows per workgroup share each twiddle read; every output is
  // still one FMA chain over j in increasing order
  __shared__ double x[kDftRows][kMaxBox];
  __shared__ double2 tw[kMaxBox];
  const long row0 = (long)blockIdx.x * kDftRows;
  const int mh = nx / 2 + 1;
  for (int e = threadIdx.x; e < kDftRows * nx; e += blockDim.x) {
    const int r = e / nx, j = e - r * nx;
    const long row = row0 + r;
    x[r][j] = row < nrows ? (in64 ? in64[row * nx + j] : (double)in32[row * nx + j]) : 0.0;
  }
  for (int j = threadIdx.x; j < nx; j += blockDim.x) tw[j] = twiddle64(j, nx);
  __syncthreads();
  for (int m = threadIdx.x; m < mh; m += blockDim.x) {
    double re[kDftRows], im[kDftRows];
#pragma unroll
    for (int r = 0; r < kDftRows; ++r) re[r] = im[r] = 0.0;
    int t = 0;
    for (int j = 0; j < nx; ++j) {
      const double2 w = tw[t];
#pragma unroll
      for (int r = 0; r < kDftRows; ++r) {
        re[r] = fma(x[r][j], w.x, re[r]);
        im[r] = fma(-x[r][j], w.y, im[r]);
      }
      t += m;
      if (t >= nx) t -= nx;
    }
#pragma unroll
    for (int r = 0; r < kDftRows; ++r)
      if (row0 + r < nrows) rows[(row0 + r) * mh + m] = make_double2(re[r], im[r]);
  }
}

// Column pass: spec[i][m][l] = sum_k rows[i][k][m] e^{-2 pi i l k / ny}.
// grid: n * ceil(mh / kDftCols) blocks (kDftCols columns of one item each);
// block: 256.
__global__ __launch_bounds__(256) void k_cdft_cols(const double2* __restrict__ rows, int nx, int ny,
                                                   double2* __restrict__ spec) {
  __shared__ double2 col[kDftCols][kMaxBox];
  __shared__ double2 tw[kMaxBox];
  const int mh = nx / 2 + 1, groups = (mh + kDftCols - 1) / kDftCols;
  const size_t item = blockIdx.x / groups;
  const int m0 = (blockIdx.x - (int)item * groups) * kDftCols;
  for (int e = threadIdx.x; e < kDftCols * ny; e += blockDim.x) {
    const int c = e / ny, k = e - c * ny;
    col[c][k] = m0 + c < mh ? rows[(item * ny + k) * mh + m0 + c] : make_double2(0.0, 0.0);
  }
  for (int k = threadIdx.x; k < ny; k += blockDim.x) tw[k] = twiddle64(k, ny);
  __syncthreads();
  for (int l = threadIdx.x; l < ny; l += blockDim.x) {
    double re[kDftCols], im[kDftCols];
#pragma unroll
    for (int c = 0; c < kDftCols; ++c) re[c] = im[c] = 0.0;
    int t = 0;
    for (int k = 0; k < ny; ++k) {
      const double2 w = tw[t];
#pragma unroll
      for (int c = 0; c < kDftCols; ++c) {
        // (a + ib)(c - is) = (ac + bs) + i(bc - as)
        re[c] = fma(col[c][k].x, w.x, fma(col[c][k].y, w.y, re[c]));
        im[c] = fma(col[c][k].y, w.x, fma(-col[c][k].x, w.y, im[c]));
      }
      t += l;
      if (t >= ny) t -= ny;
    }
#pragma unroll
    for (int c = 0; c < kDftCols; ++c)
      if (m0 + c < mh) spec[(item * mh + m0 + c) * ny + l] = make_double2(re[c], im[c]);
  }
}

// Scale each item's spectrum by 2^-e with e the exponent of its largest
// magnitude (so all |values| < 1) and store as FP32 with each column padded
// with zeros to ldy rows.  grid: n; block: 256.
__global__ __launch_bounds__(256) void k_spec_store(const double2* __restrict__ spec64, int mh, int ny,
                                                    int ldy, float2* __restrict__ spec,
                                                    int32_t* __restrict__ expo) {
  __shared__ double red[256];
  const size_t item = blockIdx.x;
  const int len = mh * ny;
  const double2* src = spec64 + item * len;
  double mx = 0.0;
  for (int e = threadIdx.x; e < len; e += 256) mx = fmax(mx, fmax(fabs(src[e].x), fabs(src[e].y)));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  int ex = 0;
  if (red[0] > 0.0) frexp(red[0], &ex);
  if (threadIdx.x == 0) expo[item] = ex;
  float2* dst = spec + item * (size_t)mh * ldy;
  for (int e = threadIdx.x; e < mh * ldy; e += 256) {
    const int m = e / ldy, l = e - m * ldy;
    float2 v = make_float2(0.f, 0.f);
    if (l < ny) {
      const double2 x = src[m * ny + l];
      v = make_float2((float)ldexp(x.x, -ex), (float)ldexp(x.y, -ex));
    }
    dst[e] = v;
  }
}

// Deterministic FP64 block sum over 256 threads.
BIOEM_DEV double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Per-image C_o, C_oo and A = sum (I - C_o/n)^2 in FP64, two passes.
__global__ __launch_bounds__(256) void k_image_stats(const float* __restrict__ imgs, int npix,
                                                     double* __restrict__ stats) {
  __shared__ double red[256];
  const float* x = imgs + (size_t)blockIdx.x * npix;
  double s = 0.0, s2 = 0.0;
  for (int e = threadIdx.x; e < npix; e += 256) {
    const double v = x[e];
    s += v;
    s2 = fma(v, v, s2);
  }
  const double c_o = block_sum256(s, red);
  const double c_oo = block_sum256(s2, red);
  const double mean = c_o / npix;
  double a = 0.0;
  for (int e = threadIdx.x; e < npix; e += 256) {
    const double d = (double)x[e] - mean;
    a = fma(d, d, a);
  }
  const double A = block_sum256(a, red);
  if (threadIdx.x == 0) {
    stats[3 * blockIdx.x + 0] = c_o;
    stats[3 * blockIdx.x + 1] = c_oo;
    stats[3 * blockIdx.x + 2] = A;
  }
}

// CTF(s|a,A) Env(s|b) for signed frequencies (m, l), Section 2.
BIOEM_DEV double ctf_env(double a, double amp, double b, int m, int l, int nx, int ny, double pixel) {
  const int ls = (l <= ny / 2) ? l : l - ny;
  const double fx = (double)m / (nx * pixel), fy = (double)ls / (ny * pixel);
  const double s2 = 4.0 * M_PI * M_PI * (fx * fx + fy * fy);
  const double ph = 0.5 * a * s2;
  double sn, cs;
  sincos(ph, &sn, &cs);
  return (-amp * cs - sqrt(1.0 - amp * amp) * sn) * exp(-0.5 * b * s2);
}

// Synthetic map, step 1: spec1[i][m][l] = S_i[m][l] 2^e_i CTF Env (FP64).
__global__ __launch_bounds__(256) void k_render_filter(const float2* __restrict__ spec,
                                                       const int32_t* __restrict__ expo, int nx, int ny,
                                                       double pixel, const double* __restrict__ ctf,
                                                       double2* __restrict__ out) {
  const int mh = nx / 2 + 1;
  const size_t item = blockIdx.y;
  const int len = mh * ny;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  const int m = e / ny, l = e - m * ny;
  // no CTF table: the ideal image I0 itself
  const double t = ctf ? ctf_env(ctf[3 * item], ctf[3 * item + 1], ctf[3 * item + 2], m, l, nx, ny, pixel) : 1.0;
  const float2 v = spec[item * (size_t)mh * spec_ld(ny) + (size_t)m * spec_ld(ny) + l];
  const double sc = ldexp(1.0, expo[item]) * t;
  out[item * len + e] = make_double2(v.x * sc, v.y * sc);
}

// Inverse column pass: g[i][k][m] = sum_l spec1[i][m][l] e^{+2 pi i l k / ny}.
__global__ __launch_bounds__(128) void k_icdft_cols(const double2* __restrict__ spec, int nx, int ny,
                                                    double2* __restrict__ g) {
  __shared__ double2 col[kMaxBox];
  __shared__ double2 tw[kMaxBox];
  const int mh = nx / 2 + 1;
  const size_t item = blockIdx.x / mh;
  const int m = blockIdx.x - item * mh;
  for (int l = threadIdx.x; l < ny; l += blockDim.x) {
    col[l] = spec[(item * mh + m) * ny + l];
    tw[l] = twiddle64(l, ny);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ny; k += blockDim.x) {
    double re = 0.0, im = 0.0;
    int t = 0;
    for (int l = 0; l < ny; ++l) {
      re = fma(col[l].x, tw[t].x, fma(-col[l].y, tw[t].y, re));
      im = fma(col[l].y, tw[t].x, fma(col[l].x, tw[t].y, im));
      t += k;
      if (t >= ny) t -= ny;
    }
    g[(item * ny + k) * mh + m] = make_double2(re, im);
  }
}

// Inverse row pass (complex-to-real): i1[i][k][j] = (1/n) sum_m w_m Re(g e^{+2 pi i m j/nx}),
// w_m = 1 for m = 0 and m = nx/2, else 2 (the Hermitian partner columns).
__global__ __launch_bounds__(128) void k_icrdft_rows(const double2* __restrict__ g, int nx, int ny,
                                                     double* __restrict__ i1) {
  __shared__ double2 row[kMaxBox / 2 + 1];
  __shared__ double2 tw[kMaxBox];
  const int mh = nx / 2 + 1;
  const size_t r = blockIdx.x;
  for (int m = threadIdx.x; m < mh; m += blockDim.x) row[m] = g[r * mh + m];
  for (int j = threadIdx.x; j < nx; j += blockDim.x) tw[j] = twiddle64(j, nx);
  __syncthreads();
  const double inv_n = 1.0 / ((double)nx * ny);
  for (int j = threadIdx.x; j < nx; j += blockDim.x) {
    double acc = 0.0;
    int t = 0;
    for (int m = 0; m < mh; ++m) {
      const double w = (m == 0 || 2 * m == nx) ? 1.0 : 2.0;
      acc = fma(w, row[m].x * tw[t].x - row[m].y * tw[t].y, acc);
      t += j;
      if (t >= nx) t -= nx;
    }
    i1[r * nx + j] = acc * inv_n;
  }
}

// Real-space PSF of Eq. (3) for each CTF set c: its half spectrum is the real
// CTF x Env table, so the PSF image is the inverse transform of (T, 0).
__global__ __launch_bounds__(256) void k_psf_spec(const double* __restrict__ ctf, int nx, int ny, double pixel,
                                                  double2* __restrict__ out) {
  const int mh = nx / 2 + 1;
  const size_t item = blockIdx.y;
  const int len = mh * ny;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  const int m = e / ny, l = e - m * ny;
  out[item * len + e] =
      make_double2(ctf_env(ctf[3 * item], ctf[3 * item + 1], ctf[3 * item + 2], m, l, nx, ny, pixel), 0.0);
}

// The PSF truncated to the disc of radius R: K[c][dy + R][dx + R] =
// psf[c][dy mod ny][dx mod nx] where dx^2 + dy^2 <= R^2, else 0.
__global__ __launch_bounds__(256) void k_psf_window(const double* __restrict__ psf, int nx, int ny, int R,
                                                    double* __restrict__ K) {
  const int w = 2 * R + 1;
  const size_t c = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= w * w) return;
  const int dy = e / w - R, dx = e % w - R;
  K[c * w * w + e] = dx * dx + dy * dy <= R * R
                         ? psf[c * (size_t)nx * ny + (size_t)((dy + ny) % ny) * nx + (dx + nx) % nx]
                         : 0.0;
}

// Eq. (5) on the box without wrap, for n ideal images and one kernel:
//   out[i][y][x] = sum_{dy,dx} K[dy + R][dx + R] I0[i][y - dy][x - dx]
// over the offsets that stay in the box (FP64 products and sum, FP32 store).
// grid: (ceil(npix / 256), n); the kernel sits in LDS ((2R+1)^2 doubles).
__global__ __launch_bounds__(256) void k_psf_conv(const double* __restrict__ i0, int nx, int ny,
                                                  const double* __restrict__ K, int R, float* __restrict__ out) {
  extern __shared__ double ks[];
  const int w = 2 * R + 1;
  for (int e = threadIdx.x; e < w * w; e += 256) ks[e] = K[e];
  __syncthreads();
  const int npix = nx * ny;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const int y = p / nx, x = p - y * nx;
  const double* src = i0 + (size_t)blockIdx.y * npix;
  const int dy0 = max(-R, y - ny + 1), dy1 = min(R, y);     // 0 <= y - dy < ny
  const int dx0 = max(-R, x - nx + 1), dx1 = min(R, x);
  double acc = 0.0;
  for (int dy = dy0; dy <= dy1; ++dy) {
    const double* row = src + (size_t)(y - dy) * nx + x;
    const double* kr = ks + (dy + R) * w + R;
    for (int dx = dx0; dx <= dx1; ++dx) acc = fma(kr[dx], row[-dx], acc);
  }
  out[(size_t)blockIdx.y * npix + p] = (float)acc;
}

// Synthetic map, last step: shift, scale, offset and noise at the given SNR.
__global__ __launch_bounds__(256) void k_render_finish(const double* __restrict__ i1, int nx, int ny,
                                                       const int32_t* __restrict__ shifts,
                                                       const double* __restrict__ norm_offset,
                                                       const float* __restrict__ noise, double snr,
                                                       float* __restrict__ out) {
  __shared__ double red[256];
  const size_t item = blockIdx.x;
  const int npix = nx * ny;
  const double* x = i1 + item * npix;
  double s = 0.0;
  for (int e = threadIdx.x; e < npix; e += 256) s += x[e];
  const double mean = block_sum256(s, red) / npix;
  double v = 0.0;
  for (int e = threadIdx.x; e < npix; e += 256) {
    const double d = x[e] - mean;
    v = fma(d, d, v);
  }
  const double var = block_sum256(v, red) / npix;
  const double sigma = noise ? sqrt(var / snr) : 0.0;
  const int dx = shifts[2 * item], dy = shifts[2 * item + 1];
  const double N = norm_offset ? norm_offset[2 * item] : 1.0;
  const double mu = norm_offset ? norm_offset[2 * item + 1] : 0.0;
  for (int e = threadIdx.x; e < npix; e += 256) {
    const int k = e / nx, j = e - k * nx;
    const int ks = ((k + dy) % ny + ny) % ny, js = ((j + dx) % nx + nx) % nx;
    double val = N * x[ks * nx + js] - mu;
    if (noise) val += sigma * (double)noise[item * npix + e];
    out[item * npix + e] = (float)val;
  }
}

__global__ __launch_bounds__(256) void k_ctf_table(const double* __restrict__ ctf, int nx, int ny,
                                                   double pixel, float* __restrict__ table) {
  const int mh = nx / 2 + 1, ldy = spec_ld(ny), len = mh * ldy;
  const int c = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  const int m = e / ldy, l = e - m * ldy;
  table[(size_t)c * len + e] =
      l < ny ? (float)ctf_env(ctf[3 * c], ctf[3 * c + 1], ctf[3 * c + 2], m, l, nx, ny, pixel) : 0.0f;
}

// B_qc = (1/n) sum_{s != 0} w_s |P_q(s) T_c(s)|^2 (Plancherel), FP64.
// grid: nq * nc blocks; block: 256.
__global__ __launch_bounds__(256) void k_proj_norms(const float2* __restrict__ pspec,
                                                    const int32_t* __restrict__ pexpo,
                                                    const float* __restrict__ table, int nc, int nx,
                                                    int ny, double* __restrict__ B) {
  __shared__ double red[256];
  const int mh = nx / 2 + 1, ldy = spec_ld(ny), len = mh * ldy;
  const int q = blockIdx.x / nc, c = blockIdx.x - q * nc;
  const float2* p = pspec + (size_t)q * len;
  const float* t = table + (size_t)c * len;
  double acc = 0.0;
  for (int e = threadIdx.x; e < len; e += 256) {
    if (e == 0) continue;   // the DC term is excluded (the mean is integrated out)
    const int m = e / ldy;
    const double w = (m == 0 || 2 * m == nx) ? 1.0 : 2.0;
    const double tt = t[e];
    const double re = p[e].x * tt, im = p[e].y * tt;
    acc = fma(w, re * re + im * im, acc);
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) B[blockIdx.x] = ldexp(s, 2 * pexpo[q]) / ((double)nx * ny);
}

// |X|^2 of a half spectrum [n][mh][ny] in place, with the DC term set to 0
// (the image mean removed).
__global__ void k_power(double2* __restrict__ spec, long total, int per_item) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const double2 v = spec[e];
    spec[e] = make_double2(e % per_item == 0 ? 0.0 : v.x * v.x + v.y * v.y, 0.0);
  }
}

// Circular autocorrelation a[n][ny][nx] re-centred (lag 0 at (ny/2, nx/2),
// i.e. out(y, x) = a((y + ny/2) mod ny, (x + nx/2) mod nx)) with lag 0 set to
// 0 (it carries the noise power), as float.
__global__ void k_ac_finish(const double* __restrict__ a, int n, int nx, int ny, float* __restrict__ out) {
  const long total = (long)n * nx * ny;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int x = (int)(e % nx);
    const long t = e / nx;
    const int y = (int)(t % ny);
    const long b = t / ny;
    const int ys = (y + ny / 2) % ny, xs = (x + nx / 2) % nx;
    out[e] = (ys == 0 && xs == 0) ? 0.0f : (float)a[(b * ny + ys) * nx + xs];
  }
}

}  // namespace

static hipError_t last() { return hipGetLastError(); }

hipError_t launch_project_images(hipStream_t s, const double* spheres, int ns, const double* quats,
                                 int nq, int nx, int ny, double pixel, double* out_i0) {
  const int rb = (kProjWaves * kProjTiles) / ((nx + 15) / 16);
  dim3 grid(((ny + 15) / 16 + rb - 1) / rb, nq);
  const size_t smem = sizeof(double4) * kProjSuper;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_project),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_project, grid, dim3(64 * kProjWaves), smem, s, spheres, ns, quats, nx, ny, pixel, out_i0);
  return last();
}

hipError_t launch_rdft2(hipStream_t s, const double* real_in, const float* real_in_f32, int n,
                        int nx, int ny, double2* rows_scratch, double2* spec64) {
  const int mh = nx / 2 + 1;
  const long nrows = (long)n * ny;
  hipLaunchKernelGGL(k_rdft_rows, dim3((unsigned)((nrows + kDftRows - 1) / kDftRows)), dim3(128), 0, s, real_in,
                     real_in_f32, nx, nrows, rows_scratch);
  hipLaunchKernelGGL(k_cdft_cols, dim3(n * ((mh + kDftCols - 1) / kDftCols)), dim3(256), 0, s, rows_scratch, nx, ny,
                     spec64);
  return last();
}

hipError_t launch_spec_store(hipStream_t s, const double2* spec64, int n, int nx, int ny,
                             float2* spec, int32_t* expo) {
  hipLaunchKernelGGL(k_spec_store, dim3(n), dim3(256), 0, s, spec64, nx / 2 + 1, ny, spec_ld(ny), spec, expo);
  return last();
}

// Sets *flag to 1 if any of the n values is not finite (NaN or infinite).
__global__ __launch_bounds__(256) void k_flag_nonfinite(const float* __restrict__ x, size_t n,
                                                        unsigned* __restrict__ flag) {
  bool bad = false;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
    bad |= !isfinite(x[e]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

hipError_t launch_flag_nonfinite(hipStream_t s, const float* x, size_t n, unsigned* flag) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flag_nonfinite, dim3(blocks), dim3(256), 0, s, x, n, flag);
  return last();
}

hipError_t launch_image_stats(hipStream_t s, const float* imgs, int n, int npix, double* stats) {
  hipLaunchKernelGGL(k_image_stats, dim3(n), dim3(256), 0, s, imgs, npix, stats);
  return last();
}

// Unit quaternion (w, x, y, z) of z-y-z Euler angles (phi, theta, psi):
// q = qz(phi) qy(theta) qz(psi) (Hamilton products), the rotation
// Rz(phi) Ry(theta) Rz(psi).
BIOEM_DEV double4 qmul(double4 a, double4 b) {
  return make_double4(a.x * b.x - a.y * b.y - a.z * b.z - a.w * b.w, a.x * b.y + a.y * b.x + a.z * b.w - a.w * b.z,
                      a.x * b.z - a.y * b.w + a.z * b.x + a.w * b.y, a.x * b.w + a.y * b.z - a.z * b.y + a.w * b.x);
}

__global__ __launch_bounds__(256) void k_euler_quat(const double* __restrict__ e, int n, double* __restrict__ q) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s1, c1, s2, c2, s3, c3;
  sincos(0.5 * e[3 * i], &s1, &c1);
  sincos(0.5 * e[3 * i + 1], &s2, &c2);
  sincos(0.5 * e[3 * i + 2], &s3, &c3);
  const double4 r = qmul(qmul(make_double4(c1, 0.0, 0.0, s1), make_double4(c2, 0.0, s2, 0.0)),
                         make_double4(c3, 0.0, 0.0, s3));
  q[4 * i] = r.x;
  q[4 * i + 1] = r.y;
  q[4 * i + 2] = r.z;
  q[4 * i + 3] = r.w;
}

hipError_t launch_euler_quat(hipStream_t s, const double* euler, int n, double* quats) {
  hipLaunchKernelGGL(k_euler_quat, dim3((n + 255) / 256), dim3(256), 0, s, euler, n, quats);
  return last();
}

hipError_t launch_render(hipStream_t s, const float2* spec, const int32_t* expo, int n, int nx,
                         int ny, double pixel, const double* ctf, const int32_t* shifts,
                         const double* norm_offset, const float* noise, double snr,
                         double2* spec64, double2* cols_scratch, double* i1, float* out) {
  const int mh = nx / 2 + 1, len = mh * ny;
  hipLaunchKernelGGL(k_render_filter, dim3((len + 255) / 256, n), dim3(256), 0, s, spec, expo, nx,
                     ny, pixel, ctf, spec64);
  hipLaunchKernelGGL(k_icdft_cols, dim3(n * mh), dim3(128), 0, s, spec64, nx, ny, cols_scratch);
  hipLaunchKernelGGL(k_icrdft_rows, dim3(n * ny), dim3(128), 0, s, cols_scratch, nx, ny, i1);
  hipLaunchKernelGGL(k_render_finish, dim3(n), dim3(256), 0, s, i1, nx, ny, shifts, norm_offset,
                     noise, snr, out);
  return last();
}

hipError_t launch_ideal(hipStream_t s, const float2* spec, const int32_t* expo, int n, int nx, int ny,
                        double2* spec64, double2* cols_scratch, double* i0) {
  const int mh = nx / 2 + 1, len = mh * ny;
  hipLaunchKernelGGL(k_render_filter, dim3((len + 255) / 256, n), dim3(256), 0, s, spec, expo, nx, ny, 1.0,
                     (const double*)nullptr, spec64);
  hipLaunchKernelGGL(k_icdft_cols, dim3(n * mh), dim3(128), 0, s, spec64, nx, ny, cols_scratch);
  hipLaunchKernelGGL(k_icrdft_rows, dim3(n * ny), dim3(128), 0, s, cols_scratch, nx, ny, i0);
  return last();
}

hipError_t launch_psf_kernels(hipStream_t s, const double* ctf, int nc, int nx, int ny, double pixel, int R,
                              double2* spec64, double2* cols_scratch, double* psf, double* K) {
  const int mh = nx / 2 + 1, len = mh * ny, w = 2 * R + 1;
  hipLaunchKernelGGL(k_psf_spec, dim3((len + 255) / 256, nc), dim3(256), 0, s, ctf, nx, ny, pixel, spec64);
  hipLaunchKernelGGL(k_icdft_cols, dim3(nc * mh), dim3(128), 0, s, spec64, nx, ny, cols_scratch);
  hipLaunchKernelGGL(k_icrdft_rows, dim3(nc * ny), dim3(128), 0, s, cols_scratch, nx, ny, psf);
  hipLaunchKernelGGL(k_psf_window, dim3((w * w + 255) / 256, nc), dim3(256), 0, s, psf, nx, ny, R, K);
  return last();
}

hipError_t launch_psf_conv(hipStream_t s, const double* i0, int n, int nx, int ny, const double* K, int R,
                           float* out) {
  const int w = 2 * R + 1;
  hipLaunchKernelGGL(k_psf_conv, dim3((nx * ny + 255) / 256, n), dim3(256), sizeof(double) * w * w, s, i0, nx,
                     ny, K, R, out);
  return last();
}

hipError_t launch_autocorr(hipStream_t s, const float* imgs, int n, int nx, int ny, double2* rows_scratch,
                           double2* spec64, double2* cols_scratch, double* a64, float* out) {
  const int mh = nx / 2 + 1;
  const long total = (long)n * mh * ny;
  hipError_t e = launch_rdft2(s, nullptr, imgs, n, nx, ny, rows_scratch, spec64);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_power, dim3((unsigned)std::min<long>((total + 255) / 256, 65536L)), dim3(256), 0, s, spec64,
                     total, mh * ny);
  hipLaunchKernelGGL(k_icdft_cols, dim3(n * mh), dim3(128), 0, s, spec64, nx, ny, cols_scratch);
  hipLaunchKernelGGL(k_icrdft_rows, dim3(n * ny), dim3(128), 0, s, cols_scratch, nx, ny, a64);
  const long pix = (long)n * nx * ny;
  hipLaunchKernelGGL(k_ac_finish, dim3((unsigned)std::min<long>((pix + 255) / 256, 65536L)), dim3(256), 0, s, a64,
                     n, nx, ny, out);
  return last();
}

// Fragment-order copy of complex spectra: one float4 (two complex values) per
// thread, written contiguously.
__global__ __launch_bounds__(256) void k_tile_spec(const float2* __restrict__ spec, long total, int nx, int ny,
                                                   float4* __restrict__ tile) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int KS = split_ks(ny), ldy = spec_ld(ny), half = nx / 2;
  const long per = (long)tile_spec_len(nx, ny);
  const long item = idx / per;
  const int w = (int)(idx - item * per);
  const int lane = w & 63, r = (w >> 6) & 3, step = w >> 8;
  const int mt = step / KS, ks = step - mt * KS;
  const int m = 16 * mt + (lane & 15), l = 32 * ks + 8 * (lane >> 4) + 2 * r;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (m < half) {
    const float2* c = spec + (size_t)item * (nx / 2 + 1) * ldy + (size_t)m * ldy;
    const float2 a = c[l], b = c[l + 1];   // l + 1 < 32 KS = ldy; rows past ny are stored zeros
    v = make_float4(a.x, a.y, b.x, b.y);
  }
  tile[idx] = v;
}

// Fragment-order copy of real tables: four consecutive rows per float4.
__global__ __launch_bounds__(256) void k_tile_table(const float* __restrict__ table, long total, int nx, int ny,
                                                    float scale, float4* __restrict__ tile) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int KS = split_ks(ny), ldy = spec_ld(ny), half = nx / 2;
  const long per = (long)tile_table_len(nx, ny);
  const long item = idx / per;
  const int w = (int)(idx - item * per);
  const int lane = w & 63, r = (w >> 6) & 1, step = w >> 7;
  const int mt = step / KS, ks = step - mt * KS;
  const int m = 16 * mt + (lane & 15), l = 32 * ks + 8 * (lane >> 4) + 4 * r;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (m < half) {
    const float* c = table + (size_t)item * (nx / 2 + 1) * ldy + (size_t)m * ldy + l;
    v = make_float4(c[0] * scale, c[1] * scale, c[2] * scale, c[3] * scale);   // a power of two: exact
  }
  tile[idx] = v;
}

hipError_t launch_tile_spec(hipStream_t s, const float2* spec, int n, int nx, int ny, float4* tile) {
  const long total = (long)n * (long)tile_spec_len(nx, ny);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_spec, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, spec, total, nx, ny, tile);
  return last();
}

// The split forms take their conjugate products Z (each component at most 4
// in magnitude with spectra scaled below 1 and CTF values at most 1) and their
// stage-1 sums over the ny rows (at most 4 ny) as fp16 hi/lo pairs.  fp16's
// subnormal range makes the split exact only to about 2^-24 in absolute terms,
// which for the many small products of a large box adds up in X; the CTF
// values are therefore scaled by 2^zs, the largest power of two that keeps the
// stage-1 sums below 2^15 (in the tile copies and, once the projection norms
// are taken, in the table itself), and the kernel takes 2 zs off kappa's
// exponent.
int split_operand_scale(int ny) {
  int zs = 0;
  while (4.0 * ny * std::ldexp(1.0, zs + 1) <= 32768.0) ++zs;
  return zs;
}

__global__ __launch_bounds__(256) void k_scale_table(float* __restrict__ t, long n, float scale) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) t[idx] *= scale;
}

hipError_t launch_scale_table(hipStream_t s, float* table, size_t n, int zs) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, table, (long)n,
                     std::ldexp(1.0f, zs));
  return last();
}

hipError_t launch_tile_table(hipStream_t s, const float* table, int n, int nx, int ny, int zs, float4* tile) {
  const long total = (long)n * (long)tile_table_len(nx, ny);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, table, total, nx, ny,
                     std::ldexp(1.0f, zs), tile);
  return last();
}

hipError_t launch_ctf_table(hipStream_t s, const double* ctf, int nc, int nx, int ny, double pixel,
                            float* table) {
  const int len = (nx / 2 + 1) * spec_ld(ny);
  hipLaunchKernelGGL(k_ctf_table, dim3((len + 255) / 256, nc), dim3(256), 0, s, ctf, nx, ny, pixel, table);
  return last();
}

hipError_t launch_proj_norms(hipStream_t s, const float2* pspec, const int32_t* pexpo, int nq,
                             const float* table, int nc, int nx, int ny, double* B) {
  hipLaunchKernelGGL(k_proj_norms, dim3(nq * nc), dim3(256), 0, s, pspec, pexpo, table, nc, nx, ny, B);
  return last();
}

}  // namespace bioem
