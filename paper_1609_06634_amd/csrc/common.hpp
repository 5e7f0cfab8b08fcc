// Internal declarations shared by the BioEM HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/bioem.h"

#include <vector>

struct bioem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // the caller's stream (nullptr: the null stream)
  std::string err;
  // optional timing of the main kernel launches of the last bioem_logpost
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
  double timed_evals = 0.0;
  // tile shapes of the split kernel chosen by the autotuner, per key
  bool autotune = false;
  std::vector<bioem_tuning> tuned;
  // device address of this device's copy of the allocation-free scratch
  // (nullptr if it could not be resolved)
  void* scratch = nullptr;
};

// Half spectra are stored column-major per item: spec[item][m][l] with
// m in [0, nx/2] (x frequency) and l in [0, ny) (y frequency), each column
// zero-padded to spec_ld(ny) rows, scaled by
// 2^-expo[item] so that every |value| <= 1 (the split-precision kernels need
// a bounded range; the scale is undone in FP64 in the likelihood epilogue).
//
// The split-precision kernel reads a second copy in its matrix-fragment
// order (tile_spec_len(nx, ny) float4 per item): for column tile mt (16
// columns m = 16 mt + j, m < nx/2), row step ks (32 rows l) and part r, the
// 64 lanes' values are contiguous, so every load instruction of a wave reads
// 1 KB in one piece:
//   tile[item][(mt*KS + ks)*4 + r][lane] = (Z(l), Z(l+1)) as (re, im, re, im),
//   lane = j + 16 g, l = 32 ks + 8 g + 2 r; zero for m >= nx/2 or l >= ny.
// Column nx/2 is read from the column-major copy.
struct bioem_proj {
  int32_t n = 0, nx = 0, ny = 0;
  double pixel = 0.0;         // A per pixel (sets the CTF frequency scale)
  float2* spec = nullptr;     // [n][nx/2+1][spec_ld(ny)]
  float4* tile = nullptr;     // [n][tile_spec_len(nx, ny)]
  float4* mf = nullptr;       // [n][mf_len(nx, ny)] orbit-order copy (FP32 matrix-core kernel)
  int32_t* expo = nullptr;    // [n]
  int device = 0;
};

struct bioem_imgs {
  int32_t n = 0, nx = 0, ny = 0;
  float2* spec = nullptr;     // [n][nx/2+1][spec_ld(ny)]
  float4* tile = nullptr;     // [n][tile_spec_len(nx, ny)]
  float4* mf = nullptr;       // [n][mf_len(nx, ny)] orbit-order copy, DC zeroed (FP32 matrix-core kernel)
  int32_t* expo = nullptr;    // [n]
  double* stats = nullptr;    // [n][3]: C_o, C_oo, A
  int device = 0;
};

// Per-evaluation (image, orientation, CTF set) result of the main kernels,
// in the scaled units of the stored spectra:
//   x2max = max over the shift window of X(d)^2,
//   srel  = sum over the window of exp(l(d) - l(d_max)), in [1, W^2],
//   d     = (dy+S)*(2S+1) + (dx+S) of the maximum (lowest index on ties).
// The FP64 likelihood terms are added by the finalisation kernel.
struct bioem_erec {
  float x2max;
  float srel;
  int32_t d;
  int32_t pad;
};

namespace bioem {

constexpr int kMaxBox = 512;

// ---- launchers implemented in the kernel sources -------------------------
// Transforms (FP64 arithmetic); all enqueue on `s`.
hipError_t launch_project_images(hipStream_t s, const double* spheres, int ns, const double* quats,
                                 int nq, int nx, int ny, double pixel, double* out_i0);
hipError_t launch_rdft2(hipStream_t s, const double* real_in, const float* real_in_f32, int n,
                        int nx, int ny, double2* rows_scratch, double2* spec64);
hipError_t launch_spec_store(hipStream_t s, const double2* spec64, int n, int nx, int ny,
                             float2* spec, int32_t* expo);
hipError_t launch_image_stats(hipStream_t s, const float* imgs, int n, int npix, double* stats);
// *flag |= 1 if any of x[0..n) is NaN or infinite (flag zeroed by the caller).
hipError_t launch_flag_nonfinite(hipStream_t s, const float* x, size_t n, unsigned* flag);
// z-y-z Euler angles [n][3] (radians) -> unit quaternions [n][4] (w, x, y, z).
hipError_t launch_euler_quat(hipStream_t s, const double* euler, int n, double* quats);
// Fragment-order copies: complex spectra [n][nx/2+1][spec_ld(ny)] -> [n][tile_spec_len],
// real tables [n][nx/2+1][spec_ld(ny)] -> [n][tile_table_len] (rows l = 32 ks + 8 g + 4 r .. +3, r < 2).
hipError_t launch_tile_spec(hipStream_t s, const float2* spec, int n, int nx, int ny, float4* tile);
hipError_t launch_tile_table(hipStream_t s, const float* table, int n, int nx, int ny, int zs, float4* tile);
// Exponent zs of the split forms' operand scale 2^zs for an ny-row box, and
// the scaling of n table values by 2^zs (exact).
int split_operand_scale(int ny);
hipError_t launch_scale_table(hipStream_t s, float* table, size_t n, int zs);
hipError_t launch_render(hipStream_t s, const float2* spec, const int32_t* expo, int n, int nx,
                         int ny, double pixel, const double* ctf, const int32_t* shifts,
                         const double* norm_offset, const float* noise, double snr,
                         double2* spec64, double2* cols_scratch, double* i1, float* out);

// Ideal images I0 (no CTF) in real space, FP64: i0 [n][ny][nx].
hipError_t launch_ideal(hipStream_t s, const float2* spec, const int32_t* expo, int n, int nx, int ny,
                        double2* spec64, double2* cols_scratch, double* i0);
// Real-space PSFs of nc CTF sets (Eq. 3) truncated to the disc of radius R:
// K [nc][2R+1][2R+1] (scratch spec64 / cols [nc][nx/2+1][ny], psf [nc][ny][nx]).
constexpr int kPsfMaxRadius = 32;
hipError_t launch_psf_kernels(hipStream_t s, const double* ctf, int nc, int nx, int ny, double pixel, int R,
                              double2* spec64, double2* cols_scratch, double* psf, double* K);
// Eq. (5) on the box without wrap: out [n][ny][nx] float = I0 [n] convolved with K.
hipError_t launch_psf_conv(hipStream_t s, const double* i0, int n, int nx, int ny, const double* K, int R,
                           float* out);

// Centred circular autocorrelation of mean-free images (lag 0 zeroed), the
// proposal network's shift-invariant input: imgs [n][ny][nx] float ->
// out [n][ny][nx] float; scratch rows/spec/cols [n][nx/2+1][ny] double2,
// a64 [n][ny][nx] double.
hipError_t launch_autocorr(hipStream_t s, const float* imgs, int n, int nx, int ny, double2* rows_scratch,
                           double2* spec64, double2* cols_scratch, double* a64, float* out);

// Likelihood support.
hipError_t launch_ctf_table(hipStream_t s, const double* ctf, int nc, int nx, int ny, double pixel,
                            float* table);
hipError_t launch_proj_norms(hipStream_t s, const float2* pspec, const int32_t* pexpo, int nq,
                             const float* table, int nc, int nx, int ny, double* B);

struct LogpostArgs {
  const float2* ispec; const int32_t* iexpo; const double* istats; int ni;   // image chunk
  const float2* pspec; const int32_t* pexpo; int nq;                        // all projections
  const float* table; const double* B; int nc;
  const float4* itile; const float4* ptile; const float4* ttile;          // fragment-order copies
  int nx, ny, S, ldy;              // ldy = spec_ld(ny)
  const int32_t* cand; int k;     // [ni][k] chunk-relative rows, or null
  bioem_erec* rec;                // [ni][nq or k][nc]
  double kscale;                  // (2^e_i 2^e_q / n)^2 kappa factor: 1 / n^2
  int zs;                         // split forms: ttile holds the CTF values times 2^zs
};
hipError_t launch_logpost_f32(hipStream_t s, const LogpostArgs& a);
// Recompute the argmax displacement (FP32 transform) of best[i]'s (q, c).
hipError_t launch_best_shift(hipStream_t s, const LogpostArgs& a, bioem_best* best);
size_t f32_smem_bytes(int nx, int ny, int S);
constexpr size_t kMaxSmem = 160 * 1024;
// Split-precision kernel, one job.  shape: compiled launch variant; ti, ts:
// item tile (images x orientation slots), 0 = default.
hipError_t launch_logpost_split(hipStream_t s, const LogpostArgs& a, bool bf16, int shape, int ti, int ts);
int split_num_shapes();
// The default one-wave-per-SIMD variant with ew CTF sets per item, and the
// item width of a variant.
int split_shape_for_ew(int ew, bool bf16);
int split_shape_ew(int shape);
// One persistent launch over several jobs; ew in {2, 4} CTF sets per item.
struct BatchJob {
  LogpostArgs a;
  int ew, ti, ts;
};
hipError_t launch_logpost_batch(hipStream_t s, const BatchJob* jobs, int njobs, bool bf16);
bool split_supported(int nx, int ny, int S);

// Plain FP32 form on the FP32 matrix cores (factored transform).  Orbit-order
// copies: mf_len(nx, ny) float4 per spectrum (images with the DC coefficient
// zeroed), mf_table_len(nx, ny) float4 per CTF table.
size_t mf_len(int nx, int ny);
size_t mf_table_len(int nx, int ny);
size_t mf32_smem_bytes(int nx, int ny);
bool mf32_supported(int nx, int ny, int S);
hipError_t launch_mf_copy_spec(hipStream_t s, const float2* spec, int n, int nx, int ny, bool zero_dc,
                               float4* out);
hipError_t launch_mf_copy_table(hipStream_t s, const float* table, int nc, int nx, int ny, float4* out);
// Operand tables of one (box, shift window): mf32_table_len float4.
size_t mf32_table_len(int nx, int ny);
hipError_t launch_mf_tables(hipStream_t s, int nx, int ny, int S, float4* tabs);
// a.rec receives one record per evaluation (d = -1: the best displacement is
// recovered afterwards); im: the chunk's image copies; ti, ts: item tile
// (images x orientation slots), 0 = default.
hipError_t launch_logpost_mf32(hipStream_t s, const LogpostArgs& a, const float4* im, const float4* pm,
                               const float4* tm, const float4* tabs, int ti, int ts);

// Per image: FP64 likelihood terms from the per-evaluation records, LSE over
// orientations, CTF sets and shifts, best grid point, per-orientation LSE.
struct FinalizeArgs {
  const bioem_erec* rec; int ni, nslots, nc, nq_total, nx, ny, S;
  const int32_t* cand; int k;     // [ni][k] chunk-relative, or null
  const double* istats; const int32_t* iexpo; const int32_t* pexpo; const double* B;
  double log_prior;
  double* logp; bioem_best* best; double* orient;
};
hipError_t launch_finalize(hipStream_t s, const FinalizeArgs& f);

// Real-space variant with border cropping (small windows, S <= kCropMaxShift).
// Calculated images p [np][ny][nx] float (index = c * nq + q), images
// [ni][ny][nx] float with stats [ni][3]; Bd [np][W] and rec [ni][np] scratch.
struct bioem_crec {
  double lmax;    // window maximum of l(d)
  double rel;     // sum_d exp(l(d) - lmax), in [1, W]
  int32_t d;      // (dy+S)*(2S+1) + (dx+S) of the maximum; -1: no valid d
  int32_t pad;
};
constexpr int kCropMaxShift = 3;
struct CropArgs {
  const float* imgs; const double* stats; int ni;
  const float* p; int np, nq;
  int nx, ny, S;
  double* Bd;
  bioem_crec* rec;
};
size_t crop_smem_bytes(int nx, int S);
hipError_t launch_crop_norms(hipStream_t s, const CropArgs& a);
hipError_t launch_crop_xcorr(hipStream_t s, const CropArgs& a);
hipError_t launch_crop_finalize(hipStream_t s, const CropArgs& a, double log_prior, double* logp,
                                bioem_best* best);

// Ensemble posterior over models (weights w [nm], device): per [ni] and
// total [1] from logp [nm][ni]; per may only be null when ni == 0.
hipError_t launch_ensemble(hipStream_t s, const double* logp, int nm, int ni, const double* w, double* per,
                           double* total);

}  // namespace bioem

// ---- device helpers ---------------------------------------------------------
#define BIOEM_DEV static __device__ __forceinline__

// Stored spectrum columns (and CTF table columns) are padded with zeros to a
// multiple of 32 rows, the K-step of the matrix-core transform.
__host__ __device__ static inline int spec_ld(int ny) { return (ny + 31) & ~31; }
// Column tiles (16 columns below nx/2) and row steps (32 rows) of the split kernel.
__host__ __device__ static inline int split_mt(int nx) { return (nx / 2 + 15) / 16; }
__host__ __device__ static inline int split_ks(int ny) { return (ny + 31) / 32; }
__host__ __device__ static inline size_t tile_spec_len(int nx, int ny) {
  return (size_t)split_mt(nx) * split_ks(ny) * 4 * 64;
}
__host__ __device__ static inline size_t tile_table_len(int nx, int ny) {
  return (size_t)split_mt(nx) * split_ks(ny) * 2 * 64;
}

// exp(2 pi i t / n) in FP64 with the argument reduced exactly (t in [0, n)).
BIOEM_DEV double2 twiddle64(long t, int n) {
  double s, c;
  sincospi(2.0 * (double)t / (double)n, &s, &c);
  return make_double2(c, s);
}
