/*
 * bioem.h - C ABI of the MI355X (gfx950) BioEM posterior engine.
 *
 * Computes, for every particle image omega and model m, the posterior of the
 * model given the image (Eq. Pmom of Cossio, Rohr et al., "BioEM:
 * GPU-accelerated computing of Bayesian inference of electron microscopy
 * images"): the likelihood of Eq. (likeli) integrated analytically over
 * normalisation N, offset mu and noise lambda, and numerically over a grid of
 * orientations (quaternions), CTF/envelope parameter sets (a, A, b) and
 * in-plane displacements d with |dx|, |dy| <= S.
 *
 * Conventions shared by every call
 *   - Images are row-major [ny][nx] float32; pixel (j, k) is centred at
 *     ((j - nx/2) * pixel, (k - ny/2) * pixel) in Angstrom.
 *   - Quaternions are (w, x, y, z), active rotation about the model origin.
 *   - Fourier transforms: forward exp(-2 pi i (l k/ny + m j/nx)), inverse with
 *     1/(nx ny) (the paper's Eqs. 1-2 read as the standard 0-based DFT).
 *   - The displacement enters as I_cal(r) = N I1(r + d) - mu (Section 2), with
 *     indices taken modulo the box, which is the Fourier variant of Section 3
 *     (Center displacement).
 *   - Priors: flat in mu and N, 1/lambda in lambda, uniform normalised over the
 *     orientation, CTF and shift grids, so
 *       log P = ln sum_{q,c,d} exp(l(q,c,d)) - ln(Nq Nc Nd)
 *     with l(q,c,d) = lgamma(n/2-1) - ln 2 - ln(n)/2 + (1-n/2) ln(pi A)
 *                     - ln(B_qc)/2 + (1-n/2) log1p(-X(d)^2/(A B_qc)),
 *     A = sum (I - mean)^2 of the image, B_qc the same of the calculated
 *     image, X(d) their cross-correlation at shift d.  Values are relative:
 *     the paper's posterior is defined up to a constant (Section 5).
 *
 * Memory and streams
 *   - Every array argument is borrowed for the duration of the call; it is
 *     host memory or device memory (a pointer valid on the context's device)
 *     as the accompanying bioem_mem value says.
 *   - The opaque handles bioem_proj / bioem_imgs own device arrays until
 *     bioem_free_proj / bioem_free_imgs.
 *   - All device work is enqueued on the context's stream.  A call that
 *     writes host memory synchronises the stream before returning; a call
 *     that writes device memory returns after enqueueing.
 *
 * Errors
 *   - Every entry point returns a bioem_status; no C++ exception crosses the
 *     ABI.  Arguments are validated before any work is enqueued.  On failure
 *     bioem_last_error(ctx) describes the cause (valid until the next call on
 *     the same context).  Per-image degeneracy (an image with zero variance,
 *     or no calculated image with non-zero variance) is not an error: that
 *     image gets status 1 and log P = NaN.
 *   - One context per host thread; calls on one context are not thread-safe.
 */
#ifndef BIOEM_H
#define BIOEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bioem_ctx bioem_ctx;
typedef struct bioem_proj bioem_proj;
typedef struct bioem_imgs bioem_imgs;

typedef enum {
  BIOEM_OK = 0,
  BIOEM_EINVAL = -1,        /* invalid argument (sizes, ranges, non-finite values) */
  BIOEM_ENOMEM = -2,        /* device allocation failed */
  BIOEM_EDEVICE = -3,       /* HIP runtime error or kernel fault */
  BIOEM_EUNSUPPORTED = -4   /* valid but outside what the library supports */
} bioem_status;

typedef enum { BIOEM_MEM_HOST = 0, BIOEM_MEM_DEVICE = 1 } bioem_mem;

/* How the inverse transforms of the cross-correlation are computed.
 *   F32:        plain FP32: FP32 operands and accumulation throughout, on the
 *               FP32 matrix cores (factored pruned transform) where the
 *               shift window allows, else a direct pruned transform on the
 *               vector ALUs (bioem_opts.kernel selects).
 *   SPLIT_F16:  DFT-as-GEMM on the matrix cores; each FP32 operand is split
 *               into fp16 hi + lo parts, three products, FP32 accumulation
 *               (about 22 significant bits for operands in fp16's normal
 *               range; the operands are scaled up by a power of two as far as
 *               the stage-1 sums allow).
 *   SPLIT_BF16: the same with bfloat16 hi + lo parts (about 16 bits).
 * The error of log P from a relative error e of the correlation grows as
 * n rho^2 / (1 - rho^2) e for n pixels: on boxes up to 224 x 224 both split
 * forms stay within 0.1 nat of the FP64 result; on the largest box (512 x 512,
 * SNR 0.5) SPLIT_F16 is off by a few 1e-2 nat and SPLIT_BF16 by about 1.4 nat,
 * so large boxes want F32 (5e-3 nat there) or SPLIT_F16.
 * In every mode the likelihood constants, log1p and the log-sum-exp are FP64
 * (the per-image constants reach ~1e5 nat at 224^2, Section 3 Numerical
 * precision notwithstanding). */
typedef enum {
  BIOEM_PREC_F32 = 0,
  BIOEM_PREC_SPLIT_BF16 = 1,
  BIOEM_PREC_SPLIT_F16 = 2
} bioem_prec;

/* Maximising grid parameters of one image (Section 3, Extra features). */
typedef struct {
  double logl;     /* maximal log-likelihood l(q,c,d) */
  int32_t q;       /* orientation index into the projection set */
  int32_t c;       /* CTF set index */
  int32_t dx, dy;  /* displacement in pixels, |dx|,|dy| <= S */
  int32_t status;  /* 0 ok, 1 degenerate image (log P = NaN) */
} bioem_best;

typedef struct {
  int32_t prec;            /* bioem_prec; 0 = F32 */
  int32_t out_mem;         /* bioem_mem of logp, best and logp_orient */
  /* Optional per-image candidate orientations (a proposal): cand_q is
   * [ni][k] int32 indices into the projection set; only those orientations
   * are evaluated, and log P keeps the full-grid prior -ln Nq, so it is a
   * lower bound of the exhaustive value.  NULL evaluates the full grid. */
  const int32_t* cand_q;
  int32_t k;
  int32_t cand_mem;        /* bioem_mem of cand_q */
  /* Optional [ni][nq] output: log posterior restricted to each orientation
   * (LSE over CTF sets and shifts, same prior), Section 3 Extra features.
   * Entries not evaluated under a proposal are -inf. */
  double* logp_orient;
  /* Kernel form, for comparisons and sweeps (0 = the library's choice).
   *   F32:   1 = FP32 matrix-core form with the factored transform (the
   *          default where supported: 0 <= S <= 31), 2 = direct pruned
   *          transform on the vector ALUs (any S);
   *   split: 1 + launch-shape index (bioem_tuning_count lists the tuned ones).
   * An unsupported choice returns BIOEM_EUNSUPPORTED. */
  int32_t kernel;
  /* Item tile (images x orientation slots walked together for cache reuse)
   * of the matrix-core kernels; 0 = default (or the autotuned tile). */
  int32_t tile_images;
  int32_t tile_slots;
  int32_t reserved;        /* must be zero */
} bioem_opts;

/* Create a context on HIP device `device`.  `hip_stream` is the hipStream_t
 * every call enqueues on; NULL means the device's null (legacy default)
 * stream, so work that other code enqueues there (a framework's default
 * stream) is ordered with the library's.  Inputs in device memory must be
 * complete in the order of that stream when a call is made. */
bioem_status bioem_create(int device, void* hip_stream, bioem_ctx** out);
void bioem_destroy(bioem_ctx* ctx);
const char* bioem_last_error(const bioem_ctx* ctx);
/* Version string of the library build. */
const char* bioem_version(void);

/* Fourier-space projections of a Gaussian-sphere model (Section 2, Eq. ideal;
 * Section 3, Model rotation).
 *   spheres [ns][5] float64: centre x, y, z (A), width sigma (A), weight
 *           (integral of the normalised 3-D Gaussian);
 *   quats   [nq][4] float64 unit quaternions (w, x, y, z);
 *   nx, ny  even box size in pixels (4 <= n <= 512); pixel_A > 0 (kept with
 *           the handle: it also sets the CTF frequency scale in bioem_logpost).
 * ns >= 1 and nq >= 1: an empty model or grid is BIOEM_EINVAL.
 * Each projection is I0[k][j] = sum_a w_a Ey_a[k] Ex_a[j] with pixel-box
 * integrals of the rotated Gaussians (FP64), then its half-spectrum DFT,
 * stored on the device twice: column-major, and in the matrix-fragment order
 * that the split-precision posterior reads (about 2 x 8 (nx/2+1) ny bytes per
 * projection in all).  *out must be released with bioem_free_proj. */
bioem_status bioem_project(bioem_ctx* ctx, const double* spheres, int32_t ns,
                           const double* quats, int32_t nq, int32_t nx, int32_t ny,
                           double pixel_A, bioem_mem in_mem, bioem_proj** out);

/* Observed images (Section 3: the spectra and per-image sums C_o, C_oo are
 * precalculated).  imgs is [ni][ny][nx] float32.  Computes, in FP64 from the
 * pixels, C_o = sum I, C_oo = sum I^2 and A = sum (I - C_o/n)^2, and the
 * half-spectrum DFT of each image (stored twice, as for bioem_project).
 * ni >= 1 (no images is BIOEM_EINVAL); a NaN or infinite pixel is
 * BIOEM_EINVAL before anything is enqueued.
 * *out must be released with bioem_free_imgs. */
bioem_status bioem_prepare_images(bioem_ctx* ctx, const float* imgs, int32_t ni, int32_t nx,
                                  int32_t ny, bioem_mem in_mem, bioem_imgs** out);

/* Per-image log posterior over orientations x CTF sets x shifts (Eq. Pmom,
 * Listing 1).  ctf is [nc][3] float64 (a in A^2, A in [0,1], b in A^2) of
 * CTF(s|a,A) Env(s|b) (Section 2); ctf is host or device per `ctf_mem`.
 * nc >= 1 (no CTF sets is BIOEM_EINVAL).
 * max_shift = S with 0 <= S < min(nx, ny)/2.  Outputs: logp [ni] float64 and
 * best [ni] (either may be NULL), and optional opts->logp_orient.  opts may
 * be NULL (F32, host outputs, full grid). */
bioem_status bioem_logpost(bioem_ctx* ctx, const bioem_proj* proj, const bioem_imgs* imgs,
                           const double* ctf, int32_t nc, bioem_mem ctf_mem, int32_t max_shift,
                           const bioem_opts* opts, double* logp, bioem_best* best);

/* Allocation-free form of bioem_logpost, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  It computes exactly what
 * bioem_logpost computes with opts = NULL except for where results go: plain
 * F32 with the library's kernel choice, full orientation grid, no
 * per-orientation output.
 *   ctf [nc][3] float64 in HOST memory (validated there, then copied into
 *   the scratch on the context's stream); logp [ni] float64 and best [ni] in
 *   DEVICE memory on the context's device (either may be NULL).
 * Every intermediate (CTF tables, projection norms, matrix-core operand
 * tables, per-evaluation records) lives in one fixed 64 MiB scratch array
 * per device, which the library holds from its load until the process ends;
 * images are processed in chunks that fit it.  No hipMalloc, hipFree or
 * event creation happens in the call (bioem_set_timing does not apply).
 * Returns after enqueueing.  Every call on a device shares that device's
 * scratch and leaves its contents behind: calls ordered on one stream are
 * safe, calls that overlap on one GPU (other streams or contexts) race.
 * Errors: as bioem_logpost, plus BIOEM_EUNSUPPORTED when the tables and one
 * image's records (16 B per orientation x CTF set) exceed the 64 MiB, and
 * BIOEM_EDEVICE when the scratch address could not be resolved at
 * bioem_create. */
bioem_status bioem_logpost_noalloc(bioem_ctx* ctx, const bioem_proj* proj, const bioem_imgs* imgs,
                                   const double* ctf, int32_t nc, int32_t max_shift, double* logp,
                                   bioem_best* best);

/* One job of a batched call: a projection set and an image set of the same
 * box, their CTF grid and shift window, an optional proposal, and outputs.
 * Field meanings are those of bioem_logpost's arguments and options. */
typedef struct {
  const bioem_proj* proj;
  const bioem_imgs* imgs;
  const double* ctf;       /* [nc][3], host or device per ctf_mem */
  int32_t nc;
  int32_t ctf_mem;
  int32_t max_shift;
  int32_t k;               /* candidates per image (with cand_q) */
  const int32_t* cand_q;   /* [ni][k] or NULL for the full grid */
  int32_t cand_mem;
  int32_t reserved;        /* must be zero */
  double* logp;            /* [ni] or NULL */
  bioem_best* best;        /* [ni] or NULL */
  double* logp_orient;     /* [ni][nq] or NULL */
} bioem_job;

/* Batch modes. */
typedef enum {
  BIOEM_BATCH_PERSISTENT = 0,  /* every job's evaluations in one persistent launch */
  BIOEM_BATCH_PER_JOB = 1      /* one launch per job, in order (for comparison) */
} bioem_batch_mode;

/* Score several jobs (different boxes, shift windows, grids, models) with
 * results identical in meaning to one bioem_logpost per job.  With a split
 * precision and BIOEM_BATCH_PERSISTENT the per-evaluation work of all jobs
 * runs in ONE persistent kernel launch whose workgroups sweep the jobs'
 * concatenated work lists (each workgroup gets a near-equal share of every
 * job, so boxes of different cost balance); per-job CTF tables, norms and
 * the FP64 finalisation run as separate small launches.  With
 * BIOEM_PREC_F32 jobs run one after another whatever the mode.  prec and
 * out_mem apply to every job.  Every job is validated before any work is
 * enqueued; the job list is borrowed for the call. */
bioem_status bioem_logpost_batch(bioem_ctx* ctx, const bioem_job* jobs, int32_t njobs, int32_t prec,
                                 int32_t out_mem, int32_t mode);

/* Autotuning of the split-precision kernel's tile shape (CTF sets per wave
 * item, item tile of images x orientations).  While enabled, the first
 * bioem_logpost / bioem_logpost_batch call that meets a new key
 * (nx, ny, S, orientation-count bucket floor(log2 nq), precision) times every
 * candidate shape on a sample of that call's own work (up to 128 images x 2048
 * orientations) and keeps the fastest for the context's lifetime; later calls
 * with the key use it.  Disabled (the default): a fixed default shape.
 * Results do not depend on the shape beyond floating-point summation order. */
bioem_status bioem_set_autotune(bioem_ctx* ctx, int32_t enable);

/* A tuned entry: its key, the chosen shape and the sampled timings. */
typedef struct {
  int32_t nx, ny, max_shift, nq_log2, prec;
  int32_t ew;              /* CTF sets per wave item */
  int32_t tile_images;     /* item tile */
  int32_t tile_slots;
  double ns_per_eval;      /* chosen shape on the sample */
  double ns_per_eval_default;  /* default shape on the sample */
} bioem_tuning;

/* Number of tuned entries of ctx, and entry idx in [0, count). */
int32_t bioem_tuning_count(const bioem_ctx* ctx);
bioem_status bioem_tuning_entry(const bioem_ctx* ctx, int32_t idx, bioem_tuning* out);

/* ---- learned orientation proposal ------------------------------------------
 * A small BF16 convolutional network maps a particle image to logits over
 * the orientation grid; its top-K orientations per image are the candidate
 * list of bioem_logpost (opts.cand_q).  It is trained on the per-orientation
 * posteriors the method itself computes (Section 3, Extra features), by the
 * forward and backward kernels of this library (bf16 matrix-core products
 * with FP32 accumulation, FP32 master weights, Adam).
 *
 * Architecture (sizes from bioem_cnn_arch): per-image standardisation; four
 * 3x3 convolutions with stride 2 and zero padding 1 (1 -> c1 -> c2 -> c3 ->
 * c4 channels, ReLU); the c4 x (box/16)^2 final map flattened (index
 * c*P + p); a hidden layer of `hidden` units (ReLU); a linear layer to nq
 * logits.  Loss: mean soft-label cross entropy against sparse targets
 * (idx, p) per image.  Parameters are one flat FP32 vector:
 * W1 [c1][1][3][3], b1 [c1], W2 [c2][c1][3][3], b2, W3, b3, W4, b4,
 * F1 [hidden][c4 (box/16)^2], g1 [hidden], F2 [nq][hidden], g2 [nq].
 * Inputs are [B][box][box] float32 (normally bioem_cnn_input of the
 * particle images); box must be a multiple of 16 (16..512). */
typedef struct bioem_cnn bioem_cnn;

typedef struct {
  int32_t box, c1, c2, c3, c4, hidden, nq;
  int32_t reserved;        /* must be zero */
} bioem_cnn_arch;

/* Create a network on ctx's device with zero parameters; the caller sets
 * them (bioem_cnn_set_params).  Release with bioem_cnn_destroy. */
bioem_status bioem_cnn_create(bioem_ctx* ctx, const bioem_cnn_arch* arch, bioem_cnn** out);
void bioem_cnn_destroy(bioem_cnn* net);
int64_t bioem_cnn_num_params(const bioem_cnn* net);
/* Copy all parameters in / out (flat order above); setting them also resets
 * the optimiser state.  mem: bioem_mem of params. */
bioem_status bioem_cnn_set_params(bioem_ctx* ctx, bioem_cnn* net, const float* params, int32_t mem);
bioem_status bioem_cnn_get_params(bioem_ctx* ctx, const bioem_cnn* net, float* params, int32_t mem);
/* Logits [B][nq] of B images (internally in batches of up to 256). */
bioem_status bioem_cnn_forward(bioem_ctx* ctx, bioem_cnn* net, const float* imgs, int32_t B, int32_t in_mem,
                               float* logits, int32_t out_mem);
/* Loss and gradient of one batch (B <= 256): targets tidx [B][T] int32 and
 * tp [B][T] float32 (each row sums to 1), memory per in_mem like imgs.  The
 * gradient is kept in the network for bioem_cnn_adam and also copied to
 * grad [nparams] when grad is not NULL (per grad_mem).  *loss (host) is the
 * batch mean. */
bioem_status bioem_cnn_backward(bioem_ctx* ctx, bioem_cnn* net, const float* imgs, int32_t B,
                                const int32_t* tidx, const float* tp, int32_t T, int32_t in_mem, float* loss,
                                float* grad, int32_t grad_mem);
/* One Adam step (bias-corrected) with the last gradient. */
bioem_status bioem_cnn_adam(bioem_ctx* ctx, bioem_cnn* net, float lr, float beta1, float beta2, float eps);
/* Top-K orientations per image (K <= nq), in increasing index order, ties to
 * the lower index: cand [B][K] int32, and the softmax mass they hold
 * mass [B] float32 (NULL to skip); outputs per out_mem. */
bioem_status bioem_cnn_propose(bioem_ctx* ctx, bioem_cnn* net, const float* imgs, int32_t B, int32_t in_mem,
                               int32_t K, int32_t* cand, float* mass, int32_t out_mem);

/* The network's input for raw images: the circular autocorrelation of each
 * mean-free image, re-centred so that lag 0 sits at pixel (ny/2, nx/2), with
 * lag 0 itself set to 0 (it carries the noise power).  It does not change
 * when the particle is shifted (circularly) within the box, so the network
 * need not learn the in-plane displacement.  imgs [B][ny][nx] float32 ->
 * out [B][ny][nx] float32 (FP64 transforms), memory per in_mem / out_mem. */
bioem_status bioem_cnn_input(bioem_ctx* ctx, const float* imgs, int32_t B, int32_t nx, int32_t ny, int32_t in_mem,
                             float* out, int32_t out_mem);

/* Top-K of each row of z [B][n] float32 (host or device per in_mem): idx
 * [B][K] int32 in increasing index order (ties to the lower index) and the
 * softmax mass of the selection, mass [B] (NULL to skip), per out_mem.  With
 * z a per-orientation log posterior this is the posterior mass the K most
 * probable orientations hold (the proposal's training targets). */
bioem_status bioem_topk(bioem_ctx* ctx, const float* z, int32_t B, int32_t n, int32_t K, int32_t in_mem,
                        int32_t* idx, float* mass, int32_t out_mem);

/* Synthetic maps (Section 3, Extra features): one calculated image per
 * projection, I_cal(r) = N I1(r + d) - mu + sigma eps with
 * I1 = F^-1[F(I0) CTF Env] and sigma^2 = var(I1)/snr.
 *   proj holds ni projections (one per image); ctf [ni][3]; shifts [ni][2]
 *   int32 (dx, dy); norm_offset [ni][2] (N, mu) or NULL for (1, 0); noise
 *   [ni][ny][nx] float32 standard-normal draws or NULL for none (snr is then
 *   ignored).  Inputs are host or device per in_mem; out [ni][ny][nx] float32
 *   per out_mem. */
bioem_status bioem_render(bioem_ctx* ctx, const bioem_proj* proj, const double* ctf,
                          const int32_t* shifts, const double* norm_offset, const float* noise,
                          double snr, bioem_mem in_mem, float* out, bioem_mem out_mem);

/* Kernel timing: while enabled, bioem_logpost records HIP events around each
 * launch of its main (per-evaluation) kernel on the context's stream.
 * bioem_get_kernel_time waits for those events and returns the summed
 * duration in milliseconds and the number of launches since timing was last
 * enabled, plus the number of evaluations (image x orientation x CTF set)
 * they covered.  bioem_set_timing resets the totals.  Used by benchmarks to
 * price the kernel against its roofline. */
bioem_status bioem_set_timing(bioem_ctx* ctx, int32_t enable);
bioem_status bioem_get_kernel_time(bioem_ctx* ctx, double* ms, int32_t* launches, double* evals);

/* Projections for orientations given as Euler angles, the other
 * representation of Section 3 (Model rotation): euler [nq][3] (phi, theta,
 * psi) in radians, z-y-z intrinsic, i.e. the rotation Rz(phi) Ry(theta)
 * Rz(psi) of the model about its origin.  The angles are turned into unit
 * quaternions on the device and projected exactly as bioem_project does;
 * arguments, ownership and errors as there (EINVAL also for a non-finite
 * angle).  A symmetry-restricted search passes the restricted angle set. */
bioem_status bioem_project_euler(bioem_ctx* ctx, const double* spheres, int32_t ns, const double* euler, int32_t nq,
                                 int32_t nx, int32_t ny, double pixel_A, bioem_mem in_mem, bioem_proj** out);

/* Real-space variant of the displacement sum (Section 3, Center
 * displacement) with border cropping instead of the Fourier variant's wrap:
 * the calculated image moved by d keeps I1(r + d) where r + d lies in the
 * box and is 0 elsewhere, so its centred sum of squares B(d) depends on d;
 * everything else is as in bioem_logpost (Eq. likeli integrated over offset,
 * scale and noise; uniform grid priors; FP64 likelihood and sums).  The
 * correlation is direct, (2S+1)^2 multiply-adds per pixel and evaluation
 * (FP32 products, FP32 row sums added in FP64), so this form is for small
 * windows: max_shift <= 3.
 *   proj: nq projections (bioem_project); imgs [ni][ny][nx] float32 raw
 *   pixels of the same box (not a bioem_imgs handle: the direct form reads
 *   pixels), host or device per in_mem; ctf [nc][3] (a, A, b) per in_mem;
 *   logp [ni] and best [ni] per out_mem (best.logl is the maximal l, ties
 *   to the lowest (q, c, dy, dx)).
 * Device memory used: nq*nc calculated images (4 B per pixel) plus records
 * of at most 1 GiB.  Returns after the results are written.
 * EINVAL: bad pointers, sizes or memory kinds, max_shift < 0 or
 * 2*max_shift >= min(nx, ny), non-finite CTF values or A outside [0, 1].
 * EUNSUPPORTED: max_shift > 3, or a box too wide for the kernel's LDS
 * staging at that window (32 rows of nx + 1 floats and p x (2S+1) rows of
 * nx + 2S floats within 160 KB, p = 32, 16, 8, 8 for S = 0, 1, 2, 3). */
bioem_status bioem_logpost_crop(bioem_ctx* ctx, const bioem_proj* proj, const float* imgs, int32_t ni,
                                int32_t in_mem, const double* ctf, int32_t nc, int32_t max_shift, double* logp,
                                bioem_best* best, int32_t out_mem);

/* bioem_logpost_crop with the calculated images built by the real-space
 * convolution of Eq. (5) instead of the Fourier filter of Eq. (4) (Section 3,
 * Imaging effects: the real-space form pays off when the PSF is negligible
 * away from the origin).  For each CTF set the PSF is the inverse transform
 * of CTF x Env on the box grid (Eq. 3, FP64), truncated to the disc
 * dx^2 + dy^2 <= psf_radius^2; each ideal projection I0 (FP64) is convolved
 * with it on the box without wrap (pixels outside the box count as zero),
 *   I1(x, y) = sum_{dx,dy} PSF(dx, dy) I0(x - dx, y - dy),
 * in FP64 and stored as FP32; the cropped displacement sum and everything
 * after it are those of bioem_logpost_crop.  Near the borders the result
 * differs from the Fourier filter, which wraps; away from them it agrees to
 * the part of the PSF beyond the radius.
 * Arguments as bioem_logpost_crop, plus psf_radius in [0, min(nx, ny)/2).
 * EINVAL: as bioem_logpost_crop, or psf_radius outside that range.
 * EUNSUPPORTED: as bioem_logpost_crop, or psf_radius > 32.
 * Device memory used beyond bioem_logpost_crop's: nc PSF images (8 B per
 * pixel, with their transform scratch) and nc (2 psf_radius + 1)^2 kernel
 * values. */
bioem_status bioem_logpost_crop_psf(bioem_ctx* ctx, const bioem_proj* proj, const float* imgs, int32_t ni,
                                    int32_t in_mem, const double* ctf, int32_t nc, int32_t max_shift,
                                    int32_t psf_radius, double* logp, bioem_best* best, int32_t out_mem);

/* Posterior of a model ensemble, Eq. (pb2) of Section 2: models m = 0..nm-1
 * with relative weights w_m (w_m >= 0, summing to 1 within 1e-9) and the
 * per-image log posteriors logp[m][i] that bioem_logpost returns for each
 * model on the same ni images (same grid sizes, so the priors match):
 *   per_image[i] = ln sum_m w_m exp(logp[m][i]),
 *   total        = sum_i per_image[i],
 * the log of Eq. (pb2)'s product over independent images (up to the same
 * constant as the per-model values).  With one weight equal to 1, total is
 * that model's log evidence over the set; differences of such totals are log
 * Bayes factors between models.  FP64; the largest weighted term is taken
 * out before the exponentials; total is summed in a fixed order
 * (deterministic).  Models with w_m = 0 take no part (also when their logp
 * is NaN, e.g. a degenerate image); a NaN among the others makes that image's
 * value NaN, and total follows IEEE rules (NaN, or +-inf).
 *   logp [nm][ni] float64, host or device per in_mem (may be NULL if ni = 0);
 *   w [nm] float64, always host memory;
 *   per_image [ni] (NULL to skip) and total [1] float64 per out_mem.
 * ni = 0 gives total = 0.  Returns after the results are written.
 * EINVAL: nm < 1, ni < 0, a NULL array that is needed, a bad memory kind, a
 * negative or non-finite weight, weights not summing to 1. */
bioem_status bioem_ensemble(bioem_ctx* ctx, const double* logp, int32_t nm, int32_t ni, int32_t in_mem,
                            const double* w, double* per_image, double* total, int32_t out_mem);

void bioem_free_proj(bioem_proj* p);
void bioem_free_imgs(bioem_imgs* p);

/* Sizes of a handle: *n items of nx x ny pixels. */
bioem_status bioem_proj_info(const bioem_proj* p, int32_t* n, int32_t* nx, int32_t* ny);
bioem_status bioem_imgs_info(const bioem_imgs* p, int32_t* n, int32_t* nx, int32_t* ny);

/* Map physical CTF parameters to the paper's (a, A, b): with s = 2 pi k and
 * electron wavelength lambda(voltage), a = lambda defocus / (2 pi) and
 * b = B / (8 pi^2), A = amplitude contrast.  Defocus > 0 is underfocus. */
bioem_status bioem_ctf_from_physical(double defocus_A, double amp_contrast, double bfactor_A2,
                                     double voltage_kV, double out_abA[3]);

#ifdef __cplusplus
}
#endif

#endif /* BIOEM_H */
