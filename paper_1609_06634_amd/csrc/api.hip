// Host side of the C ABI: argument validation, device memory, chunking and
// launch order.  All device work goes to the context's stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"

using namespace bioem;

namespace {

constexpr size_t kScratchBudget = size_t(256) << 20;   // per transform chunk
constexpr size_t kRecordBudget = size_t(1) << 30;      // per posterior image chunk

bioem_status fail(bioem_ctx* ctx, bioem_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define HIP_OR_FAIL(ctx, expr)                                                              \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, e_ == hipErrorOutOfMemory ? BIOEM_ENOMEM : BIOEM_EDEVICE, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                            \
  } while (0)

// Device buffer that frees itself.
struct DevMem {
  void* p = nullptr;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// A borrowed input made available on the device: used in place when it is
// device memory, copied (stream-ordered) when it is host memory.
struct DevIn {
  DevMem own;
  const void* d = nullptr;
  hipError_t set(const void* src, size_t bytes, bioem_mem mem, hipStream_t s) {
    if (!src) { d = nullptr; return hipSuccess; }
    if (mem == BIOEM_MEM_DEVICE) { d = src; return hipSuccess; }
    hipError_t e = own.alloc(bytes);
    if (e != hipSuccess) return e;
    d = own.p;
    return hipMemcpyAsync(own.p, src, bytes, hipMemcpyHostToDevice, s);
  }
  template <class T> const T* as() const { return static_cast<const T*>(d); }
};

// Small inputs are validated on the host; device ones are copied back first.
template <class T>
hipError_t to_host(const T* src, size_t count, bioem_mem mem, hipStream_t s, std::vector<T>& out) {
  out.resize(count);
  if (count == 0) return hipSuccess;
  if (mem == BIOEM_MEM_HOST) {
    std::memcpy(out.data(), src, count * sizeof(T));
    return hipSuccess;
  }
  hipError_t e = hipMemcpyAsync(out.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

bool valid_mem(int m) { return m == BIOEM_MEM_HOST || m == BIOEM_MEM_DEVICE; }

bool valid_box(int nx, int ny) {
  return nx >= 4 && ny >= 4 && nx <= kMaxBox && ny <= kMaxBox && nx % 2 == 0 && ny % 2 == 0;
}

// Items per transform chunk so that the FP64 scratch stays within budget.
// Launch shape of the split kernel: BIOEM_SPLIT_SHAPE overrides the default.
int split_shape_for(bioem_ctx* ctx, int nx, int ny, int S, int nc) {
  (void)ctx; (void)nx; (void)ny; (void)S; (void)nc;
  const char* env = std::getenv("BIOEM_SPLIT_SHAPE");
  if (env) {
    const int v = std::atoi(env);
    if (v >= 0 && v < split_num_shapes()) return v;
  }
  return 3;
}

int chunk_items(int n, size_t per_item) {
  size_t c = kScratchBudget / (per_item ? per_item : 1);
  if (c < 1) c = 1;
  return (int)std::min<size_t>(c, (size_t)n);
}

}  // namespace

extern "C" {

const char* bioem_version(void) { return "bioem-mi355x 0.1 (gfx950)"; }

bioem_status bioem_create(int device, void* hip_stream, bioem_ctx** out) {
  if (!out) return BIOEM_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BIOEM_EDEVICE;
  bioem_ctx* ctx = new (std::nothrow) bioem_ctx;
  if (!ctx) return BIOEM_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return BIOEM_EDEVICE; }
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return BIOEM_EDEVICE;
    }
    ctx->own_stream = true;
  }
  *out = ctx;
  return BIOEM_OK;
}

void bioem_destroy(bioem_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto e : ctx->ev_start) (void)hipEventDestroy(e);
  for (auto e : ctx->ev_stop) (void)hipEventDestroy(e);
  if (ctx->own_stream && ctx->stream) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
}

const char* bioem_last_error(const bioem_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

bioem_status bioem_set_timing(bioem_ctx* ctx, int32_t enable) {
  if (!ctx) return BIOEM_EINVAL;
  ctx->timing = enable != 0;
  ctx->ev_used = 0;
  ctx->timed_evals = 0.0;
  return BIOEM_OK;
}

bioem_status bioem_get_kernel_time(bioem_ctx* ctx, double* ms, int32_t* launches, double* evals) {
  if (!ctx) return BIOEM_EINVAL;
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  double total = 0.0;
  for (int i = 0; i < ctx->ev_used; ++i) {
    HIP_OR_FAIL(ctx, hipEventSynchronize(ctx->ev_stop[i]));
    float t = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&t, ctx->ev_start[i], ctx->ev_stop[i]));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = ctx->ev_used;
  if (evals) *evals = ctx->timed_evals;
  return BIOEM_OK;
}

void bioem_free_proj(bioem_proj* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->spec) (void)hipFree(p->spec);
  if (p->expo) (void)hipFree(p->expo);
  delete p;
}

void bioem_free_imgs(bioem_imgs* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->spec) (void)hipFree(p->spec);
  if (p->expo) (void)hipFree(p->expo);
  if (p->stats) (void)hipFree(p->stats);
  delete p;
}

bioem_status bioem_proj_info(const bioem_proj* p, int32_t* n, int32_t* nx, int32_t* ny) {
  if (!p) return BIOEM_EINVAL;
  if (n) *n = p->n;
  if (nx) *nx = p->nx;
  if (ny) *ny = p->ny;
  return BIOEM_OK;
}

bioem_status bioem_imgs_info(const bioem_imgs* p, int32_t* n, int32_t* nx, int32_t* ny) {
  if (!p) return BIOEM_EINVAL;
  if (n) *n = p->n;
  if (nx) *nx = p->nx;
  if (ny) *ny = p->ny;
  return BIOEM_OK;
}

bioem_status bioem_ctf_from_physical(double defocus_A, double amp_contrast, double bfactor_A2,
                                     double voltage_kV, double out_abA[3]) {
  if (!out_abA || !std::isfinite(defocus_A) || !std::isfinite(bfactor_A2) ||
      !(amp_contrast >= 0.0 && amp_contrast <= 1.0) || !(voltage_kV > 0.0) || !std::isfinite(voltage_kV))
    return BIOEM_EINVAL;
  // relativistic electron wavelength lambda = h / sqrt(2 m0 e V (1 + e V / (2 m0 c^2)))
  const double h = 6.62607015e-34, m0 = 9.1093837015e-31, e = 1.602176634e-19, c = 299792458.0;
  const double v = voltage_kV * 1e3;
  const double lam = h / std::sqrt(2.0 * m0 * e * v * (1.0 + e * v / (2.0 * m0 * c * c))) * 1e10;
  out_abA[0] = lam * defocus_A / (2.0 * M_PI);
  out_abA[1] = amp_contrast;
  out_abA[2] = bfactor_A2 / (8.0 * M_PI * M_PI);
  return BIOEM_OK;
}

bioem_status bioem_project(bioem_ctx* ctx, const double* spheres, int32_t ns, const double* quats,
                           int32_t nq, int32_t nx, int32_t ny, double pixel_A, bioem_mem in_mem,
                           bioem_proj** out) {
  if (!ctx) return BIOEM_EINVAL;
  if (!out) return fail(ctx, BIOEM_EINVAL, "bioem_project: out is NULL");
  *out = nullptr;
  if (!spheres || !quats || ns < 1 || nq < 1)
    return fail(ctx, BIOEM_EINVAL, "bioem_project: need ns >= 1 spheres and nq >= 1 quaternions");
  if (!valid_box(nx, ny))
    return fail(ctx, BIOEM_EINVAL, "bioem_project: box %dx%d must be even and within [4, %d]", nx, ny, kMaxBox);
  if (!(pixel_A > 0.0) || !std::isfinite(pixel_A))
    return fail(ctx, BIOEM_EINVAL, "bioem_project: pixel size must be positive and finite");
  if (!valid_mem(in_mem)) return fail(ctx, BIOEM_EINVAL, "bioem_project: bad in_mem");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<double> hs, hq;
  HIP_OR_FAIL(ctx, to_host(spheres, (size_t)ns * 5, in_mem, s, hs));
  HIP_OR_FAIL(ctx, to_host(quats, (size_t)nq * 4, in_mem, s, hq));
  if (!finite_all(hs.data(), hs.size()) || !finite_all(hq.data(), hq.size()))
    return fail(ctx, BIOEM_EINVAL, "bioem_project: non-finite sphere or quaternion value");
  for (int a = 0; a < ns; ++a)
    if (!(hs[5 * a + 3] > 0.0)) return fail(ctx, BIOEM_EINVAL, "bioem_project: sphere %d has sigma <= 0", a);
  for (int q = 0; q < nq; ++q) {
    const double* v = &hq[4 * q];
    if (!(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3] > 0.0))
      return fail(ctx, BIOEM_EINVAL, "bioem_project: quaternion %d is zero", q);
  }
  DevIn dsp, dq;
  HIP_OR_FAIL(ctx, dsp.set(hs.data(), hs.size() * 8, BIOEM_MEM_HOST, s));
  HIP_OR_FAIL(ctx, dq.set(hq.data(), hq.size() * 8, BIOEM_MEM_HOST, s));

  const int mh = nx / 2 + 1;
  const size_t len = (size_t)mh * ny, slen = (size_t)mh * spec_ld(ny);
  bioem_proj* p = new (std::nothrow) bioem_proj;
  if (!p) return fail(ctx, BIOEM_ENOMEM, "bioem_project: host allocation");
  p->n = nq; p->nx = nx; p->ny = ny; p->pixel = pixel_A; p->device = ctx->device;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->spec), sizeof(float2) * slen * nq);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->expo), sizeof(int32_t) * nq);
  if (e != hipSuccess) {
    bioem_free_proj(p);
    return fail(ctx, BIOEM_ENOMEM, "bioem_project: device allocation of %zu MB failed",
                (sizeof(float2) * slen * nq) >> 20);
  }
  const size_t per = (size_t)nx * ny * 8 + (size_t)ny * mh * 16 + len * 16;
  const int chunk = chunk_items(nq, per);
  DevMem i0, rows, s64;
  e = i0.alloc((size_t)chunk * nx * ny * 8);
  if (e == hipSuccess) e = rows.alloc((size_t)chunk * ny * mh * 16);
  if (e == hipSuccess) e = s64.alloc((size_t)chunk * len * 16);
  for (int q0 = 0; e == hipSuccess && q0 < nq; q0 += chunk) {
    const int cn = std::min(chunk, nq - q0);
    e = launch_project_images(s, dsp.as<double>(), ns, dq.as<double>() + 4 * (size_t)q0, cn, nx, ny,
                              pixel_A, i0.as<double>());
    if (e == hipSuccess) e = launch_rdft2(s, i0.as<double>(), nullptr, cn, nx, ny, rows.as<double2>(), s64.as<double2>());
    if (e == hipSuccess) e = launch_spec_store(s, s64.as<double2>(), cn, nx, ny, p->spec + slen * q0, p->expo + q0);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    bioem_free_proj(p);
    return fail(ctx, e == hipErrorOutOfMemory ? BIOEM_ENOMEM : BIOEM_EDEVICE, "bioem_project: %s",
                hipGetErrorString(e));
  }
  *out = p;
  return BIOEM_OK;
}

bioem_status bioem_prepare_images(bioem_ctx* ctx, const float* imgs, int32_t ni, int32_t nx,
                                  int32_t ny, bioem_mem in_mem, bioem_imgs** out) {
  if (!ctx) return BIOEM_EINVAL;
  if (!out) return fail(ctx, BIOEM_EINVAL, "bioem_prepare_images: out is NULL");
  *out = nullptr;
  if (!imgs || ni < 1) return fail(ctx, BIOEM_EINVAL, "bioem_prepare_images: need ni >= 1 images");
  if (!valid_box(nx, ny))
    return fail(ctx, BIOEM_EINVAL, "bioem_prepare_images: box %dx%d must be even and within [4, %d]", nx, ny, kMaxBox);
  if (!valid_mem(in_mem)) return fail(ctx, BIOEM_EINVAL, "bioem_prepare_images: bad in_mem");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int mh = nx / 2 + 1;
  const size_t len = (size_t)mh * ny, slen = (size_t)mh * spec_ld(ny), npix = (size_t)nx * ny;
  bioem_imgs* p = new (std::nothrow) bioem_imgs;
  if (!p) return fail(ctx, BIOEM_ENOMEM, "bioem_prepare_images: host allocation");
  p->n = ni; p->nx = nx; p->ny = ny; p->device = ctx->device;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->spec), sizeof(float2) * slen * ni);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->expo), sizeof(int32_t) * ni);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->stats), sizeof(double) * 3 * ni);
  if (e != hipSuccess) {
    bioem_free_imgs(p);
    return fail(ctx, BIOEM_ENOMEM, "bioem_prepare_images: device allocation failed");
  }
  const size_t per = npix * 4 + (size_t)ny * mh * 16 + len * 16;
  const int chunk = chunk_items(ni, per);
  DevMem stage, rows, s64;
  if (in_mem == BIOEM_MEM_HOST) e = stage.alloc((size_t)chunk * npix * 4);
  if (e == hipSuccess) e = rows.alloc((size_t)chunk * ny * mh * 16);
  if (e == hipSuccess) e = s64.alloc((size_t)chunk * len * 16);
  for (int i0 = 0; e == hipSuccess && i0 < ni; i0 += chunk) {
    const int cn = std::min(chunk, ni - i0);
    const float* src = imgs + npix * i0;
    if (in_mem == BIOEM_MEM_HOST) {
      e = hipMemcpyAsync(stage.p, src, npix * 4 * cn, hipMemcpyHostToDevice, s);
      src = stage.as<float>();
    }
    if (e == hipSuccess) e = launch_image_stats(s, src, cn, (int)npix, p->stats + 3 * (size_t)i0);
    if (e == hipSuccess) e = launch_rdft2(s, nullptr, src, cn, nx, ny, rows.as<double2>(), s64.as<double2>());
    if (e == hipSuccess) e = launch_spec_store(s, s64.as<double2>(), cn, nx, ny, p->spec + slen * i0, p->expo + i0);
    if (e == hipSuccess && in_mem == BIOEM_MEM_HOST) e = hipStreamSynchronize(s);  // stage reuse
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    bioem_free_imgs(p);
    return fail(ctx, e == hipErrorOutOfMemory ? BIOEM_ENOMEM : BIOEM_EDEVICE,
                "bioem_prepare_images: %s", hipGetErrorString(e));
  }
  *out = p;
  return BIOEM_OK;
}

bioem_status bioem_render(bioem_ctx* ctx, const bioem_proj* proj, const double* ctf,
                          const int32_t* shifts, const double* norm_offset, const float* noise,
                          double snr, bioem_mem in_mem, float* out, bioem_mem out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!proj || !ctf || !shifts || !out) return fail(ctx, BIOEM_EINVAL, "bioem_render: NULL argument");
  if (!valid_mem(in_mem) || !valid_mem(out_mem)) return fail(ctx, BIOEM_EINVAL, "bioem_render: bad mem kind");
  if (noise && !(snr > 0.0 && std::isfinite(snr)))
    return fail(ctx, BIOEM_EINVAL, "bioem_render: snr must be positive and finite");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int n = proj->n, nx = proj->nx, ny = proj->ny, mh = nx / 2 + 1;
  const size_t len = (size_t)mh * ny, slen = (size_t)mh * spec_ld(ny), npix = (size_t)nx * ny;
  std::vector<double> hc;
  HIP_OR_FAIL(ctx, to_host(ctf, (size_t)n * 3, in_mem, s, hc));
  if (!finite_all(hc.data(), hc.size())) return fail(ctx, BIOEM_EINVAL, "bioem_render: non-finite CTF value");
  for (int i = 0; i < n; ++i)
    if (!(hc[3 * i + 1] >= 0.0 && hc[3 * i + 1] <= 1.0))
      return fail(ctx, BIOEM_EINVAL, "bioem_render: amplitude contrast of item %d outside [0,1]", i);
  DevIn dc, dsh, dno, dnz;
  HIP_OR_FAIL(ctx, dc.set(hc.data(), hc.size() * 8, BIOEM_MEM_HOST, s));
  HIP_OR_FAIL(ctx, dsh.set(shifts, (size_t)n * 2 * 4, in_mem, s));
  HIP_OR_FAIL(ctx, dno.set(norm_offset, (size_t)n * 2 * 8, in_mem, s));
  HIP_OR_FAIL(ctx, dnz.set(noise, npix * 4 * n, in_mem, s));
  DevMem obuf;
  float* dst = out;
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, obuf.alloc(npix * 4 * n));
    dst = obuf.as<float>();
  }
  const size_t per = len * 16 + (size_t)ny * mh * 16 + npix * 8;
  const int chunk = chunk_items(n, per);
  DevMem s64, cols, i1;
  hipError_t e = s64.alloc((size_t)chunk * len * 16);
  if (e == hipSuccess) e = cols.alloc((size_t)chunk * ny * mh * 16);
  if (e == hipSuccess) e = i1.alloc((size_t)chunk * npix * 8);
  for (int i0 = 0; e == hipSuccess && i0 < n; i0 += chunk) {
    const int cn = std::min(chunk, n - i0);
    e = launch_render(s, proj->spec + slen * i0, proj->expo + i0, cn, nx, ny, proj->pixel,
                      dc.as<double>() + 3 * (size_t)i0, dsh.as<int32_t>() + 2 * (size_t)i0,
                      dno.d ? dno.as<double>() + 2 * (size_t)i0 : nullptr,
                      dnz.d ? dnz.as<float>() + npix * i0 : nullptr, snr, s64.as<double2>(),
                      cols.as<double2>(), i1.as<double>(), dst + npix * i0);
  }
  if (e == hipSuccess && out_mem == BIOEM_MEM_HOST)
    e = hipMemcpyAsync(out, dst, npix * 4 * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess)
    return fail(ctx, e == hipErrorOutOfMemory ? BIOEM_ENOMEM : BIOEM_EDEVICE, "bioem_render: %s",
                hipGetErrorString(e));
  return BIOEM_OK;
}

bioem_status bioem_logpost(bioem_ctx* ctx, const bioem_proj* proj, const bioem_imgs* imgs,
                           const double* ctf, int32_t nc, bioem_mem ctf_mem, int32_t max_shift,
                           const bioem_opts* opts, double* logp, bioem_best* best) {
  if (!ctx) return BIOEM_EINVAL;
  if (!proj || !imgs || !ctf) return fail(ctx, BIOEM_EINVAL, "bioem_logpost: NULL handle or ctf");
  bioem_opts o{};
  if (opts) o = *opts;
  if (o.reserved[0] || o.reserved[1] || o.reserved[2] || o.reserved[3])
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost: opts.reserved must be zero");
  if (!valid_mem(ctf_mem) || !valid_mem(o.out_mem) || (o.cand_q && !valid_mem(o.cand_mem)))
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost: bad mem kind");
  if (o.prec != BIOEM_PREC_F32 && o.prec != BIOEM_PREC_SPLIT_BF16 && o.prec != BIOEM_PREC_SPLIT_F16)
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost: unknown precision mode %d", o.prec);
  const int nx = proj->nx, ny = proj->ny, nq = proj->n, ni = imgs->n;
  if (imgs->nx != nx || imgs->ny != ny)
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost: image box %dx%d differs from projection box %dx%d",
                imgs->nx, imgs->ny, nx, ny);
  if ((long)nx * ny <= 2) return fail(ctx, BIOEM_EINVAL, "bioem_logpost: need more than 2 pixels");
  if (nc < 1) return fail(ctx, BIOEM_EINVAL, "bioem_logpost: need nc >= 1 CTF sets");
  if (max_shift < 0 || 2 * max_shift >= std::min(nx, ny))
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost: max_shift %d outside [0, min(nx,ny)/2)", max_shift);
  if (o.cand_q && (o.k < 1 || o.k > nq))
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost: candidate count k=%d outside [1, %d]", o.k, nq);
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<double> hc;
  HIP_OR_FAIL(ctx, to_host(ctf, (size_t)nc * 3, ctf_mem, s, hc));
  if (!finite_all(hc.data(), hc.size())) return fail(ctx, BIOEM_EINVAL, "bioem_logpost: non-finite CTF value");
  for (int c = 0; c < nc; ++c)
    if (!(hc[3 * c + 1] >= 0.0 && hc[3 * c + 1] <= 1.0))
      return fail(ctx, BIOEM_EINVAL, "bioem_logpost: amplitude contrast of CTF %d outside [0,1]", c);
  const bool split = o.prec != BIOEM_PREC_F32;
  if (split && !split_supported(nx, ny, max_shift))
    return fail(ctx, BIOEM_EUNSUPPORTED, "bioem_logpost: split-precision kernel does not support %dx%d with S=%d",
                nx, ny, max_shift);
  if (!split && f32_smem_bytes(nx, ny, max_shift) > kMaxSmem)
    return fail(ctx, BIOEM_EUNSUPPORTED, "bioem_logpost: shift window too large for the F32 kernel");
  std::vector<int32_t> hcand;
  if (o.cand_q) {
    HIP_OR_FAIL(ctx, to_host(o.cand_q, (size_t)ni * o.k, (bioem_mem)o.cand_mem, s, hcand));
    for (size_t e = 0; e < hcand.size(); ++e)
      if (hcand[e] < 0 || hcand[e] >= nq)
        return fail(ctx, BIOEM_EINVAL, "bioem_logpost: candidate %zu = %d outside [0, %d)", e, hcand[e], nq);
  }
  const int mh = nx / 2 + 1;
  const size_t len = (size_t)mh * spec_ld(ny);   // stored spectrum / table stride
  DevIn dctf, dcand;
  HIP_OR_FAIL(ctx, dctf.set(hc.data(), hc.size() * 8, BIOEM_MEM_HOST, s));
  if (o.cand_q) HIP_OR_FAIL(ctx, dcand.set(hcand.data(), hcand.size() * 4, BIOEM_MEM_HOST, s));
  DevMem table, B;
  HIP_OR_FAIL(ctx, table.alloc(sizeof(float) * len * nc));
  HIP_OR_FAIL(ctx, B.alloc(sizeof(double) * (size_t)nq * nc));
  HIP_OR_FAIL(ctx, launch_ctf_table(s, dctf.as<double>(), nc, nx, ny, proj->pixel, table.as<float>()));
  HIP_OR_FAIL(ctx, launch_proj_norms(s, proj->spec, proj->expo, nq, table.as<float>(), nc, nx, ny, B.as<double>()));

  // outputs (device staging when the caller wants host memory)
  const bool host_out = o.out_mem == BIOEM_MEM_HOST;
  DevMem dlogp, dbest, dorient;
  double* d_logp = logp;
  bioem_best* d_best = best;
  double* d_orient = o.logp_orient;
  if (host_out) {
    if (logp) { HIP_OR_FAIL(ctx, dlogp.alloc(8 * (size_t)ni)); d_logp = dlogp.as<double>(); }
    if (best) { HIP_OR_FAIL(ctx, dbest.alloc(sizeof(bioem_best) * (size_t)ni)); d_best = dbest.as<bioem_best>(); }
    if (o.logp_orient) { HIP_OR_FAIL(ctx, dorient.alloc(8 * (size_t)ni * nq)); d_orient = dorient.as<double>(); }
  }
  const int nslots = o.cand_q ? o.k : nq;
  const int shape = split ? split_shape_for(ctx, nx, ny, max_shift, nc) : 0;
  const size_t per_image = sizeof(bioem_erec) * (size_t)nslots * nc;
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(ni, kRecordBudget / per_image));
  DevMem rec;
  HIP_OR_FAIL(ctx, rec.alloc(per_image * chunk));
  const int W = 2 * max_shift + 1;
  const double log_prior = -std::log((double)nq) - std::log((double)nc) - std::log((double)W * W);
  const int nchunks = (ni + chunk - 1) / chunk;
  if (ctx->timing) {
    while ((int)ctx->ev_start.size() < ctx->ev_used + nchunks) {
      hipEvent_t a, b;
      HIP_OR_FAIL(ctx, hipEventCreate(&a));
      HIP_OR_FAIL(ctx, hipEventCreate(&b));
      ctx->ev_start.push_back(a);
      ctx->ev_stop.push_back(b);
    }
  }
  for (int i0 = 0; i0 < ni; i0 += chunk) {
    const int cn = std::min(chunk, ni - i0);
    LogpostArgs a{};
    a.ispec = imgs->spec + len * i0; a.iexpo = imgs->expo + i0; a.istats = imgs->stats + 3 * (size_t)i0; a.ni = cn;
    a.pspec = proj->spec; a.pexpo = proj->expo; a.nq = nq;
    a.table = table.as<float>(); a.B = B.as<double>(); a.nc = nc;
    a.nx = nx; a.ny = ny; a.S = max_shift; a.ldy = spec_ld(ny);
    a.cand = o.cand_q ? dcand.as<int32_t>() + (size_t)i0 * o.k : nullptr; a.k = o.k;
    a.rec = rec.as<bioem_erec>();
    a.kscale = 1.0 / ((double)nx * ny * (double)nx * ny);
    if (ctx->timing) HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev_start[ctx->ev_used], s));
    hipError_t e = split ? launch_logpost_split(s, a, o.prec == BIOEM_PREC_SPLIT_BF16, shape) : launch_logpost_f32(s, a);
    if (ctx->timing && e == hipSuccess) {
      HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev_stop[ctx->ev_used], s));
      ++ctx->ev_used;
      ctx->timed_evals += (double)cn * nslots * nc;
    }
    if (e == hipSuccess) {
      FinalizeArgs f{};
      f.rec = a.rec; f.ni = cn; f.nslots = nslots; f.nc = nc; f.nq_total = nq; f.nx = nx; f.ny = ny;
      f.S = max_shift; f.cand = a.cand; f.k = o.k;
      f.istats = a.istats; f.iexpo = a.iexpo; f.pexpo = proj->expo; f.B = a.B;
      f.log_prior = log_prior;
      f.logp = d_logp ? d_logp + i0 : nullptr;
      f.best = d_best ? d_best + i0 : nullptr;
      f.orient = d_orient ? d_orient + (size_t)i0 * nq : nullptr;
      e = launch_finalize(s, f);
      if (e == hipSuccess && split && f.best) e = launch_best_shift(s, a, f.best);
    }
    if (e != hipSuccess) return fail(ctx, BIOEM_EDEVICE, "bioem_logpost: launch failed: %s", hipGetErrorString(e));
  }
  if (host_out) {
    if (logp) HIP_OR_FAIL(ctx, hipMemcpyAsync(logp, d_logp, 8 * (size_t)ni, hipMemcpyDeviceToHost, s));
    if (best) HIP_OR_FAIL(ctx, hipMemcpyAsync(best, d_best, sizeof(bioem_best) * (size_t)ni, hipMemcpyDeviceToHost, s));
    if (o.logp_orient)
      HIP_OR_FAIL(ctx, hipMemcpyAsync(o.logp_orient, d_orient, 8 * (size_t)ni * nq, hipMemcpyDeviceToHost, s));
  }
  // Scratch (table, B, records) is freed on return, so the stream must drain.
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

}  // extern "C"
