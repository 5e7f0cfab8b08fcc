// Host side of the proposal-network ABI: parameters, workspace and the
// layer-by-layer forward and backward passes (every layer is a kernel of
// k_cnn.hip; activations are channel-major [C][B][H][W] FP32).
#include <algorithm>
#include <cmath>
#include <new>

#include "cnn.hpp"
#include "common.hpp"
#include "host_util.hpp"

using namespace bioem;
using namespace bioem::host;

struct bioem_cnn {
  int device = 0;
  bioem_cnn_arch arch{};
  long nparams = 0;
  long off[12] = {};            // W1 b1 W2 b2 W3 b3 W4 b4 F1 g1 F2 g2
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int step = 0;
  bool have_grad = false;
  int cap = 0;                  // batch size the workspace holds
  void* ws = nullptr;
  // workspace views
  float *x0 = nullptr, *y[5] = {}, *cols = nullptr, *dcols = nullptr, *dya = nullptr, *dyb = nullptr;
  float *feat = nullptr, *h = nullptr, *z = nullptr, *dz = nullptr, *dh = nullptr, *dfeat = nullptr,
        *lossb = nullptr;
  int32_t* tidx = nullptr;
  float* tp = nullptr;
  float* part = nullptr;        // split-K partials
  int tcap = 0;
};

namespace {

constexpr int kMaxBatch = 256;
constexpr size_t kPartFloats = size_t(4) << 20;   // split-K partial sums

int chan(const bioem_cnn_arch& a, int l) {
  const int c[5] = {1, a.c1, a.c2, a.c3, a.c4};
  return c[l];
}

int side(const bioem_cnn_arch& a, int l) { return a.box >> l; }   // spatial size after l layers

// Grow the workspace to hold a batch of B images and T targets per image.
hipError_t reserve(bioem_cnn* n, int B, int T) {
  if (B <= n->cap && T <= n->tcap) return hipSuccess;
  const bioem_cnn_arch& a = n->arch;
  B = std::max(B, n->cap);
  T = std::max(T, std::max(n->tcap, 1));
  size_t ysz[5], colmax = 0, ymax = 0;
  for (int l = 0; l <= 4; ++l) {
    ysz[l] = (size_t)chan(a, l) * B * side(a, l) * side(a, l);
    if (l >= 1) {
      colmax = std::max(colmax, (size_t)chan(a, l - 1) * 9 * B * side(a, l) * side(a, l));
      ymax = std::max(ymax, ysz[l]);
    }
  }
  const size_t zsz = (size_t)B * a.nq;
  const size_t floats = ysz[0] + ysz[1] + ysz[2] + ysz[3] + ysz[4] + 2 * colmax + 2 * ymax + ysz[4] * 2 +
                        (size_t)a.hidden * B * 2 + 2 * zsz + B + (size_t)B * T + kPartFloats;
  const size_t bytes = floats * sizeof(float) + (size_t)B * T * sizeof(int32_t) + 256;
  if (n->ws) (void)hipFree(n->ws);
  n->ws = nullptr;
  n->cap = n->tcap = 0;
  hipError_t e = hipMalloc(&n->ws, bytes);
  if (e != hipSuccess) return e;
  float* p = static_cast<float*>(n->ws);
  auto take = [&p](size_t k) { float* r = p; p += k; return r; };
  n->x0 = take(ysz[0]);
  n->y[0] = n->x0;
  for (int l = 1; l <= 4; ++l) n->y[l] = take(ysz[l]);
  n->cols = take(colmax);
  n->dcols = take(colmax);
  n->dya = take(ymax);
  n->dyb = take(ymax);
  n->feat = take(ysz[4]);
  n->dfeat = take(ysz[4]);
  n->h = take((size_t)a.hidden * B);
  n->dh = take((size_t)a.hidden * B);
  n->z = take(zsz);
  n->dz = take(zsz);
  n->lossb = take(B);
  n->part = take(kPartFloats);
  n->tp = take((size_t)B * T);
  n->tidx = reinterpret_cast<int32_t*>(p);
  n->cap = B;
  n->tcap = T;
  return hipSuccess;
}

// Forward pass of B <= cap images already on the device; logits in n->z.
hipError_t forward(hipStream_t s, bioem_cnn* n, const float* imgs, int B) {
  const bioem_cnn_arch& a = n->arch;
  hipError_t e = cnn::standardize(s, imgs, B, a.box * a.box, n->x0);
  for (int l = 1; l <= 4 && e == hipSuccess; ++l) {
    const int cin = chan(a, l - 1), cout = chan(a, l), H = side(a, l - 1);
    const long P = (long)B * side(a, l) * side(a, l);
    e = cnn::im2col(s, n->y[l - 1], cin, B, H, H, n->cols);
    if (e == hipSuccess)
      e = cnn::gemm(s, cout, (int)P, cin * 9, n->w + n->off[2 * (l - 1)], cin * 9, 1, n->cols, P, 1, n->y[l], P, 1,
                    1.0f, 0.0f, n->part, kPartFloats);
    if (e == hipSuccess) e = cnn::bias_relu(s, n->y[l], n->w + n->off[2 * (l - 1) + 1], cout, P, true);
  }
  const int P4 = side(a, 4) * side(a, 4), F = a.c4 * P4;
  if (e == hipSuccess) e = cnn::flatten(s, n->y[4], a.c4, B, P4, false, n->feat);
  if (e == hipSuccess)
    e = cnn::gemm(s, a.hidden, B, F, n->w + n->off[8], F, 1, n->feat, B, 1, n->h, B, 1, 1.0f, 0.0f, n->part, kPartFloats);
  if (e == hipSuccess) e = cnn::bias_relu(s, n->h, n->w + n->off[9], a.hidden, B, true);
  if (e == hipSuccess)
    e = cnn::gemm(s, B, a.nq, a.hidden, n->h, 1, B, n->w + n->off[10], 1, a.hidden, n->z, a.nq, 1, 1.0f, 0.0f, n->part, kPartFloats);
  if (e == hipSuccess) e = cnn::bias_cols(s, n->z, n->w + n->off[11], B, a.nq);
  return e;
}

// Backward pass after forward(): gradient of the mean loss into n->g.
hipError_t backward(hipStream_t s, bioem_cnn* n, int B, int T) {
  const bioem_cnn_arch& a = n->arch;
  float* g = n->g;
  const float* w = n->w;
  hipError_t e = cnn::softmax_xent(s, n->z, B, a.nq, n->tidx, n->tp, T, n->dz, n->lossb);
  // output layer
  if (e == hipSuccess)
    e = cnn::gemm(s, a.nq, a.hidden, B, n->dz, 1, a.nq, n->h, 1, B, g + n->off[10], a.hidden, 1, 1.0f, 0.0f, n->part, kPartFloats);
  if (e == hipSuccess) e = cnn::row_sum(s, n->dz, a.nq, 1, a.nq, B, 1.0f, g + n->off[11]);
  if (e == hipSuccess)
    e = cnn::gemm(s, a.hidden, B, a.nq, w + n->off[10], 1, a.hidden, n->dz, 1, a.nq, n->dh, B, 1, 1.0f, 0.0f, n->part, kPartFloats);
  if (e == hipSuccess) e = cnn::relu_bwd(s, n->dh, n->h, (long)a.hidden * B);
  // hidden layer
  const int P4 = side(a, 4) * side(a, 4), F = a.c4 * P4;
  if (e == hipSuccess)
    e = cnn::gemm(s, a.hidden, F, B, n->dh, B, 1, n->feat, 1, B, g + n->off[8], F, 1, 1.0f, 0.0f, n->part, kPartFloats);
  if (e == hipSuccess) e = cnn::row_sum(s, n->dh, a.hidden, B, 1, B, 1.0f, g + n->off[9]);
  if (e == hipSuccess)
    e = cnn::gemm(s, F, B, a.hidden, w + n->off[8], 1, F, n->dh, B, 1, n->dfeat, B, 1, 1.0f, 0.0f, n->part, kPartFloats);
  // back to the [c4][B][P4] activation, then the convolutions from the top
  float* dy = n->dya;
  float* dnext = n->dyb;
  if (e == hipSuccess) e = cnn::flatten(s, n->dfeat, a.c4, B, P4, true, dy);
  for (int l = 4; l >= 1 && e == hipSuccess; --l) {
    const int cin = chan(a, l - 1), cout = chan(a, l), H = side(a, l - 1);
    const long P = (long)B * side(a, l) * side(a, l);
    e = cnn::relu_bwd(s, dy, n->y[l], (long)cout * P);
    if (e == hipSuccess) e = cnn::row_sum(s, dy, cout, P, 1, P, 1.0f, g + n->off[2 * (l - 1) + 1]);
    if (e == hipSuccess) e = cnn::im2col(s, n->y[l - 1], cin, B, H, H, n->cols);
    if (e == hipSuccess)
      e = cnn::gemm(s, cout, cin * 9, (int)P, dy, P, 1, n->cols, 1, P, g + n->off[2 * (l - 1)], cin * 9, 1, 1.0f, 0.0f, n->part, kPartFloats);
    if (l > 1 && e == hipSuccess) {
      e = cnn::gemm(s, cin * 9, (int)P, cout, w + n->off[2 * (l - 1)], 1, cin * 9, dy, P, 1, n->dcols, P, 1, 1.0f, 0.0f, n->part, kPartFloats);
      if (e == hipSuccess) e = cnn::col2im(s, n->dcols, cin, B, H, H, dnext);
      std::swap(dy, dnext);
    }
  }
  return e;
}

bool valid_arch(const bioem_cnn_arch& a) {
  return a.reserved == 0 && a.box >= 16 && a.box <= 512 && a.box % 16 == 0 && a.c1 >= 1 && a.c2 >= 1 &&
         a.c3 >= 1 && a.c4 >= 1 && a.c1 <= 1024 && a.c2 <= 1024 && a.c3 <= 1024 && a.c4 <= 1024 &&
         a.hidden >= 1 && a.hidden <= 4096 && a.nq >= 1 && a.nq <= (1 << 22);
}

}  // namespace

extern "C" {

bioem_status bioem_cnn_create(bioem_ctx* ctx, const bioem_cnn_arch* arch, bioem_cnn** out) {
  if (!ctx) return BIOEM_EINVAL;
  if (!arch || !out) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_create: NULL argument");
  *out = nullptr;
  if (!valid_arch(*arch)) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_create: invalid architecture");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  bioem_cnn* n = new (std::nothrow) bioem_cnn;
  if (!n) return fail(ctx, BIOEM_ENOMEM, "bioem_cnn_create: out of host memory");
  n->device = ctx->device;
  n->arch = *arch;
  long off = 0;
  for (int l = 1; l <= 4; ++l) {
    n->off[2 * (l - 1)] = off;
    off += (long)chan(*arch, l) * chan(*arch, l - 1) * 9;
    n->off[2 * (l - 1) + 1] = off;
    off += chan(*arch, l);
  }
  n->off[8] = off; off += (long)arch->hidden * arch->c4 * (arch->box / 16) * (arch->box / 16);
  n->off[9] = off; off += arch->hidden;
  n->off[10] = off; off += (long)arch->nq * arch->hidden;
  n->off[11] = off; off += arch->nq;
  n->nparams = off;
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(float) * 4 * (size_t)off) != hipSuccess) {
    delete n;
    return fail(ctx, BIOEM_ENOMEM, "bioem_cnn_create: device allocation failed");
  }
  n->w = static_cast<float*>(p);
  n->g = n->w + off;
  n->m = n->g + off;
  n->v = n->m + off;
  if (hipMemsetAsync(p, 0, sizeof(float) * 4 * (size_t)off, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipFree(p);
    delete n;
    return fail(ctx, BIOEM_EDEVICE, "bioem_cnn_create: clearing parameters failed");
  }
  *out = n;
  return BIOEM_OK;
}

void bioem_cnn_destroy(bioem_cnn* n) {
  if (!n) return;
  (void)hipSetDevice(n->device);
  if (n->ws) (void)hipFree(n->ws);
  if (n->w) (void)hipFree(n->w);
  delete n;
}

int64_t bioem_cnn_num_params(const bioem_cnn* n) { return n ? n->nparams : 0; }

bioem_status bioem_cnn_set_params(bioem_ctx* ctx, bioem_cnn* n, const float* params, int32_t mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!n || !params || !valid_mem(mem)) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_set_params: bad argument");
  if (n->device != ctx->device) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_set_params: network on another device");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  const size_t bytes = sizeof(float) * (size_t)n->nparams;
  HIP_OR_FAIL(ctx, hipMemcpyAsync(n->w, params, bytes, mem == BIOEM_MEM_HOST ? hipMemcpyHostToDevice
                                                                           : hipMemcpyDeviceToDevice, ctx->stream));
  HIP_OR_FAIL(ctx, hipMemsetAsync(n->m, 0, 2 * bytes, ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  n->step = 0;
  n->have_grad = false;
  return BIOEM_OK;
}

bioem_status bioem_cnn_get_params(bioem_ctx* ctx, const bioem_cnn* n, float* params, int32_t mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!n || !params || !valid_mem(mem)) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_get_params: bad argument");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(params, n->w, sizeof(float) * (size_t)n->nparams,
                                  mem == BIOEM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                  ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  return BIOEM_OK;
}

bioem_status bioem_cnn_forward(bioem_ctx* ctx, bioem_cnn* n, const float* imgs, int32_t B, int32_t in_mem,
                               float* logits, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!n || !imgs || !logits || B < 1 || !valid_mem(in_mem) || !valid_mem(out_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_cnn_forward: bad argument");
  if (n->device != ctx->device) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_forward: network on another device");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int npix = n->arch.box * n->arch.box, nq = n->arch.nq;
  const int bb = std::min<int>(B, kMaxBatch);
  HIP_OR_FAIL(ctx, reserve(n, bb, 1));
  DevMem stage;
  if (in_mem == BIOEM_MEM_HOST) HIP_OR_FAIL(ctx, stage.alloc(sizeof(float) * (size_t)bb * npix));
  for (int b0 = 0; b0 < B; b0 += bb) {
    const int cb = std::min(bb, B - b0);
    const float* src = imgs + (size_t)b0 * npix;
    if (in_mem == BIOEM_MEM_HOST) {
      HIP_OR_FAIL(ctx, hipMemcpyAsync(stage.p, src, sizeof(float) * (size_t)cb * npix, hipMemcpyHostToDevice, s));
      src = stage.as<float>();
    }
    HIP_OR_FAIL(ctx, forward(s, n, src, cb));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(logits + (size_t)b0 * nq, n->z, sizeof(float) * (size_t)cb * nq,
                                    out_mem == BIOEM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

bioem_status bioem_cnn_backward(bioem_ctx* ctx, bioem_cnn* n, const float* imgs, int32_t B,
                                const int32_t* tidx, const float* tp, int32_t T, int32_t in_mem, float* loss,
                                float* grad, int32_t grad_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!n || !imgs || !tidx || !tp || B < 1 || B > kMaxBatch || T < 1 || !valid_mem(in_mem) ||
      (grad && !valid_mem(grad_mem)))
    return fail(ctx, BIOEM_EINVAL, "bioem_cnn_backward: bad argument (1 <= B <= %d, T >= 1)", kMaxBatch);
  if (n->device != ctx->device) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_backward: network on another device");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int npix = n->arch.box * n->arch.box;
  // targets are validated on the host (indices in range)
  std::vector<int32_t> hidx;
  HIP_OR_FAIL(ctx, to_host(tidx, (size_t)B * T, (bioem_mem)in_mem, s, hidx));
  for (size_t e = 0; e < hidx.size(); ++e)
    if (hidx[e] < 0 || hidx[e] >= n->arch.nq)
      return fail(ctx, BIOEM_EINVAL, "bioem_cnn_backward: target index %d outside [0, %d)", hidx[e], n->arch.nq);
  HIP_OR_FAIL(ctx, reserve(n, B, T));
  const hipMemcpyKind k = in_mem == BIOEM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  HIP_OR_FAIL(ctx, hipMemcpyAsync(n->tidx, hidx.data(), sizeof(int32_t) * (size_t)B * T, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(n->tp, tp, sizeof(float) * (size_t)B * T, k, s));
  DevMem stage;
  const float* src = imgs;
  if (in_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, stage.alloc(sizeof(float) * (size_t)B * npix));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(stage.p, imgs, sizeof(float) * (size_t)B * npix, hipMemcpyHostToDevice, s));
    src = stage.as<float>();
  }
  HIP_OR_FAIL(ctx, forward(s, n, src, B));
  HIP_OR_FAIL(ctx, backward(s, n, B, T));
  std::vector<float> lb(B);
  HIP_OR_FAIL(ctx, hipMemcpyAsync(lb.data(), n->lossb, sizeof(float) * B, hipMemcpyDeviceToHost, s));
  if (grad)
    HIP_OR_FAIL(ctx, hipMemcpyAsync(grad, n->g, sizeof(float) * (size_t)n->nparams,
                                    grad_mem == BIOEM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  if (loss) {
    double t = 0.0;
    for (float x : lb) t += x;
    *loss = (float)(t / B);
  }
  n->have_grad = true;
  return BIOEM_OK;
}

bioem_status bioem_cnn_adam(bioem_ctx* ctx, bioem_cnn* n, float lr, float beta1, float beta2, float eps) {
  if (!ctx) return BIOEM_EINVAL;
  if (!n || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(ctx, BIOEM_EINVAL, "bioem_cnn_adam: bad argument");
  if (!n->have_grad) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_adam: no gradient (call bioem_cnn_backward first)");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  ++n->step;
  HIP_OR_FAIL(ctx, cnn::adam(ctx->stream, n->w, n->g, n->m, n->v, n->nparams, lr, beta1, beta2, eps, n->step));
  return BIOEM_OK;
}

bioem_status bioem_cnn_propose(bioem_ctx* ctx, bioem_cnn* n, const float* imgs, int32_t B, int32_t in_mem,
                               int32_t K, int32_t* cand, float* mass, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!n || !imgs || !cand || B < 1 || !valid_mem(in_mem) || !valid_mem(out_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_cnn_propose: bad argument");
  if (K < 1 || K > n->arch.nq) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_propose: K=%d outside [1, %d]", K, n->arch.nq);
  if (n->device != ctx->device) return fail(ctx, BIOEM_EINVAL, "bioem_cnn_propose: network on another device");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int npix = n->arch.box * n->arch.box, nq = n->arch.nq;
  const int bb = std::min<int>(B, kMaxBatch);
  HIP_OR_FAIL(ctx, reserve(n, bb, 1));
  DevMem stage, dc, dm;
  if (in_mem == BIOEM_MEM_HOST) HIP_OR_FAIL(ctx, stage.alloc(sizeof(float) * (size_t)bb * npix));
  int32_t* c_out = cand;
  float* m_out = mass;
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, dc.alloc(sizeof(int32_t) * (size_t)B * K));
    c_out = dc.as<int32_t>();
    if (mass) {
      HIP_OR_FAIL(ctx, dm.alloc(sizeof(float) * (size_t)B));
      m_out = dm.as<float>();
    }
  }
  for (int b0 = 0; b0 < B; b0 += bb) {
    const int cb = std::min(bb, B - b0);
    const float* src = imgs + (size_t)b0 * npix;
    if (in_mem == BIOEM_MEM_HOST) {
      HIP_OR_FAIL(ctx, hipMemcpyAsync(stage.p, src, sizeof(float) * (size_t)cb * npix, hipMemcpyHostToDevice, s));
      src = stage.as<float>();
    }
    HIP_OR_FAIL(ctx, forward(s, n, src, cb));
    HIP_OR_FAIL(ctx, cnn::topk(s, n->z, cb, nq, K, c_out + (size_t)b0 * K, m_out ? m_out + b0 : nullptr));
  }
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, hipMemcpyAsync(cand, c_out, sizeof(int32_t) * (size_t)B * K, hipMemcpyDeviceToHost, s));
    if (mass) HIP_OR_FAIL(ctx, hipMemcpyAsync(mass, m_out, sizeof(float) * (size_t)B, hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

bioem_status bioem_cnn_input(bioem_ctx* ctx, const float* imgs, int32_t B, int32_t nx, int32_t ny, int32_t in_mem,
                             float* out, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!imgs || !out || B < 1 || nx < 4 || ny < 4 || nx > kMaxBox || ny > kMaxBox || nx % 2 || ny % 2 ||
      !valid_mem(in_mem) || !valid_mem(out_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_cnn_input: bad argument");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int bb = std::min<int>(B, kMaxBatch), mh = nx / 2 + 1;
  const size_t npix = (size_t)nx * ny, nspec = (size_t)mh * ny;
  DevMem scratch, stage_in, stage_out;
  HIP_OR_FAIL(ctx, scratch.alloc((sizeof(double2) * 3 * nspec + sizeof(double) * npix) * bb));
  double2* rows = scratch.as<double2>();
  double2* spec = rows + nspec * bb;
  double2* cols = spec + nspec * bb;
  double* a64 = reinterpret_cast<double*>(cols + nspec * bb);
  if (in_mem == BIOEM_MEM_HOST) HIP_OR_FAIL(ctx, stage_in.alloc(sizeof(float) * npix * bb));
  if (out_mem == BIOEM_MEM_HOST) HIP_OR_FAIL(ctx, stage_out.alloc(sizeof(float) * npix * bb));
  for (int b0 = 0; b0 < B; b0 += bb) {
    const int cb = std::min(bb, B - b0);
    const float* src = imgs + npix * b0;
    if (in_mem == BIOEM_MEM_HOST) {
      HIP_OR_FAIL(ctx, hipMemcpyAsync(stage_in.p, src, sizeof(float) * npix * cb, hipMemcpyHostToDevice, s));
      src = stage_in.as<float>();
    }
    float* dst = out_mem == BIOEM_MEM_HOST ? stage_out.as<float>() : out + npix * b0;
    HIP_OR_FAIL(ctx, launch_autocorr(s, src, cb, nx, ny, rows, spec, cols, a64, dst));
    if (out_mem == BIOEM_MEM_HOST)
      HIP_OR_FAIL(ctx, hipMemcpyAsync(out + npix * b0, dst, sizeof(float) * npix * cb, hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

bioem_status bioem_topk(bioem_ctx* ctx, const float* z, int32_t B, int32_t n, int32_t K, int32_t in_mem,
                        int32_t* idx, float* mass, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!z || !idx || B < 1 || n < 1 || K < 1 || K > n || !valid_mem(in_mem) || !valid_mem(out_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_topk: bad argument");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  DevIn dz;
  HIP_OR_FAIL(ctx, dz.set(z, sizeof(float) * (size_t)B * n, (bioem_mem)in_mem, s));
  DevMem di, dm;
  int32_t* i_out = idx;
  float* m_out = mass;
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, di.alloc(sizeof(int32_t) * (size_t)B * K));
    i_out = di.as<int32_t>();
    if (mass) {
      HIP_OR_FAIL(ctx, dm.alloc(sizeof(float) * (size_t)B));
      m_out = dm.as<float>();
    }
  }
  HIP_OR_FAIL(ctx, cnn::topk(s, dz.as<float>(), B, n, K, i_out, m_out));
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, hipMemcpyAsync(idx, i_out, sizeof(int32_t) * (size_t)B * K, hipMemcpyDeviceToHost, s));
    if (mass) HIP_OR_FAIL(ctx, hipMemcpyAsync(mass, m_out, sizeof(float) * (size_t)B, hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

}  // extern "C"
