// Host side of the C ABI: argument validation, device memory, chunking and
// launch order.  All device work goes to the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "host_util.hpp"

using namespace bioem;
using namespace bioem::host;

// Scratch of bioem_logpost_noalloc: tables, norms and per-evaluation records
// of one call.  Each device holds its own copy from the library's load to the
// end of the process; host code reaches it only through the device address
// that hipGetSymbolAddress returns for the current device (the array's name is
// a host-side stand-in there).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// The scratch address on `device`, resolved once per device with that device
// current; nullptr when the runtime cannot give it.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[device] = ptr;
  }
  return g_scratch[device];
}

}  // namespace

namespace {

constexpr size_t kScratchBudget = size_t(1) << 30;     // per transform chunk
constexpr size_t kRecordBudget = size_t(1) << 30;      // per posterior image chunk

bool valid_box(int nx, int ny) {
  return nx >= 4 && ny >= 4 && nx <= kMaxBox && ny <= kMaxBox && nx % 2 == 0 && ny % 2 == 0;
}


// Items per transform chunk so that the FP64 scratch stays within budget.
int chunk_items(int n, size_t per_item) {
  size_t c = kScratchBudget / (per_item ? per_item : 1);
  if (c < 1) c = 1;
  return (int)std::min<size_t>(c, (size_t)n);
}

}  // namespace


// ---- posterior jobs --------------------------------------------------------

namespace {

constexpr size_t kBatchRecordBudget = size_t(16) << 30;   // records of one persistent launch

// A validated bioem_logpost job with its device-side inputs, tables and
// output staging.
struct Job {
  const bioem_proj* proj = nullptr;
  const bioem_imgs* imgs = nullptr;
  int nx = 0, ny = 0, nq = 0, ni = 0, nc = 0, S = 0, k = 0, nslots = 0;
  double log_prior = 0.0;
  bool has_cand = false;
  DevIn dctf, dcand;
  DevMem table, ttable, B;
  DevMem dlogp, dbest, dorient;
  double* d_logp = nullptr;
  bioem_best* d_best = nullptr;
  double* d_orient = nullptr;
  double* logp = nullptr;          // caller's outputs
  bioem_best* best = nullptr;
  double* orient = nullptr;
  size_t len = 0;                  // stored spectrum stride
  int kernel = 0, ti = 0, ts = 0;  // bioem_opts kernel form and item tile (0 = default)
  bool mf = false;                 // F32 on the FP32 matrix cores
  int zs = 0;                      // split forms: operand scale exponent (CTF tile copies times 2^zs)
  DevMem mftab, mftm;              // its operand tables and orbit-order CTF tables
  Job() = default;
  Job(Job&&) = default;
};

// With a carve every device buffer of the job is a piece of it (nothing is
// allocated): the CTF grid must then be host memory and the outputs device
// memory.
bioem_status plan_job(bioem_ctx* ctx, const bioem_job& jb, int prec, int out_mem, Job& J, const char* who,
                      int kernel = 0, int ti = 0, int ts = 0, Carve* carve = nullptr) {
  const bioem_proj* proj = jb.proj;
  const bioem_imgs* imgs = jb.imgs;
  if (!proj || !imgs || !jb.ctf) return fail(ctx, BIOEM_EINVAL, "%s: NULL handle or ctf", who);
  if (!valid_mem(jb.ctf_mem) || !valid_mem(out_mem) || (jb.cand_q && !valid_mem(jb.cand_mem)))
    return fail(ctx, BIOEM_EINVAL, "%s: bad mem kind", who);
  if (prec != BIOEM_PREC_F32 && prec != BIOEM_PREC_SPLIT_BF16 && prec != BIOEM_PREC_SPLIT_F16)
    return fail(ctx, BIOEM_EINVAL, "%s: unknown precision mode %d", who, prec);
  const int nx = proj->nx, ny = proj->ny, nq = proj->n, ni = imgs->n, nc = jb.nc, S = jb.max_shift;
  if (imgs->nx != nx || imgs->ny != ny)
    return fail(ctx, BIOEM_EINVAL, "%s: image box %dx%d differs from projection box %dx%d", who, imgs->nx,
                imgs->ny, nx, ny);
  if (proj->device != ctx->device || imgs->device != ctx->device)
    return fail(ctx, BIOEM_EINVAL, "%s: handle on another device", who);
  if ((long)nx * ny <= 2) return fail(ctx, BIOEM_EINVAL, "%s: need more than 2 pixels", who);
  if (nc < 1) return fail(ctx, BIOEM_EINVAL, "%s: need nc >= 1 CTF sets", who);
  if (S < 0 || 2 * S >= std::min(nx, ny))
    return fail(ctx, BIOEM_EINVAL, "%s: max_shift %d outside [0, min(nx,ny)/2)", who, S);
  if (jb.cand_q && (jb.k < 1 || jb.k > nq))
    return fail(ctx, BIOEM_EINVAL, "%s: candidate count k=%d outside [1, %d]", who, jb.k, nq);
  hipStream_t s = ctx->stream;
  if (carve && (jb.ctf_mem != BIOEM_MEM_HOST || out_mem != BIOEM_MEM_DEVICE || jb.cand_q))
    return fail(ctx, BIOEM_EINVAL, "%s: needs host CTF values, device outputs and no proposal", who);
  std::vector<double> hcopy;
  const double* hc = jb.ctf;
  if (jb.ctf_mem != BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, to_host(jb.ctf, (size_t)nc * 3, (bioem_mem)jb.ctf_mem, s, hcopy));
    hc = hcopy.data();
  }
  if (!finite_all(hc, (size_t)nc * 3)) return fail(ctx, BIOEM_EINVAL, "%s: non-finite CTF value", who);
  for (int c = 0; c < nc; ++c)
    if (!(hc[3 * c + 1] >= 0.0 && hc[3 * c + 1] <= 1.0))
      return fail(ctx, BIOEM_EINVAL, "%s: amplitude contrast of CTF %d outside [0,1]", who, c);
  const bool split = prec != BIOEM_PREC_F32;
  if (ti < 0 || ts < 0 || ti > 4096 || ts > 65536 || (ti > 0) != (ts > 0))
    return fail(ctx, BIOEM_EINVAL, "%s: item tile %dx%d outside [1, 4096] x [1, 65536]", who, ti, ts);
  bool mf = false;
  if (split) {
    if (kernel < 0 || kernel > split_num_shapes())
      return fail(ctx, BIOEM_EINVAL, "%s: kernel %d outside [0, %d] for a split precision", who, kernel,
                  split_num_shapes());
    if (!split_supported(nx, ny, S))
      return fail(ctx, BIOEM_EUNSUPPORTED, "%s: split-precision kernel does not support %dx%d with S=%d", who,
                  nx, ny, S);
  } else {
    if (kernel < 0 || kernel > 2) return fail(ctx, BIOEM_EINVAL, "%s: kernel %d outside [0, 2] for F32", who, kernel);
    mf = kernel != 2 && mf32_supported(nx, ny, S);
    if (kernel == 1 && !mf)
      return fail(ctx, BIOEM_EUNSUPPORTED, "%s: FP32 matrix-core kernel does not support %dx%d with S=%d", who, nx,
                  ny, S);
  }
  // the vector-ALU kernel, and the best-displacement pass of the other forms
  if (f32_smem_bytes(nx, ny, S) > kMaxSmem)
    return fail(ctx, BIOEM_EUNSUPPORTED, "%s: shift window too large for %dx%d", who, nx, ny);
  std::vector<int32_t> hcand;
  if (jb.cand_q) {
    HIP_OR_FAIL(ctx, to_host(jb.cand_q, (size_t)ni * jb.k, (bioem_mem)jb.cand_mem, s, hcand));
    for (size_t e = 0; e < hcand.size(); ++e)
      if (hcand[e] < 0 || hcand[e] >= nq)
        return fail(ctx, BIOEM_EINVAL, "%s: candidate %zu = %d outside [0, %d)", who, e, hcand[e], nq);
    // a repeated orientation would be scored and summed twice
    std::vector<int32_t> row(jb.k);
    for (int i = 0; i < ni; ++i) {
      std::copy(hcand.begin() + (size_t)i * jb.k, hcand.begin() + (size_t)(i + 1) * jb.k, row.begin());
      std::sort(row.begin(), row.end());
      if (std::adjacent_find(row.begin(), row.end()) != row.end())
        return fail(ctx, BIOEM_EINVAL, "%s: image %d lists orientation %d twice among its candidates", who, i,
                    *std::adjacent_find(row.begin(), row.end()));
    }
  }
  J.proj = proj; J.imgs = imgs;
  J.nx = nx; J.ny = ny; J.nq = nq; J.ni = ni; J.nc = nc; J.S = S;
  J.kernel = kernel; J.ti = ti; J.ts = ts; J.mf = mf;
  J.has_cand = jb.cand_q != nullptr;
  J.k = J.has_cand ? jb.k : 0;
  J.nslots = J.has_cand ? jb.k : nq;
  const int W = 2 * S + 1;
  J.log_prior = -std::log((double)nq) - std::log((double)nc) - std::log((double)W * W);
  J.len = (size_t)(nx / 2 + 1) * spec_ld(ny);
  HIP_OR_FAIL(ctx, J.dctf.set(hc, (size_t)nc * 3 * 8, BIOEM_MEM_HOST, s, carve));
  if (J.has_cand) HIP_OR_FAIL(ctx, J.dcand.set(hcand.data(), hcand.size() * 4, BIOEM_MEM_HOST, s));
  HIP_OR_FAIL(ctx, J.table.get(sizeof(float) * J.len * nc, carve));
  HIP_OR_FAIL(ctx, J.B.get(sizeof(double) * (size_t)nq * nc, carve));
  HIP_OR_FAIL(ctx, launch_ctf_table(s, J.dctf.as<double>(), nc, nx, ny, proj->pixel, J.table.as<float>()));
  if (split) {
    HIP_OR_FAIL(ctx, J.ttable.get(sizeof(float4) * tile_table_len(nx, ny) * nc, carve));
    J.zs = split_operand_scale(ny);
    HIP_OR_FAIL(ctx, launch_tile_table(s, J.table.as<float>(), nc, nx, ny, J.zs, J.ttable.as<float4>()));
  }
  if (mf) {
    HIP_OR_FAIL(ctx, J.mftab.get(sizeof(float4) * mf32_table_len(nx, ny), carve));
    HIP_OR_FAIL(ctx, launch_mf_tables(s, nx, ny, S, J.mftab.as<float4>()));
    HIP_OR_FAIL(ctx, J.mftm.get(sizeof(float4) * mf_table_len(nx, ny) * nc, carve));
    HIP_OR_FAIL(ctx, launch_mf_copy_table(s, J.table.as<float>(), nc, nx, ny, J.mftm.as<float4>()));
  }
  HIP_OR_FAIL(ctx, launch_proj_norms(s, proj->spec, proj->expo, nq, J.table.as<float>(), nc, nx, ny,
                                     J.B.as<double>()));
  // the split forms read the table (packed column, best-displacement pass)
  // with the same operand scale as its tile copies; the norms above are taken
  // first, and the best-displacement pass only compares values
  if (split && J.zs) HIP_OR_FAIL(ctx, launch_scale_table(s, J.table.as<float>(), J.len * nc, J.zs));
  J.logp = jb.logp; J.best = jb.best; J.orient = jb.logp_orient;
  J.d_logp = jb.logp; J.d_best = jb.best; J.d_orient = jb.logp_orient;
  if (out_mem == BIOEM_MEM_HOST) {
    if (J.logp) { HIP_OR_FAIL(ctx, J.dlogp.alloc(8 * (size_t)ni)); J.d_logp = J.dlogp.as<double>(); }
    if (J.best) { HIP_OR_FAIL(ctx, J.dbest.alloc(sizeof(bioem_best) * (size_t)ni)); J.d_best = J.dbest.as<bioem_best>(); }
    if (J.orient) { HIP_OR_FAIL(ctx, J.dorient.alloc(8 * (size_t)ni * nq)); J.d_orient = J.dorient.as<double>(); }
  }
  return BIOEM_OK;
}

// Kernel arguments of images [i0, i0 + cn) of a job, records at rec.
LogpostArgs job_args(const Job& J, int i0, int cn, bioem_erec* rec) {
  LogpostArgs a{};
  a.ispec = J.imgs->spec + J.len * i0; a.iexpo = J.imgs->expo + i0; a.istats = J.imgs->stats + 3 * (size_t)i0;
  a.ni = cn;
  a.pspec = J.proj->spec; a.pexpo = J.proj->expo; a.nq = J.nq;
  a.table = J.table.as<float>(); a.B = J.B.as<double>(); a.nc = J.nc;
  a.itile = J.imgs->tile + tile_spec_len(J.nx, J.ny) * i0; a.ptile = J.proj->tile;
  a.ttile = J.ttable.p ? J.ttable.as<float4>() : nullptr;
  a.nx = J.nx; a.ny = J.ny; a.S = J.S; a.ldy = spec_ld(J.ny);
  a.cand = J.has_cand ? J.dcand.as<int32_t>() + (size_t)i0 * J.k : nullptr; a.k = J.k;
  a.rec = rec;
  a.kscale = 1.0 / ((double)J.nx * J.ny * (double)J.nx * J.ny);
  a.zs = J.zs;
  return a;
}

hipError_t finalize_chunk(hipStream_t s, const Job& J, const LogpostArgs& a, int i0, bool split) {
  FinalizeArgs f{};
  f.rec = a.rec; f.ni = a.ni; f.nslots = J.nslots; f.nc = J.nc; f.nq_total = J.nq; f.nx = J.nx; f.ny = J.ny;
  f.S = J.S; f.cand = a.cand; f.k = J.k;
  f.istats = a.istats; f.iexpo = a.iexpo; f.pexpo = J.proj->expo; f.B = a.B;
  f.log_prior = J.log_prior;
  f.logp = J.d_logp ? J.d_logp + i0 : nullptr;
  f.best = J.d_best ? J.d_best + i0 : nullptr;
  f.orient = J.d_orient ? J.d_orient + (size_t)i0 * J.nq : nullptr;
  hipError_t e = launch_finalize(s, f);
  if (e == hipSuccess && split && f.best) e = launch_best_shift(s, a, f.best);
  return e;
}

bioem_status ensure_events(bioem_ctx* ctx, int n) {
  while ((int)ctx->ev_start.size() < ctx->ev_used + n) {
    hipEvent_t a, b;
    HIP_OR_FAIL(ctx, hipEventCreate(&a));
    HIP_OR_FAIL(ctx, hipEventCreate(&b));
    ctx->ev_start.push_back(a);
    ctx->ev_stop.push_back(b);
  }
  return BIOEM_OK;
}

// Tile shape of the split kernel for a job: the tuned entry of its key, a
// new tuning run, or the default (BIOEM_SPLIT_SHAPE overrides the variant).
struct SplitCfg {
  int shape, ew, ti, ts;
};

constexpr int kTuneEW[] = {2, 4};   // the first is the default
constexpr int kTuneTiles[][2] = {{32, 128}, {16, 128}, {64, 64}, {8, 256}};   // the first is the default

int ilog2(int v) {
  int r = 0;
  while (v > 1) { v >>= 1; ++r; }
  return r;
}

bioem_status tune_job(bioem_ctx* ctx, const Job& J, int prec, bioem_tuning& out) {
  hipStream_t s = ctx->stream;
  const bool bf16 = prec == BIOEM_PREC_SPLIT_BF16;
  // a sample large enough that the item tiles meet the caches as in the
  // full job (a few hundred thousand evaluations per candidate)
  const int ni_s = std::min(J.ni, 128);
  const int nslots_s = J.has_cand ? J.k : std::min(J.nq, 2048);
  DevMem rec;
  HIP_OR_FAIL(ctx, rec.alloc(sizeof(bioem_erec) * (size_t)ni_s * nslots_s * J.nc));
  LogpostArgs a = job_args(J, 0, ni_s, rec.as<bioem_erec>());
  if (!J.has_cand) a.nq = nslots_s;   // the first orientations stand for the grid
  hipEvent_t e0, e1;
  HIP_OR_FAIL(ctx, hipEventCreate(&e0));
  HIP_OR_FAIL(ctx, hipEventCreate(&e1));
  const double evals = (double)ni_s * nslots_s * J.nc;
  double best = 1e300, def = 1e300;
  int bew = kTuneEW[0], bti = kTuneTiles[0][0], bts = kTuneTiles[0][1];
  hipError_t err = hipSuccess;
  for (int ew : kTuneEW)
    for (const auto& t : kTuneTiles) {
      const int shape = split_shape_for_ew(ew, bf16);
      float ms = 0.0f;
      for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {   // first run warms the caches
        err = hipEventRecord(e0, s);
        if (err == hipSuccess) err = launch_logpost_split(s, a, bf16, shape, t[0], t[1]);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      }
      if (err != hipSuccess) break;
      const double ns = ms * 1e6 / evals;
      if (ew == kTuneEW[0] && t[0] == kTuneTiles[0][0] && t[1] == kTuneTiles[0][1]) def = ns;
      if (ns < best) { best = ns; bew = ew; bti = t[0]; bts = t[1]; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(ctx, BIOEM_EDEVICE, "autotune: %s", hipGetErrorString(err));
  out = bioem_tuning{};
  out.nx = J.nx; out.ny = J.ny; out.max_shift = J.S; out.nq_log2 = ilog2(J.nq); out.prec = prec;
  out.ew = bew; out.tile_images = bti; out.tile_slots = bts;
  out.ns_per_eval = best; out.ns_per_eval_default = def;
  return BIOEM_OK;
}

bioem_status split_cfg(bioem_ctx* ctx, const Job& J, int prec, SplitCfg& cfg) {
  const bool bf16 = prec == BIOEM_PREC_SPLIT_BF16;
  cfg = SplitCfg{J.kernel > 0 ? J.kernel - 1 : split_shape_for_ew(2, bf16), 2, J.ti, J.ts};
  // an explicit launch shape or item tile (bioem_opts) bypasses the autotuner
  if (J.kernel > 0 || J.ti > 0 || !ctx->autotune) {
    cfg.ew = split_shape_ew(cfg.shape);
    return BIOEM_OK;
  }
  const int lq = ilog2(J.nq);
  for (const bioem_tuning& t : ctx->tuned)
    if (t.nx == J.nx && t.ny == J.ny && t.max_shift == J.S && t.nq_log2 == lq && t.prec == prec) {
      cfg = SplitCfg{split_shape_for_ew(t.ew, bf16), t.ew, t.tile_images, t.tile_slots};
      return BIOEM_OK;
    }
  bioem_tuning t;
  const bioem_status st = tune_job(ctx, J, prec, t);
  if (st != BIOEM_OK) return st;
  ctx->tuned.push_back(t);
  cfg = SplitCfg{split_shape_for_ew(t.ew, bf16), t.ew, t.tile_images, t.tile_slots};
  return BIOEM_OK;
}

// One job: image chunks bounded by the record budget (by what is left of
// the carve, when one is given), main kernel, then the FP64 finalisation of
// each chunk.
bioem_status run_job(bioem_ctx* ctx, Job& J, int prec, Carve* carve = nullptr) {
  hipStream_t s = ctx->stream;
  const bool split = prec != BIOEM_PREC_F32;
  SplitCfg cfg{0, 4, 0, 0};
  if (split) {
    const bioem_status st = split_cfg(ctx, J, prec, cfg);
    if (st != BIOEM_OK) return st;
  }
  const size_t per_image = sizeof(bioem_erec) * (size_t)J.nslots * J.nc;
  const size_t budget = carve ? carve->left() : kRecordBudget;
  if (carve && budget < per_image)
    return fail(ctx, BIOEM_EUNSUPPORTED, "bioem_logpost: records of one image (%zu B) exceed the scratch left (%zu B)",
                per_image, budget);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(J.ni, budget / per_image));
  DevMem rec;
  HIP_OR_FAIL(ctx, rec.get(per_image * chunk, carve));
  const int nchunks = (J.ni + chunk - 1) / chunk;
  const bool timing = ctx->timing && !carve;   // event creation stays out of the allocation-free form
  if (timing) {
    const bioem_status st = ensure_events(ctx, nchunks);
    if (st != BIOEM_OK) return st;
  }
  for (int i0 = 0; i0 < J.ni; i0 += chunk) {
    const int cn = std::min(chunk, J.ni - i0);
    const LogpostArgs a = job_args(J, i0, cn, rec.as<bioem_erec>());
    if (timing) HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev_start[ctx->ev_used], s));
    hipError_t e = split  ? launch_logpost_split(s, a, prec == BIOEM_PREC_SPLIT_BF16, cfg.shape, cfg.ti, cfg.ts)
                   : J.mf ? launch_logpost_mf32(s, a, J.imgs->mf + mf_len(J.nx, J.ny) * i0, J.proj->mf,
                                                J.mftm.as<float4>(), J.mftab.as<float4>(), J.ti, J.ts)
                          : launch_logpost_f32(s, a);
    if (timing && e == hipSuccess) {
      HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev_stop[ctx->ev_used], s));
      ++ctx->ev_used;
      ctx->timed_evals += (double)cn * J.nslots * J.nc;
    }
    if (e == hipSuccess) e = finalize_chunk(s, J, a, i0, split || J.mf);
    if (e != hipSuccess) return fail(ctx, BIOEM_EDEVICE, "bioem_logpost: launch failed: %s", hipGetErrorString(e));
  }
  return BIOEM_OK;
}

// Every job's evaluations in one persistent launch (per round of image
// chunks when the records of all jobs exceed the budget), then per-job
// finalisation.
bioem_status run_batch_persistent(bioem_ctx* ctx, std::vector<Job>& J, int prec) {
  hipStream_t s = ctx->stream;
  const int nj = (int)J.size();
  std::vector<SplitCfg> cfg(nj);
  size_t total = 0;
  for (int j = 0; j < nj; ++j) {
    const bioem_status st = split_cfg(ctx, J[j], prec, cfg[j]);
    if (st != BIOEM_OK) return st;
    total += sizeof(bioem_erec) * (size_t)J[j].ni * J[j].nslots * J[j].nc;
  }
  const int rounds = (int)std::max<size_t>(1, (total + kBatchRecordBudget - 1) / kBatchRecordBudget);
  std::vector<int> chunk(nj);
  size_t per_round = 0;
  for (int j = 0; j < nj; ++j) {
    chunk[j] = std::max(1, (J[j].ni + rounds - 1) / rounds);
    per_round += sizeof(bioem_erec) * (size_t)chunk[j] * J[j].nslots * J[j].nc;
  }
  DevMem rec;
  HIP_OR_FAIL(ctx, rec.alloc(per_round));
  if (ctx->timing) {
    const bioem_status st = ensure_events(ctx, rounds);
    if (st != BIOEM_OK) return st;
  }
  for (int r = 0; r < rounds; ++r) {
    std::vector<BatchJob> bj;
    std::vector<int> which, first;
    size_t off = 0;
    double evals = 0.0;
    for (int j = 0; j < nj; ++j) {
      const int i0 = r * chunk[j];
      if (i0 >= J[j].ni) continue;
      const int cn = std::min(chunk[j], J[j].ni - i0);
      BatchJob b;
      b.a = job_args(J[j], i0, cn, reinterpret_cast<bioem_erec*>(static_cast<char*>(rec.p) + off));
      b.ew = cfg[j].ew; b.ti = cfg[j].ti; b.ts = cfg[j].ts;
      bj.push_back(b);
      which.push_back(j);
      first.push_back(i0);
      off += sizeof(bioem_erec) * (size_t)cn * J[j].nslots * J[j].nc;
      evals += (double)cn * J[j].nslots * J[j].nc;
    }
    if (bj.empty()) continue;
    if (ctx->timing) HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev_start[ctx->ev_used], s));
    hipError_t e = launch_logpost_batch(s, bj.data(), (int)bj.size(), prec == BIOEM_PREC_SPLIT_BF16);
    if (ctx->timing && e == hipSuccess) {
      HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev_stop[ctx->ev_used], s));
      ++ctx->ev_used;
      ctx->timed_evals += evals;
    }
    for (size_t b = 0; b < bj.size() && e == hipSuccess; ++b) e = finalize_chunk(s, J[which[b]], bj[b].a, first[b], true);
    if (e != hipSuccess)
      return fail(ctx, BIOEM_EDEVICE, "bioem_logpost_batch: launch failed: %s", hipGetErrorString(e));
  }
  return BIOEM_OK;
}

bioem_status copy_out(bioem_ctx* ctx, Job& J, int out_mem) {
  if (out_mem != BIOEM_MEM_HOST) return BIOEM_OK;
  hipStream_t s = ctx->stream;
  if (J.logp) HIP_OR_FAIL(ctx, hipMemcpyAsync(J.logp, J.d_logp, 8 * (size_t)J.ni, hipMemcpyDeviceToHost, s));
  if (J.best)
    HIP_OR_FAIL(ctx, hipMemcpyAsync(J.best, J.d_best, sizeof(bioem_best) * (size_t)J.ni, hipMemcpyDeviceToHost, s));
  if (J.orient)
    HIP_OR_FAIL(ctx, hipMemcpyAsync(J.orient, J.d_orient, 8 * (size_t)J.ni * J.nq, hipMemcpyDeviceToHost, s));
  return BIOEM_OK;
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
  // NULL is the device's null (legacy default) stream, which other users of
  // that stream (e.g. a framework's default stream) are ordered with
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->scratch = scratch_address(device);
  *out = ctx;
  return BIOEM_OK;
}

void bioem_destroy(bioem_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto e : ctx->ev_start) (void)hipEventDestroy(e);
  for (auto e : ctx->ev_stop) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(ctx->stream);
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
  if (p->tile) (void)hipFree(p->tile);
  if (p->mf) (void)hipFree(p->mf);
  if (p->expo) (void)hipFree(p->expo);
  delete p;
}

void bioem_free_imgs(bioem_imgs* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->spec) (void)hipFree(p->spec);
  if (p->tile) (void)hipFree(p->tile);
  if (p->mf) (void)hipFree(p->mf);
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
  const size_t tlen = tile_spec_len(nx, ny), mlen = mf_len(nx, ny);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->spec), sizeof(float2) * slen * nq);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->tile), sizeof(float4) * tlen * nq);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->mf), sizeof(float4) * mlen * nq);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->expo), sizeof(int32_t) * nq);
  if (e != hipSuccess) {
    bioem_free_proj(p);
    return fail(ctx, BIOEM_ENOMEM, "bioem_project: device allocation of %zu MB failed",
                ((sizeof(float2) * slen + sizeof(float4) * (tlen + mlen)) * nq) >> 20);
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
    if (e == hipSuccess) e = launch_tile_spec(s, p->spec + slen * q0, cn, nx, ny, p->tile + tlen * q0);
    if (e == hipSuccess) e = launch_mf_copy_spec(s, p->spec + slen * q0, cn, nx, ny, false, p->mf + mlen * q0);
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
  // every pixel must be finite (checked before any work is enqueued)
  if (in_mem == BIOEM_MEM_HOST) {
    for (size_t e = 0; e < npix * ni; ++e)
      if (!std::isfinite(imgs[e]))
        return fail(ctx, BIOEM_EINVAL, "bioem_prepare_images: pixel %zu of image %zu is not finite", e % npix,
                    e / npix);
  } else {
    DevMem flag;
    unsigned hflag = 0;
    HIP_OR_FAIL(ctx, flag.alloc(sizeof(unsigned)));
    HIP_OR_FAIL(ctx, hipMemsetAsync(flag.p, 0, sizeof(unsigned), s));
    HIP_OR_FAIL(ctx, launch_flag_nonfinite(s, imgs, npix * ni, flag.as<unsigned>()));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&hflag, flag.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
    if (hflag) return fail(ctx, BIOEM_EINVAL, "bioem_prepare_images: an image holds a non-finite pixel");
  }
  bioem_imgs* p = new (std::nothrow) bioem_imgs;
  if (!p) return fail(ctx, BIOEM_ENOMEM, "bioem_prepare_images: host allocation");
  p->n = ni; p->nx = nx; p->ny = ny; p->device = ctx->device;
  const size_t tlen = tile_spec_len(nx, ny), mlen = mf_len(nx, ny);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->spec), sizeof(float2) * slen * ni);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->tile), sizeof(float4) * tlen * ni);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->mf), sizeof(float4) * mlen * ni);
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
    if (e == hipSuccess) e = launch_tile_spec(s, p->spec + slen * i0, cn, nx, ny, p->tile + tlen * i0);
    if (e == hipSuccess) e = launch_mf_copy_spec(s, p->spec + slen * i0, cn, nx, ny, true, p->mf + mlen * i0);
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
  bioem_opts o{};
  if (opts) o = *opts;
  if (o.reserved) return fail(ctx, BIOEM_EINVAL, "bioem_logpost: opts.reserved must be zero");
  bioem_job jb{};
  jb.proj = proj; jb.imgs = imgs; jb.ctf = ctf; jb.nc = nc; jb.ctf_mem = ctf_mem; jb.max_shift = max_shift;
  jb.k = o.k; jb.cand_q = o.cand_q; jb.cand_mem = o.cand_mem;
  jb.logp = logp; jb.best = best; jb.logp_orient = o.logp_orient;
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  Job J;
  bioem_status st = plan_job(ctx, jb, o.prec, o.out_mem, J, "bioem_logpost", o.kernel, o.tile_images, o.tile_slots);
  if (st != BIOEM_OK) return st;
  st = run_job(ctx, J, o.prec);
  if (st != BIOEM_OK) return st;
  st = copy_out(ctx, J, o.out_mem);
  if (st != BIOEM_OK) return st;
  // Scratch (table, B, records) is freed on return, so the stream must drain.
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  return BIOEM_OK;
}

bioem_status bioem_logpost_noalloc(bioem_ctx* ctx, const bioem_proj* proj, const bioem_imgs* imgs,
                                   const double* ctf, int32_t nc, int32_t max_shift, double* logp,
                                   bioem_best* best) {
  if (!ctx) return BIOEM_EINVAL;
  if (!ctx->scratch)
    return fail(ctx, BIOEM_EDEVICE, "bioem_logpost_noalloc: scratch address of device %d unavailable", ctx->device);
  if (proj && imgs) {
    // the fixed tables and one image's records must fit
    const size_t nq = (size_t)std::max(proj->n, 0), ncs = (size_t)std::max(nc, 0);
    const size_t len = (size_t)(proj->nx / 2 + 1) * spec_ld(proj->ny);
    const bool mf = nc > 0 && valid_box(proj->nx, proj->ny) && max_shift >= 0 &&
                    2 * max_shift < std::min(proj->nx, proj->ny) && mf32_supported(proj->nx, proj->ny, max_shift);
    size_t need = Carve::up(24 * ncs) + Carve::up(4 * len * ncs) + Carve::up(8 * nq * ncs) +
                  Carve::up(sizeof(bioem_erec) * nq * ncs);
    if (mf)
      need += Carve::up(sizeof(float4) * mf32_table_len(proj->nx, proj->ny)) +
              Carve::up(sizeof(float4) * mf_table_len(proj->nx, proj->ny) * ncs);
    if (need > kNoAllocBytes)
      return fail(ctx, BIOEM_EUNSUPPORTED,
                  "bioem_logpost_noalloc: needs %zu bytes of scratch for %zu orientations x %zu CTF sets, more than "
                  "its %zu",
                  need, nq, ncs, kNoAllocBytes);
  }
  bioem_job jb{};
  jb.proj = proj; jb.imgs = imgs; jb.ctf = ctf; jb.nc = nc; jb.ctf_mem = BIOEM_MEM_HOST; jb.max_shift = max_shift;
  jb.logp = logp; jb.best = best;
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  Carve carve;
  carve.base = static_cast<char*>(ctx->scratch);
  carve.cap = kNoAllocBytes;
  Job J;
  bioem_status st = plan_job(ctx, jb, BIOEM_PREC_F32, BIOEM_MEM_DEVICE, J, "bioem_logpost_noalloc", 0, 0, 0, &carve);
  if (st != BIOEM_OK) return st;
  return run_job(ctx, J, BIOEM_PREC_F32, &carve);
}

bioem_status bioem_logpost_batch(bioem_ctx* ctx, const bioem_job* jobs, int32_t njobs, int32_t prec,
                                 int32_t out_mem, int32_t mode) {
  if (!ctx) return BIOEM_EINVAL;
  if (!jobs || njobs < 1) return fail(ctx, BIOEM_EINVAL, "bioem_logpost_batch: need njobs >= 1 jobs");
  if (mode != BIOEM_BATCH_PERSISTENT && mode != BIOEM_BATCH_PER_JOB)
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost_batch: unknown mode %d", mode);
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  std::vector<Job> J(njobs);
  for (int j = 0; j < njobs; ++j) {
    if (jobs[j].reserved) return fail(ctx, BIOEM_EINVAL, "bioem_logpost_batch: job %d reserved must be zero", j);
    char who[64];
    std::snprintf(who, sizeof who, "bioem_logpost_batch (job %d)", j);
    const bioem_status st = plan_job(ctx, jobs[j], prec, out_mem, J[j], who);
    if (st != BIOEM_OK) return st;
  }
  bioem_status st = BIOEM_OK;
  if (mode == BIOEM_BATCH_PER_JOB || prec == BIOEM_PREC_F32) {
    for (int j = 0; j < njobs && st == BIOEM_OK; ++j) st = run_job(ctx, J[j], prec);
  } else {
    st = run_batch_persistent(ctx, J, prec);
  }
  for (int j = 0; j < njobs && st == BIOEM_OK; ++j) st = copy_out(ctx, J[j], out_mem);
  if (st != BIOEM_OK) return st;
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  return BIOEM_OK;
}

bioem_status bioem_set_autotune(bioem_ctx* ctx, int32_t enable) {
  if (!ctx) return BIOEM_EINVAL;
  ctx->autotune = enable != 0;
  return BIOEM_OK;
}

int32_t bioem_tuning_count(const bioem_ctx* ctx) { return ctx ? (int32_t)ctx->tuned.size() : 0; }

bioem_status bioem_tuning_entry(const bioem_ctx* ctx, int32_t idx, bioem_tuning* out) {
  if (!ctx || !out || idx < 0 || idx >= (int32_t)ctx->tuned.size()) return BIOEM_EINVAL;
  *out = ctx->tuned[idx];
  return BIOEM_OK;
}

bioem_status bioem_project_euler(bioem_ctx* ctx, const double* spheres, int32_t ns, const double* euler, int32_t nq,
                                 int32_t nx, int32_t ny, double pixel_A, bioem_mem in_mem, bioem_proj** out) {
  if (!ctx) return BIOEM_EINVAL;
  if (!out) return fail(ctx, BIOEM_EINVAL, "bioem_project_euler: out is NULL");
  *out = nullptr;
  if (!spheres || !euler || ns < 1 || nq < 1 || !valid_mem(in_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_project_euler: bad argument");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::vector<double> he;
  HIP_OR_FAIL(ctx, to_host(euler, (size_t)nq * 3, in_mem, s, he));
  if (!finite_all(he.data(), he.size())) return fail(ctx, BIOEM_EINVAL, "bioem_project_euler: non-finite angle");
  DevIn de, dsp;
  HIP_OR_FAIL(ctx, de.set(euler, sizeof(double) * 3 * (size_t)nq, in_mem, s));
  HIP_OR_FAIL(ctx, dsp.set(spheres, sizeof(double) * 5 * (size_t)ns, in_mem, s));
  DevMem dq;
  HIP_OR_FAIL(ctx, dq.alloc(sizeof(double) * 4 * (size_t)nq));
  HIP_OR_FAIL(ctx, launch_euler_quat(s, de.as<double>(), nq, dq.as<double>()));
  return bioem_project(ctx, dsp.as<double>(), ns, dq.as<double>(), nq, nx, ny, pixel_A, BIOEM_MEM_DEVICE, out);
}

}  // extern "C"

namespace {

// The cropping posterior with calculated images from the Fourier filter of
// Eq. (4) (psf_radius < 0) or the real-space PSF convolution of Eq. (5).
bioem_status crop_impl(bioem_ctx* ctx, const bioem_proj* proj, const float* imgs, int32_t ni, int32_t in_mem,
                       const double* ctf, int32_t nc, int32_t max_shift, int32_t psf_radius, double* logp,
                       bioem_best* best, int32_t out_mem) {
  if (!proj || !imgs || !ctf || !logp || !best || ni < 1 || nc < 1 || !valid_mem(in_mem) || !valid_mem(out_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop: bad argument");
  const int nx = proj->nx, ny = proj->ny, nq = proj->n, S = max_shift;
  if (proj->device != ctx->device) return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop: handle on another device");
  if (S < 0 || 2 * S >= std::min(nx, ny))
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop: max_shift %d outside [0, min(nx, ny)/2)", S);
  if (S > kCropMaxShift || crop_smem_bytes(nx, S) > kMaxSmem)
    return fail(ctx, BIOEM_EUNSUPPORTED, "bioem_logpost_crop: the direct form takes max_shift <= %d (and "
                "%zu bytes of LDS at this box)", kCropMaxShift, crop_smem_bytes(nx, S));
  if ((size_t)nq * nc > (size_t)INT32_MAX / 2)
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop: too many orientation x CTF pairs");
  const int R = psf_radius;
  if (R >= 0 && 2 * R >= std::min(nx, ny))
    return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop_psf: psf_radius %d outside [0, min(nx, ny)/2)", R);
  if (R > kPsfMaxRadius)
    return fail(ctx, BIOEM_EUNSUPPORTED, "bioem_logpost_crop_psf: psf_radius %d above %d", R, kPsfMaxRadius);
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int np = nq * nc, W = (2 * S + 1) * (2 * S + 1), mh = nx / 2 + 1;
  const size_t npix = (size_t)nx * ny, len = (size_t)mh * ny, slen = (size_t)mh * spec_ld(ny);
  std::vector<double> hc;
  HIP_OR_FAIL(ctx, to_host(ctf, (size_t)nc * 3, (bioem_mem)in_mem, s, hc));
  if (!finite_all(hc.data(), hc.size())) return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop: non-finite CTF value");
  for (int c = 0; c < nc; ++c)
    if (!(hc[3 * c + 1] >= 0.0 && hc[3 * c + 1] <= 1.0))
      return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop: amplitude contrast of set %d outside [0,1]", c);
  DevIn dimg;
  HIP_OR_FAIL(ctx, dimg.set(imgs, sizeof(float) * npix * ni, (bioem_mem)in_mem, s));
  DevMem stats, P, Bd, rec, crep, shifts, dlogp, dbest;
  HIP_OR_FAIL(ctx, stats.alloc(sizeof(double) * 3 * (size_t)ni));
  HIP_OR_FAIL(ctx, launch_image_stats(s, dimg.as<float>(), ni, (int)npix, stats.as<double>()));
  // calculated images I1 = F^-1[F(I0) CTF Env], one per (CTF set, orientation)
  HIP_OR_FAIL(ctx, P.alloc(sizeof(float) * npix * np));
  HIP_OR_FAIL(ctx, crep.alloc(sizeof(double) * 3 * (size_t)nq));
  HIP_OR_FAIL(ctx, shifts.alloc(sizeof(int32_t) * 2 * (size_t)nq));
  HIP_OR_FAIL(ctx, hipMemsetAsync(shifts.p, 0, sizeof(int32_t) * 2 * (size_t)nq, s));
  std::vector<double> rep(3 * (size_t)nq);
  const size_t per = len * 16 + (size_t)ny * mh * 16 + npix * 8;
  const int chunk = chunk_items(nq, per);
  DevMem s64, cols, i1;
  HIP_OR_FAIL(ctx, s64.alloc((size_t)chunk * len * 16));
  HIP_OR_FAIL(ctx, cols.alloc((size_t)chunk * ny * mh * 16));
  HIP_OR_FAIL(ctx, i1.alloc((size_t)chunk * npix * 8));
  if (R >= 0) {
    // Eq. (5): each CTF set's PSF, truncated to the disc of radius R, then
    // every ideal image convolved with it on the box
    const size_t w2 = (size_t)(2 * R + 1) * (2 * R + 1);
    DevIn dctf;
    DevMem pspec, pcols, ppsf, K;
    HIP_OR_FAIL(ctx, dctf.set(hc.data(), hc.size() * 8, BIOEM_MEM_HOST, s));
    HIP_OR_FAIL(ctx, pspec.alloc((size_t)nc * len * 16));
    HIP_OR_FAIL(ctx, pcols.alloc((size_t)nc * ny * mh * 16));
    HIP_OR_FAIL(ctx, ppsf.alloc((size_t)nc * npix * 8));
    HIP_OR_FAIL(ctx, K.alloc(sizeof(double) * nc * w2));
    HIP_OR_FAIL(ctx, launch_psf_kernels(s, dctf.as<double>(), nc, nx, ny, proj->pixel, R, pspec.as<double2>(),
                                        pcols.as<double2>(), ppsf.as<double>(), K.as<double>()));
    for (int q0 = 0; q0 < nq; q0 += chunk) {
      const int cn = std::min(chunk, nq - q0);
      HIP_OR_FAIL(ctx, launch_ideal(s, proj->spec + slen * q0, proj->expo + q0, cn, nx, ny, s64.as<double2>(),
                                    cols.as<double2>(), i1.as<double>()));
      for (int c = 0; c < nc; ++c)
        HIP_OR_FAIL(ctx, launch_psf_conv(s, i1.as<double>(), cn, nx, ny, K.as<double>() + w2 * c, R,
                                         P.as<float>() + npix * ((size_t)c * nq + q0)));
    }
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s));   // the PSF buffers are freed on leaving this block
  }
  for (int c = 0; c < nc && R < 0; ++c) {
    for (int q = 0; q < nq; ++q)
      for (int k = 0; k < 3; ++k) rep[3 * (size_t)q + k] = hc[3 * (size_t)c + k];
    HIP_OR_FAIL(ctx, hipMemcpyAsync(crep.p, rep.data(), rep.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s));   // rep is rewritten for the next set
    for (int q0 = 0; q0 < nq; q0 += chunk) {
      const int cn = std::min(chunk, nq - q0);
      HIP_OR_FAIL(ctx, launch_render(s, proj->spec + slen * q0, proj->expo + q0, cn, nx, ny, proj->pixel,
                                     crep.as<double>() + 3 * (size_t)q0, shifts.as<int32_t>() + 2 * (size_t)q0,
                                     nullptr, nullptr, 1.0, s64.as<double2>(), cols.as<double2>(),
                                     i1.as<double>(), P.as<float>() + npix * ((size_t)c * nq + q0)));
    }
  }
  HIP_OR_FAIL(ctx, Bd.alloc(sizeof(double) * W * (size_t)np));
  CropArgs a{};
  a.p = P.as<float>(); a.np = np; a.nq = nq; a.nx = nx; a.ny = ny; a.S = S; a.Bd = Bd.as<double>();
  HIP_OR_FAIL(ctx, launch_crop_norms(s, a));
  // per-evaluation records for a chunk of images at a time
  const int ci = std::max(1, std::min<int>(ni, (int)std::min<size_t>(kScratchBudget / (sizeof(bioem_crec) * np),
                                                                      (size_t)INT32_MAX)));
  HIP_OR_FAIL(ctx, rec.alloc(sizeof(bioem_crec) * (size_t)ci * np));
  double* lo = logp;
  bioem_best* bo = best;
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, dlogp.alloc(sizeof(double) * ni));
    HIP_OR_FAIL(ctx, dbest.alloc(sizeof(bioem_best) * ni));
    lo = dlogp.as<double>();
    bo = dbest.as<bioem_best>();
  }
  const double log_prior = -std::log((double)nq) - std::log((double)nc) - std::log((double)W);
  for (int i0 = 0; i0 < ni; i0 += ci) {
    a.imgs = dimg.as<float>() + npix * i0;
    a.stats = stats.as<double>() + 3 * (size_t)i0;
    a.ni = std::min(ci, ni - i0);
    a.rec = rec.as<bioem_crec>();
    HIP_OR_FAIL(ctx, launch_crop_xcorr(s, a));
    HIP_OR_FAIL(ctx, launch_crop_finalize(s, a, log_prior, lo + i0, bo + i0));
  }
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, hipMemcpyAsync(logp, lo, sizeof(double) * ni, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(best, bo, sizeof(bioem_best) * ni, hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

}  // namespace

extern "C" {

bioem_status bioem_logpost_crop(bioem_ctx* ctx, const bioem_proj* proj, const float* imgs, int32_t ni,
                                int32_t in_mem, const double* ctf, int32_t nc, int32_t max_shift, double* logp,
                                bioem_best* best, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  return crop_impl(ctx, proj, imgs, ni, in_mem, ctf, nc, max_shift, -1, logp, best, out_mem);
}

bioem_status bioem_logpost_crop_psf(bioem_ctx* ctx, const bioem_proj* proj, const float* imgs, int32_t ni,
                                    int32_t in_mem, const double* ctf, int32_t nc, int32_t max_shift,
                                    int32_t psf_radius, double* logp, bioem_best* best, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (psf_radius < 0) return fail(ctx, BIOEM_EINVAL, "bioem_logpost_crop_psf: psf_radius %d < 0", psf_radius);
  return crop_impl(ctx, proj, imgs, ni, in_mem, ctf, nc, max_shift, psf_radius, logp, best, out_mem);
}

bioem_status bioem_ensemble(bioem_ctx* ctx, const double* logp, int32_t nm, int32_t ni, int32_t in_mem,
                            const double* w, double* per_image, double* total, int32_t out_mem) {
  if (!ctx) return BIOEM_EINVAL;
  if (!w || !total || nm < 1 || ni < 0 || (ni > 0 && !logp) || !valid_mem(in_mem) || !valid_mem(out_mem))
    return fail(ctx, BIOEM_EINVAL, "bioem_ensemble: bad argument");
  double wsum = 0.0;
  for (int m = 0; m < nm; ++m) {
    if (!std::isfinite(w[m]) || w[m] < 0.0)
      return fail(ctx, BIOEM_EINVAL, "bioem_ensemble: weight %d is negative or not finite", m);
    wsum += w[m];
  }
  if (!(std::fabs(wsum - 1.0) <= 1e-9))
    return fail(ctx, BIOEM_EINVAL, "bioem_ensemble: weights sum to %.17g, not 1", wsum);
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  DevIn dl, dw;
  HIP_OR_FAIL(ctx, dl.set(ni > 0 ? logp : nullptr, sizeof(double) * (size_t)nm * ni, (bioem_mem)in_mem, s));
  HIP_OR_FAIL(ctx, dw.set(w, sizeof(double) * (size_t)nm, BIOEM_MEM_HOST, s));
  DevMem dper, dtot;
  double* per = per_image;
  double* tot = total;
  if (out_mem == BIOEM_MEM_HOST || !per_image) {
    HIP_OR_FAIL(ctx, dper.alloc(sizeof(double) * (size_t)ni));
    per = dper.as<double>();
  }
  if (out_mem == BIOEM_MEM_HOST) {
    HIP_OR_FAIL(ctx, dtot.alloc(sizeof(double)));
    tot = dtot.as<double>();
  }
  HIP_OR_FAIL(ctx, launch_ensemble(s, dl.as<double>(), nm, ni, dw.as<double>(), per, tot));
  if (out_mem == BIOEM_MEM_HOST) {
    if (per_image && ni > 0)
      HIP_OR_FAIL(ctx, hipMemcpyAsync(per_image, per, sizeof(double) * (size_t)ni, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(total, tot, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIP_OR_FAIL(ctx, hipStreamSynchronize(s));
  return BIOEM_OK;
}

}  // extern "C"
