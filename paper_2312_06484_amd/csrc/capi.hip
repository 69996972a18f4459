// C ABI of the AIRPF library (declared in include/airpf.h): argument
// validation, model constants, device workspaces and launches.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "airpf.h"
#include "internal.h"

namespace {

// AIRPF_WORKSPACE_CAP=<bytes>: no context buffer may grow beyond this size
// (a request that needs more reports AIRPF_E_NOMEM, as a failed allocation
// would); read at each growth
size_t workspace_cap() {
  const char* e = std::getenv("AIRPF_WORKSPACE_CAP");
  if (!e) return ~size_t(0);
  const long long v = std::atoll(e);
  return v > 0 ? static_cast<size_t>(v) : ~size_t(0);
}

// Grow-only device buffer owned by a context.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  airpf_status ensure(size_t bytes) {
    if (bytes <= cap) return AIRPF_OK;
    if (bytes > workspace_cap()) return AIRPF_E_NOMEM;
    if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
    size_t want = bytes < 256 ? 256 : bytes;
    if (hipMalloc(&p, want) != hipSuccess) { p = nullptr; return AIRPF_E_NOMEM; }
    cap = want;
    return AIRPF_OK;
  }
  void release() { if (p) (void)hipFree(p); p = nullptr; cap = 0; }
};

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }
// at most 1024 blocks of at most 256 islands each per problem
constexpr int kMaxIslands = 65536;
constexpr int kMaxBlocks = 1024;
int ilog2(int64_t v) { int s = 0; while ((int64_t(1) << s) < v) ++s; return s; }
bool all_finite(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i) if (!std::isfinite(p[i])) return false;
  return true;
}

// Fixed device scratch of airpf_run_noalloc: every workspace of such a call
// (resampled states, island tree, ENF records, barrier flags, the record
// ring, uploaded observations) is carved from this array, so the call
// allocates nothing.  Each device the library runs on holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in,
// never the device memory: host code uses the per-device address that
// hipGetSymbolAddress returned (scratch_addr below), never the array's name.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// Resolves (once per device, with that device current) the device address of
// this device's copy of the scratch array; nullptr on failure.
unsigned char* scratch_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  return g_scratch_ptr[device];
}

}  // namespace

struct airpf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  unsigned char* scratch = nullptr;   // this device's copy of the no-allocation scratch array
  hipEvent_t ev[2] = {nullptr, nullptr};
  double last_kernel_ms = 0.0;
  DevBuf x1[2], tree[2], part[2], misc, ybuf, ad_lc[2], ad_dq[2];
  DevBuf t_sstar, t_enf, t_lpost, t_anc, t_pi, t_dig, t_fmean;
  DevBuf s_pi, s_sstar, s_lpre, s_ckx, s_ckL, s_recx, s_reca, s_lam[2], s_del[2], s_grad, s_nu;
  DevBuf dbg_in, dbg_in32, dbg_out, dbg_out2, dbg_out32;
  DevBuf batch;
  // tiler cost ratios (pass time / step overhead) and particles per lane
  // measured by AIRPF_FLAG_AUTOTUNE, keyed by batch shape
  std::map<uint64_t, double> tuned_ratio;
  std::map<uint64_t, int> tuned_ppt;
};

#define HIP_OK(expr) do { if ((expr) != hipSuccess) return AIRPF_E_DEVICE; } while (0)
#define ST_OK(expr) do { airpf_status _s = (expr); if (_s != AIRPF_OK) return _s; } while (0)

extern "C" const char* airpf_status_str(airpf_status s) {
  switch (s) {
    case AIRPF_OK: return "ok";
    case AIRPF_E_INVALID_ARG: return "invalid argument";
    case AIRPF_E_DOMAIN: return "parameter outside the model's domain";
    case AIRPF_E_NOMEM: return "device memory allocation failed";
    case AIRPF_E_DEVICE: return "device error";
    case AIRPF_E_UNSUPPORTED: return "unsupported request";
    case AIRPF_E_TOO_LARGE: return "workspace exceeds the fixed no-allocation scratch (64 MiB per device)";
  }
  return "unknown status";
}

extern "C" airpf_status airpf_ctx_create(int device, void* hip_stream, airpf_ctx** out) {
  if (!out) return AIRPF_E_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return AIRPF_E_DEVICE;
  HIP_OK(hipSetDevice(device));
  auto* c = new airpf_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess ||
      (c->scratch = scratch_addr(device)) == nullptr) {
    for (hipEvent_t e : c->ev) if (e) (void)hipEventDestroy(e);
    delete c;
    return AIRPF_E_DEVICE;
  }
  *out = c;
  return AIRPF_OK;
}

extern "C" airpf_status airpf_ctx_destroy(airpf_ctx* c) {
  if (!c) return AIRPF_E_INVALID_ARG;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
  for (DevBuf* b : {&c->x1[0], &c->x1[1], &c->tree[0], &c->tree[1], &c->part[0], &c->part[1], &c->misc,
                    &c->ad_lc[0], &c->ad_lc[1], &c->ad_dq[0], &c->ad_dq[1],
                    &c->ybuf, &c->t_sstar, &c->t_enf, &c->t_lpost, &c->t_anc, &c->t_pi, &c->t_dig, &c->t_fmean,
                    &c->dbg_in, &c->dbg_in32, &c->dbg_out, &c->dbg_out2, &c->dbg_out32, &c->s_pi,
                    &c->s_sstar, &c->s_lpre, &c->s_ckx, &c->s_ckL, &c->s_recx, &c->s_reca, &c->s_lam[0],
                    &c->s_lam[1], &c->s_del[0], &c->s_del[1], &c->s_grad, &c->s_nu, &c->batch})
    b->release();
  for (hipEvent_t e : c->ev) if (e) (void)hipEventDestroy(e);
  delete c;
  return AIRPF_OK;
}

namespace {

// Validates the model and theta, fills the model block of the kernel
// arguments and the weight constant cst = c - 40 log 2 - log N, where c is the
// additive constant of log g_n.  The constants follow the model definitions
// in include/airpf.h.
airpf_status prepare_model(const airpf_model* model, const double* theta, int32_t d_theta, int32_t N,
                           airpf::ModelArgs* mp, double* cst_q, int* dx_out, int* dy_out) {
  std::memset(mp, 0, sizeof(*mp));
  if (!model || (!theta && d_theta != 0)) return AIRPF_E_INVALID_ARG;
  const double LOG2PI = std::log(2.0 * M_PI);
  double c_log = 0.0;
  int dx = 1, dy = 1;
  switch (model->kind) {
    case AIRPF_LG1: {
      if (d_theta != 3 || model->dx != 1 || model->dy != 1) return AIRPF_E_INVALID_ARG;
      if (!all_finite(theta, 3)) return AIRPF_E_INVALID_ARG;
      if (!(theta[1] > 0.0) || !(theta[2] > 0.0)) return AIRPF_E_DOMAIN;
      c_log = -std::log(theta[2]) - 0.5 * LOG2PI;
      break;
    }
    case AIRPF_SV: {
      if (d_theta != 3 || model->dx != 1 || model->dy != 1) return AIRPF_E_INVALID_ARG;
      if (!all_finite(theta, 3)) return AIRPF_E_INVALID_ARG;
      if (!(std::fabs(theta[1]) < 1.0) || !(theta[2] > 0.0)) return AIRPF_E_DOMAIN;
      mp->s0 = theta[2] / std::sqrt(1.0 - theta[1] * theta[1]);
      {
        const double om = 1.0 - theta[1] * theta[1];
        mp->ds0_dphi = theta[2] * theta[1] / (om * std::sqrt(om));
        mp->ds0_dsig = 1.0 / std::sqrt(om);
      }
      c_log = -0.5 * LOG2PI;
      break;
    }
    case AIRPF_LGD: {
      dx = model->dx;
      dy = model->dy;
      if (!(dx == 2 || dx == 3 || dx == 4 || dx == 8) || dy < 1 || dy > airpf::kMaxDy) return AIRPF_E_INVALID_ARG;
      if (d_theta != dx * dx || !model->consts || model->n_consts != 3 + dx * dy) return AIRPF_E_INVALID_ARG;
      if (!all_finite(theta, d_theta) || !all_finite(model->consts, model->n_consts)) return AIRPF_E_INVALID_ARG;
      const double q = model->consts[0], r = model->consts[1], p0 = model->consts[2];
      if (!(q > 0.0) || !(r > 0.0) || !(p0 > 0.0)) return AIRPF_E_DOMAIN;
      mp->sq = std::sqrt(q);
      mp->sp0 = std::sqrt(p0);
      mp->hr = 1.0 / (2.0 * r);
      for (int i = 0; i < dx * dy; ++i) mp->H[i] = model->consts[3 + i];
      c_log = -(0.5 * static_cast<double>(dy)) * std::log(2.0 * M_PI * r);
      break;
    }
    case AIRPF_BIN: {
      if (d_theta != 0 || model->dx != 1 || model->dy != 1) return AIRPF_E_INVALID_ARG;
      mp->log3 = std::log(3.0);
      c_log = std::log(0.75);
      break;
    }
    case AIRPF_BCP: {
      if (d_theta != 1 || model->dx != 2 || model->dy != 2 || !model->consts || model->n_consts != 2)
        return AIRPF_E_INVALID_ARG;
      const double al = model->consts[0], be = model->consts[1];
      if (!all_finite(theta, 1) || !all_finite(model->consts, 2)) return AIRPF_E_INVALID_ARG;
      if (!(al >= 1.0 && be >= 1.0 && al == std::floor(al) && be == std::floor(be) && al + be <= 7.0))
        return AIRPF_E_INVALID_ARG;
      if (!(theta[0] >= 0.0 && theta[0] <= 1.0)) return AIRPF_E_DOMAIN;
      mp->ab[0] = static_cast<int>(al);
      mp->ab[1] = static_cast<int>(be);
      dx = dy = 2;
      break;
    }
    default:
      return AIRPF_E_INVALID_ARG;
  }
  for (int i = 0; i < d_theta; ++i) mp->th[i] = theta[i];
  // binary32 particles: every parameter and derived constant rounded once
  for (int i = 0; i < d_theta; ++i) mp->thf[i] = static_cast<float>(theta[i]);
  for (int i = 0; i < airpf::kMaxDy * 8; ++i) mp->Hf[i] = static_cast<float>(mp->H[i]);
  mp->s0f = static_cast<float>(mp->s0);
  mp->sqf = static_cast<float>(mp->sq);
  mp->sp0f = static_cast<float>(mp->sp0);
  mp->hrf = static_cast<float>(mp->hr);
  mp->isyf = model->kind == AIRPF_LG1 ? static_cast<float>(1.0 / theta[2]) : 0.0f;
  mp->dy = dy;
  *cst_q = c_log - 40.0 * std::log(2.0) - std::log(static_cast<double>(N));
  *dx_out = dx;
  *dy_out = dy;
  return AIRPF_OK;
}

// AIRPF_TUNE_CACHE=<file>: the tiler's measured choices persist across
// processes in that text file, one line "<batch-shape key, hex> <ratio>
// <particles per lane>" per shape (0, or a line without the third field:
// the default rule); it is read when the context's own cache misses and
// appended after a measurement (an unreadable or absent file is a miss).
bool tune_cache_lookup(uint64_t key, double* ratio, int* ppt) {
  const char* path = std::getenv("AIRPF_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[160];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    unsigned long long k = 0;
    double r = 0.0;
    int p = 0;
    const int got = std::sscanf(line, "%llx %lf %d", &k, &r, &p);
    if (got < 2 || k != key || !(r > 0.0) || !std::isfinite(r)) continue;
    if (got < 3 || (p != 4 && p != 8)) p = 0;
    *ratio = r;                                        // the last line of a key wins
    *ppt = p;
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(uint64_t key, double ratio, int ppt) {
  const char* path = std::getenv("AIRPF_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%016llx %.17g %d\n", static_cast<unsigned long long>(key), ratio, ppt);
    std::fclose(f);
  }
}

// A tracer range (roctx) around one call of the ABI, shown by profilers that
// trace markers (rocprofv3 --marker-trace); a no-op otherwise.
struct Range {
  explicit Range(const char* name) { roctxRangePush(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

airpf_options default_options() {
  airpf_options o;
  o.tau = 0.3;
  o.resampling = AIRPF_SYSTEMATIC;
  o.precision = AIRPF_FP32;
  o.score_mode = AIRPF_PATHSPACE;
  o.ckpt_every = 0;
  o.flags = 0;
  o.resample_ess = 0.0;
  o.arity = 2;
  return o;
}

void set_nan(double* p) { if (p) *p = std::nan(""); }

}  // namespace

namespace {

// Everything airpf_run and airpf_score share: validation, model constants,
// the launch plan and the forward kernel's workspaces.
struct Prepared {
  airpf::FwdArgs a;
  airpf::FwdLaunch L;
  airpf::FwdPlan plan;
  airpf_options opt;
  int dx = 1, dy = 1, S = 0;
  // bound of the block count of any launch of this problem (the kernel
  // variant a launch takes, and so its G, may differ from the plan's)
  int gmax = 1;
};

// fixed != nullptr: every workspace is carved from that device array of
// kNoallocScratchBytes (airpf_run_noalloc) instead of the context's buffers.
airpf_status prepare(airpf_ctx* ctx, const airpf_model* model, const double* theta, int32_t d_theta,
                     const double* y, int64_t T, int32_t m, int32_t N, uint64_t seed,
                     const airpf_options* opt_in, double* log_z_out, int max_blocks, Prepared* P,
                     unsigned char* fixed = nullptr) {
  set_nan(log_z_out);
  if (!ctx || !model || (!theta && d_theta != 0) || !y || !log_z_out) return AIRPF_E_INVALID_ARG;
  if (T < 1 || T > (int64_t(1) << 30) || !is_pow2(m) || N < 1 || N > 2048) return AIRPF_E_INVALID_ARG;
  if (m > kMaxIslands) return AIRPF_E_UNSUPPORTED;
  P->opt = opt_in ? *opt_in : default_options();
  if ((model->kind == AIRPF_BIN || model->kind == AIRPF_BCP) && P->opt.precision == AIRPF_FP32)
    P->opt.precision = AIRPF_FP64;                  // word-driven models keep their states in double
  const airpf_options& opt = P->opt;
  if (!(opt.tau == opt.tau)) return AIRPF_E_INVALID_ARG;
  if (opt.precision != AIRPF_FP32 && opt.precision != AIRPF_FP64) return AIRPF_E_INVALID_ARG;
  if (opt.resampling != AIRPF_SYSTEMATIC && opt.resampling != AIRPF_MULTINOMIAL) return AIRPF_E_INVALID_ARG;
  if (!(opt.resample_ess >= 0.0) || !std::isfinite(opt.resample_ess)) return AIRPF_E_INVALID_ARG;
  const bool adapt = opt.resample_ess > 0.0;
  // adaptive internal resampling: systematic when an island resamples, states
  // in double, every workspace from the context
  if (adapt && (opt.resampling != AIRPF_SYSTEMATIC || fixed)) return AIRPF_E_UNSUPPORTED;
  if (adapt) P->opt.precision = AIRPF_FP64;
  // r-ary interactions: r a power of two and m a power of r
  const int32_t arity = opt.arity == 0 ? 2 : opt.arity;
  if (arity < 2 || !is_pow2(arity) || ilog2(m) % ilog2(arity) != 0) return AIRPF_E_INVALID_ARG;

  airpf::FwdArgs& a = P->a;
  std::memset(&a, 0, sizeof(a));
  a.arity_log2 = ilog2(arity);
  a.multinomial = opt.resampling == AIRPF_MULTINOMIAL ? 1 : 0;
  const airpf_status st = prepare_model(model, theta, d_theta, N, &a.mp, &a.cst_q, &P->dx, &P->dy);
  if (st == AIRPF_E_DOMAIN) { *log_z_out = -INFINITY; return st; }
  if (st != AIRPF_OK) return st;
  const bool y_dev = (opt.flags & AIRPF_FLAG_Y_ON_DEVICE) != 0;
  if (!y_dev && !all_finite(y, T * P->dy)) return AIRPF_E_INVALID_ARG;

  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  P->S = ilog2(m);
  a.T = T; a.m = m; a.N = N; a.S = P->S; a.dy = P->dy; a.seed = seed; a.tau = opt.tau;
  a.n0 = 0; a.n1 = T;
  a.shortcut_all = opt.tau > 1.0 + 1e-9;
  a.no_interaction = opt.tau <= 0.5 / m;

  // AIRPF_MAX_BLOCKS caps the blocks of a launch (tiling tests); results do
  // not depend on it
  if (const char* env = std::getenv("AIRPF_MAX_BLOCKS")) {
    const int cap = std::atoi(env);
    if (cap >= 1 && cap < max_blocks) max_blocks = cap;
  }
  airpf::FwdLaunch& L = P->L;
  L.kind = model->kind; L.dx = P->dx; L.fp64 = opt.precision == AIRPF_FP64;
  L.num_cus = ctx->num_cus; L.max_blocks = max_blocks; L.plan_only = 1; L.stream = s;
  {
    const hipError_t e = airpf::launch_forward(L, a, &P->plan);
    if (e == hipErrorInvalidValue) return AIRPF_E_UNSUPPORTED;   // no tiling fits the LDS plan
    if (e != hipSuccess) return AIRPF_E_DEVICE;
  }

  const size_t store = L.fp64 ? 8 : 4;
  const size_t nstate = size_t(m) * N * P->dx * store;
  P->gmax = std::min(max_blocks, m);
  // ENF records: (log2(m/G) + 1) levels of G blocks, largest at G = gmax
  const size_t part_words = 3 * size_t(ilog2(m / P->gmax) + 1) * size_t(P->gmax);
  // misc: [0,8) log Zhat, [8,12) status, [64, 64 + 4G) barrier flags, then
  // the level-1 record ring of the pipelined kernel (kRingCopies copies of
  // 9G doubles, G <= 256)
  const size_t ring_off = (64 + 4 * size_t(P->gmax) + 255) & ~size_t(255);
  const int gring = std::min(P->gmax, 256);
  const size_t misc_bytes = ring_off + 8 * 3 * airpf::kRingSlots * size_t(gring) * airpf::kRingCopies;
  const size_t y_bytes = sizeof(double) * size_t(T) * P->dy;
  unsigned char* misc = nullptr;
  void* ybuf = nullptr;
  if (fixed) {
    // one 256-byte aligned piece after another; nothing is allocated
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = (off + 255) & ~size_t(255); off = o + bytes; return fixed + o; };
    for (int p = 0; p < 2; ++p) {
      a.x1[p] = take(nstate);
      a.tree[p] = reinterpret_cast<double*>(take(sizeof(double) * 2 * size_t(m)));
      a.part[p] = reinterpret_cast<double*>(take(sizeof(double) * part_words));
    }
    misc = take(misc_bytes);
    if (!y_dev) ybuf = take(y_bytes);
    if (off > kNoallocScratchBytes) return AIRPF_E_TOO_LARGE;
  } else {
    for (int p = 0; p < 2; ++p) {
      ST_OK(ctx->x1[p].ensure(nstate));
      ST_OK(ctx->tree[p].ensure(sizeof(double) * 2 * size_t(m)));
      ST_OK(ctx->part[p].ensure(sizeof(double) * part_words));
      a.x1[p] = ctx->x1[p].p;
      a.tree[p] = static_cast<double*>(ctx->tree[p].p);
      a.part[p] = static_cast<double*>(ctx->part[p].p);
    }
    ST_OK(ctx->misc.ensure(misc_bytes));
    misc = static_cast<unsigned char*>(ctx->misc.p);
    if (adapt) {
      for (int p = 0; p < 2; ++p) {
        ST_OK(ctx->ad_lc[p].ensure(sizeof(double) * size_t(m) * N));
        ST_OK(ctx->ad_dq[p].ensure(sizeof(double) * size_t(m)));
        a.lc1[p] = static_cast<double*>(ctx->ad_lc[p].p);
        a.dq1[p] = static_cast<double*>(ctx->ad_dq[p].p);
      }
      a.ess_frac = opt.resample_ess;
      a.log_N = std::log(static_cast<double>(N));
    }
    if (!y_dev) {
      ST_OK(ctx->ybuf.ensure(y_bytes));
      ybuf = ctx->ybuf.p;
    }
  }
  a.out_logz = reinterpret_cast<double*>(misc);
  a.status = reinterpret_cast<int*>(misc + 8);
  a.bad_y = reinterpret_cast<int*>(misc + 12);
  a.check_y = y_dev ? 1 : 0;
  a.bar = reinterpret_cast<unsigned*>(misc + 64);
  a.ring = reinterpret_cast<double*>(misc + ring_off);
  if (y_dev) {
    a.y = y;
  } else {
    HIP_OK(hipMemcpyAsync(ybuf, y, y_bytes, hipMemcpyHostToDevice, s));
    a.y = static_cast<const double*>(ybuf);
  }
  HIP_OK(airpf::fill_u32(misc, 0u, 16 + int64_t(P->gmax), s));
  HIP_OK(airpf::fill_u32(misc + ring_off, 0xFFFFFFFFu, 2 * 3 * airpf::kRingSlots * int64_t(gring) * airpf::kRingCopies,
                         s));   // NaN
  return AIRPF_OK;
}

// zero the barrier flags before a cooperative launch
airpf_status reset_flags(airpf_ctx* ctx, const Prepared& P) {
  HIP_OK(airpf::fill_u32(P.a.bar, 0u, P.gmax, ctx->stream));
  return AIRPF_OK;
}

airpf_status attach_trace(airpf_ctx* ctx, Prepared& P, airpf_trace* trace) {
  airpf::FwdArgs& a = P.a;
  if (!trace) return AIRPF_OK;
  const int64_t T = a.T;
  const int m = a.m, N = a.N, S = P.S;
  hipStream_t s = ctx->stream;
  if (trace->enf) a.shortcut_all = 0;
  if (trace->sstar) { ST_OK(ctx->t_sstar.ensure(4 * size_t(T))); a.tr_sstar = static_cast<int32_t*>(ctx->t_sstar.p);
                      HIP_OK(airpf::fill_u32(a.tr_sstar, 0u, T, s)); }
  if (trace->enf) { ST_OK(ctx->t_enf.ensure(8 * size_t(T) * (S + 1))); a.tr_enf = static_cast<double*>(ctx->t_enf.p);
                    HIP_OK(airpf::fill_u32(a.tr_enf, 0x7ff80000u, 2 * int64_t(T) * (S + 1), s)); }
  if (trace->lpost) { ST_OK(ctx->t_lpost.ensure(8 * size_t(T) * m)); a.tr_lpost = static_cast<double*>(ctx->t_lpost.p); }
  if (trace->anc && T > 1) { ST_OK(ctx->t_anc.ensure(4 * size_t(T - 1) * m * N)); a.tr_anc = static_cast<int32_t*>(ctx->t_anc.p); }
  if (trace->pi && T > 1) { ST_OK(ctx->t_pi.ensure(4 * size_t(T - 1) * m)); a.tr_pi = static_cast<int32_t*>(ctx->t_pi.p); }
  if (trace->digest) { ST_OK(ctx->t_dig.ensure(16 * size_t(T))); a.tr_digest = static_cast<unsigned long long*>(ctx->t_dig.p);
                       HIP_OK(airpf::fill_u32(a.tr_digest, 0u, 4 * int64_t(T), s)); }
  if (trace->fmean) { ST_OK(ctx->t_fmean.ensure(8 * size_t(T) * m)); a.tr_fmean = static_cast<double*>(ctx->t_fmean.p); }
  return AIRPF_OK;
}

airpf_status copy_trace(airpf_ctx* ctx, const Prepared& P, airpf_trace* trace) {
  if (!trace) return AIRPF_OK;
  const airpf::FwdArgs& a = P.a;
  const int64_t T = a.T;
  const int m = a.m, N = a.N, S = P.S;
  hipStream_t s = ctx->stream;
  if (trace->sstar && a.tr_sstar) HIP_OK(hipMemcpyAsync(trace->sstar, a.tr_sstar, 4 * size_t(T), hipMemcpyDeviceToHost, s));
  if (trace->enf && a.tr_enf) HIP_OK(hipMemcpyAsync(trace->enf, a.tr_enf, 8 * size_t(T) * (S + 1), hipMemcpyDeviceToHost, s));
  if (trace->lpost && a.tr_lpost) HIP_OK(hipMemcpyAsync(trace->lpost, a.tr_lpost, 8 * size_t(T) * m, hipMemcpyDeviceToHost, s));
  if (trace->anc && a.tr_anc) HIP_OK(hipMemcpyAsync(trace->anc, a.tr_anc, 4 * size_t(T - 1) * m * N, hipMemcpyDeviceToHost, s));
  if (trace->pi && a.tr_pi) HIP_OK(hipMemcpyAsync(trace->pi, a.tr_pi, 4 * size_t(T - 1) * m, hipMemcpyDeviceToHost, s));
  if (trace->digest && a.tr_digest) HIP_OK(hipMemcpyAsync(trace->digest, a.tr_digest, 16 * size_t(T), hipMemcpyDeviceToHost, s));
  if (trace->fmean && a.tr_fmean) HIP_OK(hipMemcpyAsync(trace->fmean, a.tr_fmean, 8 * size_t(T) * m, hipMemcpyDeviceToHost, s));
  return AIRPF_OK;
}

airpf_status finish(airpf_ctx* ctx, const Prepared& P, double* log_z_out) {
  double lz = 0.0;
  int kstatus[2] = {0, 0};                     // the status word and the bad-observation flag
  hipStream_t s = ctx->stream;
  HIP_OK(hipMemcpyAsync(&lz, P.a.out_logz, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(kstatus, P.a.status, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (kstatus[1] != 0) return AIRPF_E_INVALID_ARG;     // a device-resident observation was not finite
  if (kstatus[0] != 0) return AIRPF_E_DEVICE;
  float ms = 0.0f;
  HIP_OK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  ctx->last_kernel_ms = ms;
  *log_z_out = lz;
  return AIRPF_OK;
}

}  // namespace

extern "C" airpf_status airpf_run(airpf_ctx* ctx, const airpf_model* model, const double* theta, int32_t d_theta,
                                  const double* y, int64_t T, int32_t m, int32_t N, uint64_t seed,
                                  const airpf_options* opt_in, double* log_z_out, airpf_trace* trace) {
  const Range range("airpf_run");
  Prepared P;
  ST_OK(prepare(ctx, model, theta, d_theta, y, T, m, N, seed, opt_in, log_z_out, kMaxBlocks, &P));
  ST_OK(attach_trace(ctx, P, trace));
  P.L.plan_only = 0;
  HIP_OK(hipEventRecord(ctx->ev[0], ctx->stream));
  if (airpf::launch_forward(P.L, P.a, &P.plan) != hipSuccess) return AIRPF_E_DEVICE;
  HIP_OK(hipEventRecord(ctx->ev[1], ctx->stream));
  ST_OK(copy_trace(ctx, P, trace));
  return finish(ctx, P, log_z_out);
}

// airpf_run with every workspace in the device's fixed scratch array: no
// hipMalloc, hipFree or allocating library call.  Calls that overlap on one
// device share (and race on) that array.
extern "C" airpf_status airpf_run_noalloc(airpf_ctx* ctx, const airpf_model* model, const double* theta,
                                          int32_t d_theta, const double* y, int64_t T, int32_t m, int32_t N,
                                          uint64_t seed, const airpf_options* opt_in, double* log_z_out) {
  if (!ctx) { set_nan(log_z_out); return AIRPF_E_INVALID_ARG; }
  Prepared P;
  ST_OK(prepare(ctx, model, theta, d_theta, y, T, m, N, seed, opt_in, log_z_out, kMaxBlocks, &P, ctx->scratch));
  P.L.plan_only = 0;
  HIP_OK(hipEventRecord(ctx->ev[0], ctx->stream));
  if (airpf::launch_forward(P.L, P.a, &P.plan) != hipSuccess) return AIRPF_E_DEVICE;
  HIP_OK(hipEventRecord(ctx->ev[1], ctx->stream));
  return finish(ctx, P, log_z_out);
}

extern "C" airpf_status airpf_score(airpf_ctx* ctx, const airpf_model* model, const double* theta,
                                    int32_t d_theta, const double* y, int64_t T, int32_t m, int32_t N,
                                    uint64_t seed, const airpf_options* opt_in, double* log_z_out,
                                    double* grad_out, airpf_trace* trace) {
  const Range range("airpf_score");
  if (grad_out) for (int i = 0; i < d_theta; ++i) grad_out[i] = std::nan("");
  if (!grad_out) { set_nan(log_z_out); return AIRPF_E_INVALID_ARG; }
  const airpf_options opt = opt_in ? *opt_in : default_options();
  if ((opt.score_mode != AIRPF_PATHSPACE && opt.score_mode != AIRPF_PATHWISE) || opt.ckpt_every < 0) {
    set_nan(log_z_out);
    return AIRPF_E_INVALID_ARG;
  }
  // (multinomial internal resampling: the reverse pass sorts each step's
  // slots by ancestor)
  // adaptive internal resampling: forward only
  if (opt.resample_ess != 0.0 || (opt.arity != 0 && opt.arity != 2)) { set_nan(log_z_out); return AIRPF_E_UNSUPPORTED; }
  // the word-driven models' mutations are not differentiable in theta
  if (model && (model->kind == AIRPF_BIN || model->kind == AIRPF_BCP)) { set_nan(log_z_out); return AIRPF_E_UNSUPPORTED; }
  if (model && ((model->kind == AIRPF_LGD && N > 512) || (model->kind != AIRPF_LGD && N > 1024))) {
    set_nan(log_z_out);
    return AIRPF_E_UNSUPPORTED;
  }
  if (ctx) HIP_OK(hipSetDevice(ctx->device));

  // the reverse kernel's co-residency bounds the plan of both launches
  airpf::BwdArgs b;
  std::memset(&b, 0, sizeof(b));
  b.N = N;
  int bwd_max = 0;
  if (model && ctx) {
    airpf::FwdLaunch Lq;
    Lq.kind = model->kind; Lq.dx = model->kind == AIRPF_LGD ? model->dx : 1;
    Lq.fp64 = opt.precision == AIRPF_FP64; Lq.num_cus = ctx->num_cus; Lq.max_blocks = 1024; Lq.plan_only = 1;
    Lq.stream = ctx->stream;
    if (airpf::launch_backward(Lq, b, &bwd_max) != hipSuccess || bwd_max < 1) {
      set_nan(log_z_out);
      return (model->kind == AIRPF_LGD && !(Lq.dx == 2 || Lq.dx == 3 || Lq.dx == 4 || Lq.dx == 8)) ? AIRPF_E_INVALID_ARG
                                                                                                 : AIRPF_E_DEVICE;
    }
  }
  Prepared P;
  ST_OK(prepare(ctx, model, theta, d_theta, y, T, m, N, seed, opt_in, log_z_out, bwd_max < kMaxBlocks ? bwd_max : kMaxBlocks, &P));
  ST_OK(attach_trace(ctx, P, trace));
  airpf::FwdArgs& a = P.a;
  hipStream_t s = ctx->stream;
  const int dx = P.dx;
  const size_t store = P.L.fp64 ? 8 : 4;
  const size_t per_step = size_t(m) * N * (dx * store + 2);

  // checkpoint interval
  int64_t K = opt.ckpt_every;
  if (K == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = size_t(8) << 30;
    const size_t budget = free_b / 3;
    if (per_step * size_t(T) <= budget) K = T;
    else { K = 1; while (K * K < T) ++K; }
  }
  if (K > T) K = T;
  const int64_t C = (T + K - 1) / K;

  // workspaces of the score
  ST_OK(ctx->s_pi.ensure(4 * size_t(T) * m));
  ST_OK(ctx->s_sstar.ensure(4 * size_t(T)));
  ST_OK(ctx->s_lpre.ensure(8 * size_t(T) * m));
  ST_OK(ctx->s_ckx.ensure(size_t(C) * m * N * dx * store));
  ST_OK(ctx->s_ckL.ensure(8 * size_t(C) * m));
  ST_OK(ctx->s_recx.ensure(size_t(K) * m * N * dx * store));
  ST_OK(ctx->s_reca.ensure(2 * size_t(K) * m * N));
  for (int p = 0; p < 2; ++p) {
    ST_OK(ctx->s_lam[p].ensure(size_t(m) * N * dx * store));
    ST_OK(ctx->s_del[p].ensure(size_t(m) * N * store));
  }
  const int Pn = d_theta;
  ST_OK(ctx->s_grad.ensure(8 * size_t(m) * Pn + 8 * 64));
  ST_OK(ctx->s_nu.ensure(8 * 2 * size_t(m)));

  // forward: keep island maps, stage counts, entering weights, checkpoints;
  // with a single segment the particle history is recorded right away
  int32_t* keep_pi = a.tr_pi;
  a.tr_pi = static_cast<int32_t*>(ctx->s_pi.p);
  int32_t* keep_sstar = a.tr_sstar;
  a.tr_sstar = static_cast<int32_t*>(ctx->s_sstar.p);
  a.tr_lpre = static_cast<double*>(ctx->s_lpre.p);
  a.ck_every = K;
  a.ck_x = ctx->s_ckx.p;
  a.ck_L = static_cast<double*>(ctx->s_ckL.p);
  if (C == 1) {
    a.rec_x = ctx->s_recx.p;
    a.rec_anc = static_cast<uint16_t*>(ctx->s_reca.p);
  }
  P.L.plan_only = 0;
  HIP_OK(hipEventRecord(ctx->ev[0], s));
  if (airpf::launch_forward(P.L, a, &P.plan) != hipSuccess) return AIRPF_E_DEVICE;
  if (keep_pi && T > 1)
    HIP_OK(hipMemcpyAsync(keep_pi, a.tr_pi, 4 * size_t(T - 1) * m, hipMemcpyDeviceToDevice, s));
  if (keep_sstar) HIP_OK(hipMemcpyAsync(keep_sstar, a.tr_sstar, 4 * size_t(T), hipMemcpyDeviceToDevice, s));

  // A run in which every island died stopped at that step, so its records end
  // there: the estimate is zero and its score is taken as zero, with no
  // reverse sweep.  A forward pass that failed skips the sweep too.
  {
    double lz_fwd = 0.0;
    int st_fwd[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(&lz_fwd, a.out_logz, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(st_fwd, a.status, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (st_fwd[0] != 0 || st_fwd[1] != 0 || lz_fwd == -INFINITY) {
      HIP_OK(hipEventRecord(ctx->ev[1], s));
      a.tr_pi = keep_pi;
      a.tr_sstar = keep_sstar;
      ST_OK(copy_trace(ctx, P, trace));
      const airpf_status fs = finish(ctx, P, log_z_out);
      for (int p = 0; p < d_theta; ++p) grad_out[p] = fs == AIRPF_OK ? 0.0 : std::nan("");
      return fs;
    }
  }

  // reverse, one segment at a time, tiled as the serial forward kernel would
  // be (the pipelined forward's tiling stops at 256 blocks; the reverse
  // kernel's own co-residency bounds both): results do not depend on it
  airpf::FwdPlan bplan;
  {
    airpf::FwdLaunch Lp = P.L;
    Lp.plan_only = 1;
    airpf::FwdArgs q = a;
    q.replay_pi = 1;
    if (airpf::launch_forward(Lp, q, &bplan) != hipSuccess) return AIRPF_E_DEVICE;
  }
  b.mp = a.mp; b.y = a.y; b.T = T; b.m = m; b.N = N; b.S = P.S; b.c = bplan.c; b.lc = ilog2(bplan.c);
  b.G = bplan.G; b.dy = P.dy; b.seed = seed;
  b.log_mN = std::log(static_cast<double>(m) * static_cast<double>(N));
  b.c_log = a.cst_q + 40.0 * std::log(2.0) + std::log(static_cast<double>(N));
  b.log_N = std::log(static_cast<double>(N));
  b.pathwise = opt.score_mode == AIRPF_PATHWISE ? 1 : 0;
  b.multinomial = opt.resampling == AIRPF_MULTINOMIAL ? 1 : 0;
  b.nu[0] = static_cast<double*>(ctx->s_nu.p);
  b.nu[1] = b.nu[0] + m;
  b.logz = a.out_logz;
  b.rec_x = ctx->s_recx.p;
  b.rec_anc = static_cast<const uint16_t*>(ctx->s_reca.p);
  b.pi_all = a.tr_pi;
  b.sstar_all = a.tr_sstar;
  b.lpre_all = a.tr_lpre;
  for (int p = 0; p < 2; ++p) { b.lam[p] = ctx->s_lam[p].p; b.del[p] = ctx->s_del[p].p; }
  b.gisl = static_cast<double*>(ctx->s_grad.p);
  double* gsum = b.gisl + size_t(m) * Pn;
  b.bar = a.bar;
  b.status = a.status;
  HIP_OK(airpf::fill_u32(b.gisl, 0u, 2 * int64_t(m) * Pn, s));
  for (int64_t cidx = C - 1; cidx >= 0; --cidx) {
    const int64_t lo = cidx * K, hi = (cidx + 1) * K < T ? (cidx + 1) * K : T;
    if (C > 1) {
      airpf::FwdArgs r = a;
      r.n0 = lo; r.n1 = hi; r.replay_pi = 1; r.ck_in = lo > 0 ? 1 : 0;
      r.sstar_in = static_cast<const int32_t*>(ctx->s_sstar.p);
      r.rec_x = ctx->s_recx.p;
      r.rec_anc = static_cast<uint16_t*>(ctx->s_reca.p);
      r.tr_sstar = nullptr; r.tr_enf = nullptr; r.tr_lpost = nullptr; r.tr_anc = nullptr; r.tr_digest = nullptr;
      r.tr_lpre = nullptr;
      ST_OK(reset_flags(ctx, P));
      if (airpf::launch_forward(P.L, r, &P.plan) != hipSuccess) return AIRPF_E_DEVICE;
    }
    b.n_lo = lo;
    b.n_hi = hi;
    ST_OK(reset_flags(ctx, P));
    if (airpf::launch_backward(P.L, b, nullptr) != hipSuccess) return AIRPF_E_DEVICE;
  }
  HIP_OK(airpf::launch_island_grad_sum(b.gisl, m, Pn, gsum, s));
  HIP_OK(hipEventRecord(ctx->ev[1], s));
  HIP_OK(hipMemcpyAsync(grad_out, gsum, 8 * size_t(Pn), hipMemcpyDeviceToHost, s));
  a.tr_pi = keep_pi;                 // the caller's trace arrays were filled above
  a.tr_sstar = keep_sstar;
  ST_OK(copy_trace(ctx, P, trace));
  const airpf_status fs = finish(ctx, P, log_z_out);
  if (fs != AIRPF_OK) for (int p = 0; p < Pn; ++p) grad_out[p] = std::nan("");
  return fs;
}

extern "C" airpf_status airpf_ctx_last_kernel_ms(airpf_ctx* ctx, double* ms) {
  if (!ctx || !ms) return AIRPF_E_INVALID_ARG;
  *ms = ctx->last_kernel_ms;
  return AIRPF_OK;
}

extern "C" airpf_status airpf_debug_eval(airpf_ctx* ctx, int32_t which, int64_t n, const double* in,
                                         const uint32_t* in_u32, double* out, double* out2, uint32_t* out_u32) {
  if (!ctx || n < 0 || which < 0 || which > 8) return AIRPF_E_INVALID_ARG;
  if (n == 0) return AIRPF_OK;
  // 0-2, 5-7 read doubles; 3, 8 read word pairs; 4 reads Philox blocks
  const bool uses_in = which <= 2 || (which >= 5 && which <= 7), uses_in32 = which == 3 || which == 4 || which == 8;
  const bool uses_out2 = which == 2 || which == 3 || which == 7 || which == 8;
  if ((uses_in && !in) || (uses_in32 && !in_u32) || (which != 4 && !out) || (uses_out2 && !out2) ||
      (which == 4 && !out_u32))
    return AIRPF_E_INVALID_ARG;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const size_t n32 = (which == 3 || which == 8) ? 2 * size_t(n) : 6 * size_t(n);
  ST_OK(ctx->dbg_in.ensure(8 * size_t(n)));
  ST_OK(ctx->dbg_in32.ensure(4 * n32));
  ST_OK(ctx->dbg_out.ensure(8 * size_t(n)));
  ST_OK(ctx->dbg_out2.ensure(8 * size_t(n)));
  ST_OK(ctx->dbg_out32.ensure(16 * size_t(n)));
  if (uses_in) HIP_OK(hipMemcpyAsync(ctx->dbg_in.p, in, 8 * size_t(n), hipMemcpyHostToDevice, s));
  if (uses_in32) HIP_OK(hipMemcpyAsync(ctx->dbg_in32.p, in_u32, 4 * n32, hipMemcpyHostToDevice, s));
  HIP_OK(airpf::launch_debug_eval(which, n, static_cast<const double*>(ctx->dbg_in.p),
                                  static_cast<const uint32_t*>(ctx->dbg_in32.p), static_cast<double*>(ctx->dbg_out.p),
                                  static_cast<double*>(ctx->dbg_out2.p), static_cast<uint32_t*>(ctx->dbg_out32.p), s));
  if (which != 4) HIP_OK(hipMemcpyAsync(out, ctx->dbg_out.p, 8 * size_t(n), hipMemcpyDeviceToHost, s));
  if (uses_out2) HIP_OK(hipMemcpyAsync(out2, ctx->dbg_out2.p, 8 * size_t(n), hipMemcpyDeviceToHost, s));
  if (which == 4) HIP_OK(hipMemcpyAsync(out_u32, ctx->dbg_out32.p, 16 * size_t(n), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return AIRPF_OK;
}

// ======================================================================
// Batched multi-theta calls
// ======================================================================
namespace {

int pow2_ceil_i(int64_t v) { int p = 1; while (p < v) p <<= 1; return p; }

// Bump allocator of one context buffer (256-byte aligned pieces).
struct Arena {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + (bytes ? bytes : 1);
    return o;
  }
};

// One valid problem of a batch and its workspace (offsets into the arena).
struct Item {
  int idx = 0;
  airpf::ModelArgs mp;
  double cst_q = 0.0;
  int64_t T = 0, K = 0, C = 0;
  int m = 0, N = 0, S = 0, TP = 0, tpb = 0, G = 1;
  uint64_t seed = 0;
  const double* y_dev = nullptr;
  size_t o_y = 0, o_x1[2] = {0, 0}, o_tree[2] = {0, 0}, o_part[2] = {0, 0}, o_flags = 0;
  size_t o_pi = 0, o_sstar = 0, o_lpre = 0, o_ckx = 0, o_ckL = 0, o_recx = 0, o_reca = 0;
  size_t o_lam[2] = {0, 0}, o_del[2] = {0, 0}, o_gisl = 0, o_gsum = 0, o_nu = 0;
};

// Tiler.  Modelled time of a problem over `steps` filter steps on G blocks:
// steps * (1 + ratio * passes), passes = ceil(islands per block / islands
// per pass): a step's fixed part (the grid synchronisation and island
// cascade) is the unit and `ratio` prices one pass of island work.  The
// default ratio 1/3 was measured on MI355X (12 us per step, 4 us per pass);
// AIRPF_TILER="alpha,beta" (microseconds) replaces it, and
// AIRPF_FLAG_AUTOTUNE measures it per batch shape (see airpf_run_batch).
// Start from the fewest blocks that keep a block's islands within the LDS
// plan (<= 256) and double the block count of the slowest problem while the
// device's co-residency allows.
bool tile(std::vector<Item*>& its, const std::vector<int64_t>& steps, int capacity, double ratio) {
  auto passes = [](const Item* it, int G) { const int c = it->m / G; return (c + it->tpb - 1) / it->tpb; };
  auto cost = [&](size_t i, int G) { return double(steps[i]) * (1.0 + ratio * passes(its[i], G)); };
  int used = 0;
  for (Item* it : its) {
    int g = pow2_ceil_i((it->m + 255) / 256);
    if (g > it->m) g = it->m;
    it->G = g;
    used += g;
  }
  if (used > capacity) return false;
  for (;;) {
    int best = -1;
    double worst = -1.0;
    for (size_t i = 0; i < its.size(); ++i) {
      Item* it = its[i];
      const int G2 = it->G * 2;
      if (G2 > it->m || G2 > 256 || passes(it, it->G) <= 1 || used + it->G > capacity) continue;
      const double c0 = cost(i, it->G);
      if (c0 > worst) { worst = c0; best = int(i); }
    }
    if (best < 0) break;
    // only grow the problem that bounds the batch; stop when it cannot grow
    double top = -1.0;
    for (size_t i = 0; i < its.size(); ++i) top = std::max(top, cost(i, its[i]->G));
    if (worst < top) break;
    used += its[best]->G;
    its[best]->G *= 2;
  }
  return true;
}

}  // namespace

extern "C" airpf_status airpf_run_batch(airpf_ctx* ctx, const airpf_model* model, int32_t B,
                                        const airpf_problem* probs, const airpf_options* opt_in,
                                        int32_t want_score, double* log_z_out, double* grad_out,
                                        airpf_status* item_status) {
  const Range range("airpf_run_batch");
  if (!ctx || !model || B < 0 || (B > 0 && (!probs || !log_z_out || !item_status))) return AIRPF_E_INVALID_ARG;
  if (model->kind == AIRPF_BIN || model->kind == AIRPF_BCP) return AIRPF_E_UNSUPPORTED;   // single problems only
  const airpf_options opt = opt_in ? *opt_in : default_options();
  // adaptive internal resampling and r-ary interactions: single problems
  if (opt.resample_ess != 0.0 || (opt.arity != 0 && opt.arity != 2)) return AIRPF_E_UNSUPPORTED;
  if (want_score && !grad_out) return AIRPF_E_INVALID_ARG;
  if (!(opt.tau == opt.tau) || (opt.precision != AIRPF_FP32 && opt.precision != AIRPF_FP64) || opt.ckpt_every < 0)
    return AIRPF_E_INVALID_ARG;
  if (opt.resampling != AIRPF_SYSTEMATIC && opt.resampling != AIRPF_MULTINOMIAL) return AIRPF_E_INVALID_ARG;
  // multinomial draws: forward only (the reverse pass needs sorted ancestors)
  const int mult = opt.resampling == AIRPF_MULTINOMIAL ? 1 : 0;
  if (want_score && opt.score_mode != AIRPF_PATHSPACE && opt.score_mode != AIRPF_PATHWISE) return AIRPF_E_INVALID_ARG;
  const bool y_dev = (opt.flags & AIRPF_FLAG_Y_ON_DEVICE) != 0;
  const bool fp64 = opt.precision == AIRPF_FP64;
  const size_t store = fp64 ? 8 : 4;

  // ---- validation, model constants ----
  std::vector<Item> items;
  items.reserve(B);
  int dx = 1, dy = 1, n_max = 1;
  // parameters per problem, fixed by the model: the packing of grad_out
  const int Pn = model->kind == AIRPF_LGD ? model->dx * model->dx : 3;
  if (Pn < 1 || Pn > airpf::kMaxTheta) return AIRPF_E_INVALID_ARG;
  for (int32_t i = 0; i < B; ++i) {
    const airpf_problem& pr = probs[i];
    log_z_out[i] = std::nan("");
    if (want_score) for (int q = 0; q < Pn; ++q) grad_out[size_t(i) * Pn + q] = std::nan("");
    Item it;
    airpf_status st = AIRPF_OK;
    if (!pr.theta || !pr.y || pr.T < 1 || pr.T > (int64_t(1) << 30) || !is_pow2(pr.m) || pr.N < 1 || pr.N > 2048)
      st = AIRPF_E_INVALID_ARG;
    else if (pr.m > kMaxIslands)
      st = AIRPF_E_UNSUPPORTED;
    if (st == AIRPF_OK) st = prepare_model(model, pr.theta, pr.d_theta, pr.N, &it.mp, &it.cst_q, &dx, &dy);
    if (st == AIRPF_OK && pr.d_theta != Pn) st = AIRPF_E_INVALID_ARG;
    if (st == AIRPF_OK && !y_dev && !all_finite(pr.y, pr.T * dy)) st = AIRPF_E_INVALID_ARG;
    if (st == AIRPF_OK && want_score && airpf::backward_ppt(model->kind, dx, pr.N) == 0) st = AIRPF_E_UNSUPPORTED;
    item_status[i] = st;
    if (st == AIRPF_E_DOMAIN) log_z_out[i] = -INFINITY;
    if (st != AIRPF_OK) continue;
    it.idx = i; it.T = pr.T; it.m = pr.m; it.N = pr.N; it.S = ilog2(pr.m); it.seed = pr.seed;
    it.y_dev = y_dev ? pr.y : nullptr;
    if (pr.N > n_max) n_max = pr.N;
    items.push_back(it);
  }
  if (items.empty()) return AIRPF_OK;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;

  const int ppt_rule = airpf::forward_ppt(model->kind, dx, n_max, !want_score);
  int ppt_f = ppt_rule;
  const int ppt_b = want_score ? airpf::backward_ppt(model->kind, dx, n_max) : 0;
  airpf::BatchLaunch BL;
  BL.kind = model->kind; BL.dx = dx; BL.fp64 = fp64; BL.n_max = n_max; BL.num_cus = ctx->num_cus;
  BL.plain = want_score ? 0 : 1;          // the score's forward launches record and replay
  BL.multinomial = mult;
  BL.stream = s; BL.blocks = 0; BL.probs = nullptr; BL.bmap = nullptr;
  int cap_f = 0, cap_fp = 0;
  // particles per lane of the forward launches: the items' teams, the LDS
  // bound of any tiling and the co-resident block counts follow from it
  auto set_ppt = [&](int p) -> airpf_status {
    ppt_f = p;
    for (Item& it : items) {
      it.TP = pow2_ceil_i((it.N + p - 1) / p);
      it.tpb = 256 / it.TP;
    }
    BL.ppt = p;
    BL.smem = airpf::forward_smem(fp64, p, dx, 256, 256, airpf::kResidentBudget, mult);   // bound of any tiling below
    HIP_OK(airpf::forward_batch_capacity(BL, &cap_f));
    airpf::BatchLaunch BP = BL;
    BP.plain = 1;
    HIP_OK(airpf::forward_batch_capacity(BP, &cap_fp));
    return AIRPF_OK;
  };
  // the autotuner's choices of particles per lane: a forward-only
  // systematic batch of a one-dimensional model whose islands fit four per
  // lane (at most 1024 particles) may take four or eight (results do not
  // depend on it); otherwise the rule's
  std::vector<int> ppt_cand{ppt_rule};
  if ((opt.flags & AIRPF_FLAG_AUTOTUNE) && !std::getenv("AIRPF_TILER") && !want_score && !mult &&
      model->kind != AIRPF_LGD && n_max <= 1024)
    ppt_cand = {4, 8};
  int cap_f_max = 0;
  for (int p : ppt_cand) {
    ST_OK(set_ppt(p));
    cap_f_max = std::max(cap_f_max, cap_f);
  }
  ST_OK(set_ppt(ppt_rule));
  int cap_b = 0;
  if (want_score) {
    airpf::BatchLaunch BB = BL;
    BB.smem = airpf::backward_smem(fp64, ppt_b, dx);
    HIP_OK(airpf::backward_batch_capacity(BB, &cap_b));
  }

  // ---- checkpoint intervals ----
  if (want_score) {
    size_t need = 0;
    for (const Item& it : items) need += size_t(it.T) * it.m * it.N * (dx * store + 2);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = size_t(8) << 30;
    for (Item& it : items) {
      int64_t K = opt.ckpt_every;
      if (K == 0) {
        if (need <= free_b / 3) K = it.T;
        else { K = 1; while (K * K < it.T) ++K; }
      }
      if (K > it.T) K = it.T;
      it.K = K;
      it.C = (it.T + K - 1) / K;
    }
  }

  // ---- workspace: one arena ----
  Arena ar;
  const size_t o_logz = ar.take(8 * items.size());
  const size_t o_status = ar.take(64);
  const size_t o_bad = ar.take(4 * items.size());        // per problem: a device-resident observation not finite
  const size_t o_args = ar.take(sizeof(airpf::FwdArgs) * items.size() + sizeof(airpf::BwdArgs) * items.size());
  size_t o_bmap = 0;
  {
    int64_t blocks_max = 0;
    for (const Item& it : items) blocks_max += it.m;
    o_bmap = ar.take(sizeof(int2) * size_t(std::min<int64_t>(blocks_max, int64_t(cap_f_max > cap_b ? cap_f_max : cap_b) + 1)));
  }
  for (Item& it : items) {
    const size_t mN = size_t(it.m) * it.N;
    if (!y_dev) it.o_y = ar.take(8 * size_t(it.T) * dy);
    for (int p = 0; p < 2; ++p) {
      it.o_x1[p] = ar.take(mN * dx * store);
      it.o_tree[p] = ar.take(8 * 2 * size_t(it.m));
      it.o_part[p] = ar.take(8 * 3 * size_t(it.S + 1) * size_t(std::min(it.m, 256)));
    }
    it.o_flags = ar.take(4 * size_t(std::min(it.m, 256)));
    if (want_score) {
      it.o_pi = ar.take(4 * size_t(it.T) * it.m);
      it.o_sstar = ar.take(4 * size_t(it.T));
      it.o_lpre = ar.take(8 * size_t(it.T) * it.m);
      it.o_ckx = ar.take(size_t(it.C) * mN * dx * store);
      it.o_ckL = ar.take(8 * size_t(it.C) * it.m);
      it.o_recx = ar.take(size_t(it.K) * mN * dx * store);
      it.o_reca = ar.take(2 * size_t(it.K) * mN);
      for (int p = 0; p < 2; ++p) {
        it.o_lam[p] = ar.take(mN * dx * store);
        it.o_del[p] = ar.take(mN * store);
      }
      it.o_gisl = ar.take(8 * size_t(it.m) * Pn);
      it.o_nu = ar.take(8 * 2 * size_t(it.m));
      it.o_gsum = ar.take(8 * size_t(Pn));
    }
  }
  ST_OK(ctx->batch.ensure(ar.off));
  unsigned char* base = static_cast<unsigned char*>(ctx->batch.p);
  auto at = [&](size_t o) { return static_cast<void*>(base + o); };
  int* d_status = static_cast<int*>(at(o_status));
  HIP_OK(airpf::fill_u32(d_status, 0u, 16, s));
  int* d_bad = static_cast<int*>(at(o_bad));
  HIP_OK(airpf::fill_u32(d_bad, 0u, int64_t(items.size()), s));
  for (Item& it : items)
    if (!y_dev)
      HIP_OK(hipMemcpyAsync(at(it.o_y), probs[it.idx].y, 8 * size_t(it.T) * dy, hipMemcpyHostToDevice, s));

  std::vector<airpf::FwdArgs> fa;
  std::vector<airpf::BwdArgs> ba;
  std::vector<int2> bmap;
  // launch helper: tile the given items, upload arguments and block map, zero
  // their barrier flags, launch forward (mode 0) or reverse (mode 1)
  double ratio = 1.0 / 3.0;
  if (const char* env = std::getenv("AIRPF_TILER")) {
    double ea = 0, eb = 0;
    if (std::sscanf(env, "%lf,%lf", &ea, &eb) == 2 && ea > 0 && eb > 0) ratio = eb / ea;
  }
  auto launch = [&](std::vector<Item*>& act, const std::vector<int64_t>& steps, int mode,
                    const std::function<void(Item&, airpf::FwdArgs&)>& fwd_fill,
                    const std::function<void(Item&, airpf::BwdArgs&)>& bwd_fill, bool probe = false) -> airpf_status {
    if (act.empty()) return AIRPF_OK;
    if (!tile(act, steps, mode == 0 ? (probe ? cap_fp : cap_f) : cap_b, ratio)) return AIRPF_E_UNSUPPORTED;
    bmap.clear();
    fa.clear();
    ba.clear();
    int c_max = 1, G_max = 1;
    size_t res_max = 0;
    for (size_t i = 0; i < act.size(); ++i) {
      Item& it = *act[i];
      for (int b = 0; b < it.G; ++b) bmap.push_back(make_int2(int(i), b));
      c_max = std::max(c_max, it.m / it.G);
      G_max = std::max(G_max, it.G);
      HIP_OK(airpf::fill_u32(at(it.o_flags), 0u, it.G, s));
      if (mode == 0) {
        airpf::FwdArgs a;
        std::memset(&a, 0, sizeof(a));
        a.mp = it.mp; a.y = y_dev ? it.y_dev : static_cast<const double*>(at(it.o_y));
        a.T = it.T; a.m = it.m; a.N = it.N; a.S = it.S; a.TP = it.TP; a.G = it.G; a.c = it.m / it.G;
        a.lc = ilog2(a.c); a.dy = dy; a.seed = it.seed; a.tau = opt.tau; a.cst_q = it.cst_q;
        a.shortcut_all = opt.tau > 1.0 + 1e-9;
        a.no_interaction = opt.tau <= 0.5 / it.m;
        a.multinomial = mult;
        const size_t res = airpf::forward_resident_bytes(fp64, dx, a.c, it.N);
        a.res_lds = res > 0;
        res_max = std::max(res_max, res);
        for (int p = 0; p < 2; ++p) {
          a.x1[p] = at(it.o_x1[p]);
          a.tree[p] = static_cast<double*>(at(it.o_tree[p]));
          a.part[p] = static_cast<double*>(at(it.o_part[p]));
        }
        a.bar = static_cast<unsigned*>(at(it.o_flags));
        a.status = d_status;
        a.bad_y = d_bad + (&it - items.data());
        a.check_y = y_dev ? 1 : 0;
        a.out_logz = static_cast<double*>(at(o_logz)) + (&it - items.data());
        a.n0 = 0; a.n1 = it.T;
        fwd_fill(it, a);
        fa.push_back(a);
      } else {
        airpf::BwdArgs b;
        std::memset(&b, 0, sizeof(b));
        b.mp = it.mp; b.y = y_dev ? it.y_dev : static_cast<const double*>(at(it.o_y));
        b.T = it.T; b.m = it.m; b.N = it.N; b.S = it.S; b.G = it.G; b.c = it.m / it.G; b.lc = ilog2(b.c);
        b.TP = pow2_ceil_i((it.N + ppt_b - 1) / ppt_b);
        b.dy = dy; b.seed = it.seed;
        b.log_mN = std::log(static_cast<double>(it.m) * static_cast<double>(it.N));
        b.c_log = it.cst_q + 40.0 * std::log(2.0) + std::log(static_cast<double>(it.N));
        b.log_N = std::log(static_cast<double>(it.N));
        b.pathwise = opt.score_mode == AIRPF_PATHWISE ? 1 : 0;
        b.multinomial = mult;
        b.nu[0] = static_cast<double*>(at(it.o_nu));
        b.nu[1] = b.nu[0] + it.m;
        b.logz = static_cast<const double*>(at(o_logz)) + (&it - items.data());
        b.rec_x = at(it.o_recx);
        b.rec_anc = static_cast<const uint16_t*>(at(it.o_reca));
        b.pi_all = static_cast<const int32_t*>(at(it.o_pi));
        b.sstar_all = static_cast<const int32_t*>(at(it.o_sstar));
        b.lpre_all = static_cast<const double*>(at(it.o_lpre));
        for (int p = 0; p < 2; ++p) { b.lam[p] = at(it.o_lam[p]); b.del[p] = at(it.o_del[p]); }
        b.gisl = static_cast<double*>(at(it.o_gisl));
        b.bar = static_cast<unsigned*>(at(it.o_flags));
        b.status = d_status;
        bwd_fill(it, b);
        ba.push_back(b);
      }
    }
    // the batched forward kernel's LDS plan must cover every problem's tiling
    airpf::BatchLaunch L = BL;
    if (probe) L.plain = 1;
    L.blocks = int(bmap.size());
    L.smem = mode == 0 ? airpf::forward_smem(fp64, ppt_f, dx, c_max, G_max, res_max, mult)
                       : airpf::backward_smem(fp64, ppt_b, dx);
    void* d_args = at(o_args);
    if (mode == 0) HIP_OK(hipMemcpyAsync(d_args, fa.data(), sizeof(airpf::FwdArgs) * fa.size(), hipMemcpyHostToDevice, s));
    else HIP_OK(hipMemcpyAsync(d_args, ba.data(), sizeof(airpf::BwdArgs) * ba.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(at(o_bmap), bmap.data(), sizeof(int2) * bmap.size(), hipMemcpyHostToDevice, s));
    L.probs = d_args;
    L.bmap = static_cast<const int2*>(at(o_bmap));
    const hipError_t e = mode == 0 ? airpf::launch_forward_batch(L) : airpf::launch_backward_batch(L);
    // the argument and map uploads are reused by the next launch: wait here
    HIP_OK(hipStreamSynchronize(s));
    return e == hipSuccess ? AIRPF_OK : AIRPF_E_DEVICE;
  };

  std::vector<Item*> all;
  std::vector<int64_t> steps;
  for (Item& it : items) { all.push_back(&it); steps.push_back(it.T); }

  // ---- AIRPF_FLAG_AUTOTUNE: time the tilings of a few cost ratios, for
  // each choice of particles per lane, on the first (up to) 32 steps of
  // every problem (plain forward runs whose results are discarded) and keep
  // the fastest, cached per batch shape ----
  if ((opt.flags & AIRPF_FLAG_AUTOTUNE) && !std::getenv("AIRPF_TILER")) {
    uint64_t key = 0x9E3779B97F4A7C15ULL;
    auto mix = [&](uint64_t v) { key = (key ^ v) * 0xff51afd7ed558ccdULL; key ^= key >> 29; };
    mix(uint64_t(model->kind)); mix(uint64_t(dx)); mix(uint64_t(fp64)); mix(uint64_t(want_score)); mix(uint64_t(mult));
    for (const Item& it : items) { mix(uint64_t(it.T)); mix(uint64_t(it.m)); mix(uint64_t(it.N)); }
    auto hit = ctx->tuned_ratio.find(key);
    double filed = 0.0;
    int filed_ppt = 0;
    if (hit == ctx->tuned_ratio.end() && tune_cache_lookup(key, &filed, &filed_ppt)) {
      hit = ctx->tuned_ratio.emplace(key, filed).first;
      ctx->tuned_ppt[key] = filed_ppt;
    }
    if (hit != ctx->tuned_ratio.end()) {
      ratio = hit->second;
      const auto hp = ctx->tuned_ppt.find(key);
      const int p = hp == ctx->tuned_ppt.end() ? 0 : hp->second;
      if (p != 0 && std::find(ppt_cand.begin(), ppt_cand.end(), p) != ppt_cand.end()) ST_OK(set_ppt(p));
    } else {
      const double cand[] = {1.0 / 32, 1.0 / 8, 1.0 / 3, 1.0, 4.0};
      double best_ms = -1.0, best = ratio;
      int best_ppt = ppt_rule;
      for (int p : ppt_cand) {
      ST_OK(set_ppt(p));
      std::vector<std::vector<int>> seen;
      for (double r : cand) {
        ratio = r;
        std::vector<Item*> tmp = all;
        if (!tile(tmp, steps, cap_fp, ratio)) continue;
        std::vector<int> gs;
        for (const Item* it : tmp) gs.push_back(it->G);
        if (std::find(seen.begin(), seen.end(), gs) != seen.end()) continue;   // same tiling as a ratio tried
        seen.push_back(gs);
        HIP_OK(hipEventRecord(ctx->ev[0], s));
        const airpf_status pst = launch(all, steps, 0, [&](Item& it, airpf::FwdArgs& a) {
          a.T = std::min<int64_t>(it.T, 32);
          a.n1 = a.T;
        }, [](Item&, airpf::BwdArgs&) {}, true);
        HIP_OK(hipEventRecord(ctx->ev[1], s));
        HIP_OK(hipEventSynchronize(ctx->ev[1]));
        if (pst != AIRPF_OK) continue;
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        if (best_ms < 0 || ms < best_ms) { best_ms = ms; best = r; best_ppt = p; }
      }
      }
      ratio = best;
      ST_OK(set_ppt(best_ppt));
      ctx->tuned_ratio[key] = ratio;
      ctx->tuned_ppt[key] = best_ppt;
      tune_cache_store(key, ratio, best_ppt);
    }
  }
  HIP_OK(hipEventRecord(ctx->ev[0], s));
  auto no_bwd = [](Item&, airpf::BwdArgs&) {};
  airpf_status st = launch(all, steps, 0, [&](Item& it, airpf::FwdArgs& a) {
    if (!want_score) return;
    a.tr_pi = static_cast<int32_t*>(at(it.o_pi));
    a.tr_sstar = static_cast<int32_t*>(at(it.o_sstar));
    a.tr_lpre = static_cast<double*>(at(it.o_lpre));
    a.ck_every = it.K;
    a.ck_x = at(it.o_ckx);
    a.ck_L = static_cast<double*>(at(it.o_ckL));
    if (it.C == 1) { a.rec_x = at(it.o_recx); a.rec_anc = static_cast<uint16_t*>(at(it.o_reca)); }
  }, no_bwd);
  if (st != AIRPF_OK) { for (const Item& it : items) item_status[it.idx] = st; return st; }

  if (want_score) {
    // a problem whose islands all died stopped at that step (its records end
    // there): no reverse sweep, its score is zero; a failed forward launch
    // skips every sweep (reported below)
    std::vector<double> lz_fwd(items.size());
    std::vector<int> bad_fwd(items.size());
    int st_fwd = 0;
    HIP_OK(hipMemcpyAsync(lz_fwd.data(), at(o_logz), 8 * lz_fwd.size(), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(bad_fwd.data(), d_bad, 4 * bad_fwd.size(), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(&st_fwd, d_status, 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    auto swept = [&](const Item& it) {
      const size_t i = &it - items.data();
      return st_fwd == 0 && bad_fwd[i] == 0 && lz_fwd[i] != -INFINITY;
    };
    for (Item& it : items) HIP_OK(airpf::fill_u32(at(it.o_gisl), 0u, 2 * int64_t(it.m) * Pn, s));
    int64_t Cmax = 0;
    for (const Item& it : items) Cmax = std::max(Cmax, it.C);
    for (int64_t j = 0; j < Cmax && st == AIRPF_OK; ++j) {
      std::vector<Item*> act, rec;
      std::vector<int64_t> st_act, st_rec;
      for (Item& it : items) {
        const int64_t cidx = it.C - 1 - j;
        if (cidx < 0 || !swept(it)) continue;
        const int64_t lo = cidx * it.K, hi = std::min(it.T, (cidx + 1) * it.K);
        act.push_back(&it);
        st_act.push_back(hi - lo);
        if (it.C > 1) { rec.push_back(&it); st_rec.push_back(hi - lo); }
      }
      st = launch(rec, st_rec, 0, [&](Item& it, airpf::FwdArgs& a) {
        const int64_t cidx = it.C - 1 - j;
        a.n0 = cidx * it.K; a.n1 = std::min(it.T, (cidx + 1) * it.K);
        a.replay_pi = 1; a.ck_in = a.n0 > 0 ? 1 : 0; a.ck_every = it.K;
        a.sstar_in = static_cast<const int32_t*>(at(it.o_sstar));
        a.ck_x = at(it.o_ckx); a.ck_L = static_cast<double*>(at(it.o_ckL));
        a.tr_pi = static_cast<int32_t*>(at(it.o_pi));
        a.rec_x = at(it.o_recx); a.rec_anc = static_cast<uint16_t*>(at(it.o_reca));
      }, no_bwd);
      if (st != AIRPF_OK) break;
      st = launch(act, st_act, 1, [](Item&, airpf::FwdArgs&) {}, [&](Item& it, airpf::BwdArgs& b) {
        const int64_t cidx = it.C - 1 - j;
        b.n_lo = cidx * it.K; b.n_hi = std::min(it.T, (cidx + 1) * it.K);
      });
    }
    if (st == AIRPF_OK)
      for (Item& it : items)
        HIP_OK(airpf::launch_island_grad_sum(static_cast<const double*>(at(it.o_gisl)), it.m, Pn,
                                             static_cast<double*>(at(it.o_gsum)), s));
  }
  HIP_OK(hipEventRecord(ctx->ev[1], s));
  if (st != AIRPF_OK) { for (const Item& it : items) item_status[it.idx] = st; return st; }

  std::vector<double> lz(items.size());
  std::vector<int> bad(items.size());
  int kstatus = 0;
  HIP_OK(hipMemcpyAsync(lz.data(), at(o_logz), 8 * lz.size(), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(bad.data(), d_bad, 4 * bad.size(), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&kstatus, d_status, 4, hipMemcpyDeviceToHost, s));
  if (want_score)
    for (const Item& it : items)
      HIP_OK(hipMemcpyAsync(grad_out + size_t(it.idx) * Pn, at(it.o_gsum), 8 * size_t(Pn), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (kstatus != 0) {
    for (const Item& it : items) item_status[it.idx] = AIRPF_E_DEVICE;
    return AIRPF_E_DEVICE;
  }
  float ms = 0.0f;
  HIP_OK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  ctx->last_kernel_ms = ms;
  for (size_t i = 0; i < items.size(); ++i) {
    if (bad[i]) {                                  // reported per item; the outputs stay NaN
      item_status[items[i].idx] = AIRPF_E_INVALID_ARG;
      if (want_score) for (int q = 0; q < Pn; ++q) grad_out[size_t(items[i].idx) * Pn + q] = std::nan("");
      continue;
    }
    log_z_out[items[i].idx] = lz[i];
  }
  return AIRPF_OK;
}
