// C ABI of the AIRPF library (declared in include/airpf.h): argument
// validation, model constants, device workspaces and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "airpf.h"
#include "internal.h"

namespace {

// Grow-only device buffer owned by a context.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  airpf_status ensure(size_t bytes) {
    if (bytes <= cap) return AIRPF_OK;
    if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
    size_t want = bytes < 256 ? 256 : bytes;
    if (hipMalloc(&p, want) != hipSuccess) { p = nullptr; return AIRPF_E_NOMEM; }
    cap = want;
    return AIRPF_OK;
  }
  void release() { if (p) (void)hipFree(p); p = nullptr; cap = 0; }
};

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) { int s = 0; while ((int64_t(1) << s) < v) ++s; return s; }
bool all_finite(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i) if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

struct airpf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  double last_kernel_ms = 0.0;
  DevBuf x1[2], tree[2], part[2], misc, ybuf;
  DevBuf t_sstar, t_enf, t_lpost, t_anc, t_pi, t_dig;
  DevBuf dbg_in, dbg_in32, dbg_out, dbg_out2, dbg_out32;
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
      hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess) {
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
                    &c->ybuf, &c->t_sstar, &c->t_enf, &c->t_lpost, &c->t_anc, &c->t_pi, &c->t_dig,
                    &c->dbg_in, &c->dbg_in32, &c->dbg_out, &c->dbg_out2, &c->dbg_out32})
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
  if (!model || !theta) return AIRPF_E_INVALID_ARG;
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
    default:
      return AIRPF_E_INVALID_ARG;
  }
  for (int i = 0; i < d_theta; ++i) mp->th[i] = theta[i];
  mp->dy = dy;
  *cst_q = c_log - 40.0 * std::log(2.0) - std::log(static_cast<double>(N));
  *dx_out = dx;
  *dy_out = dy;
  return AIRPF_OK;
}

airpf_options default_options() {
  airpf_options o;
  o.tau = 0.3;
  o.resampling = AIRPF_SYSTEMATIC;
  o.precision = AIRPF_FP32;
  o.score_mode = AIRPF_PATHSPACE;
  o.ckpt_every = 0;
  o.flags = 0;
  return o;
}

void set_nan(double* p) { if (p) *p = std::nan(""); }

}  // namespace

extern "C" airpf_status airpf_run(airpf_ctx* ctx, const airpf_model* model, const double* theta, int32_t d_theta,
                                  const double* y, int64_t T, int32_t m, int32_t N, uint64_t seed,
                                  const airpf_options* opt_in, double* log_z_out, airpf_trace* trace) {
  set_nan(log_z_out);
  if (!ctx || !model || !theta || !y || !log_z_out) return AIRPF_E_INVALID_ARG;
  if (T < 1 || T > (int64_t(1) << 30) || !is_pow2(m) || m > (1 << 24) || N < 1 || N > 2048)
    return AIRPF_E_INVALID_ARG;
  const airpf_options opt = opt_in ? *opt_in : default_options();
  if (!(opt.tau == opt.tau)) return AIRPF_E_INVALID_ARG;
  if (opt.precision != AIRPF_FP32 && opt.precision != AIRPF_FP64) return AIRPF_E_INVALID_ARG;
  if (opt.resampling != AIRPF_SYSTEMATIC) return AIRPF_E_UNSUPPORTED;

  airpf::FwdArgs a;
  std::memset(&a, 0, sizeof(a));
  int dx = 1, dy = 1;
  const airpf_status st = prepare_model(model, theta, d_theta, N, &a.mp, &a.cst_q, &dx, &dy);
  if (st == AIRPF_E_DOMAIN) { *log_z_out = -INFINITY; return st; }
  if (st != AIRPF_OK) return st;
  const bool y_dev = (opt.flags & AIRPF_FLAG_Y_ON_DEVICE) != 0;
  if (!y_dev && !all_finite(y, T * dy)) return AIRPF_E_INVALID_ARG;

  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int S = ilog2(m);
  const bool want_enf = trace && trace->enf;
  a.T = T; a.m = m; a.N = N; a.S = S; a.dy = dy; a.seed = seed; a.tau = opt.tau;
  a.shortcut_all = (opt.tau > 1.0 + 1e-9) && !want_enf;

  airpf::FwdLaunch L;
  L.kind = model->kind; L.dx = dx; L.fp64 = opt.precision == AIRPF_FP64;
  L.num_cus = ctx->num_cus; L.max_blocks = 1024; L.plan_only = 1; L.stream = s;
  airpf::FwdPlan plan;
  HIP_OK(airpf::launch_forward(L, a, &plan));

  const size_t store = L.fp64 ? 8 : 4;
  const size_t nstate = size_t(m) * N * dx * store;
  const int lc = ilog2(plan.c);
  for (int p = 0; p < 2; ++p) {
    ST_OK(ctx->x1[p].ensure(nstate));
    ST_OK(ctx->tree[p].ensure(sizeof(double) * 2 * size_t(m)));
    ST_OK(ctx->part[p].ensure(sizeof(double) * size_t(lc + 1) * plan.G));
    a.x1[p] = ctx->x1[p].p;
    a.tree[p] = static_cast<double*>(ctx->tree[p].p);
    a.part[p] = static_cast<double*>(ctx->part[p].p);
  }
  // misc: [0,8) log Zhat, [8,12) status, [64, 64 + 4G) barrier flags
  ST_OK(ctx->misc.ensure(64 + 4 * size_t(plan.G)));
  unsigned char* misc = static_cast<unsigned char*>(ctx->misc.p);
  a.out_logz = reinterpret_cast<double*>(misc);
  a.status = reinterpret_cast<int*>(misc + 8);
  a.bar = reinterpret_cast<unsigned*>(misc + 64);
  if (y_dev) {
    a.y = y;
  } else {
    ST_OK(ctx->ybuf.ensure(sizeof(double) * size_t(T) * dy));
    HIP_OK(hipMemcpyAsync(ctx->ybuf.p, y, sizeof(double) * size_t(T) * dy, hipMemcpyHostToDevice, s));
    a.y = static_cast<const double*>(ctx->ybuf.p);
  }
  HIP_OK(airpf::fill_u32(misc, 0u, 16 + int64_t(plan.G), s));

  if (trace) {
    if (trace->sstar) { ST_OK(ctx->t_sstar.ensure(4 * size_t(T))); a.tr_sstar = static_cast<int32_t*>(ctx->t_sstar.p);
                        HIP_OK(airpf::fill_u32(a.tr_sstar, 0u, T, s)); }
    if (trace->enf) { ST_OK(ctx->t_enf.ensure(8 * size_t(T) * (S + 1))); a.tr_enf = static_cast<double*>(ctx->t_enf.p);
                      HIP_OK(airpf::fill_u32(a.tr_enf, 0x7ff80000u, 2 * int64_t(T) * (S + 1), s)); }
    if (trace->lpost) { ST_OK(ctx->t_lpost.ensure(8 * size_t(T) * m)); a.tr_lpost = static_cast<double*>(ctx->t_lpost.p); }
    if (trace->anc && T > 1) { ST_OK(ctx->t_anc.ensure(4 * size_t(T - 1) * m * N)); a.tr_anc = static_cast<int32_t*>(ctx->t_anc.p); }
    if (trace->pi && T > 1) { ST_OK(ctx->t_pi.ensure(4 * size_t(T - 1) * m)); a.tr_pi = static_cast<int32_t*>(ctx->t_pi.p); }
    if (trace->digest) { ST_OK(ctx->t_dig.ensure(16 * size_t(T))); a.tr_digest = static_cast<unsigned long long*>(ctx->t_dig.p);
                         HIP_OK(airpf::fill_u32(a.tr_digest, 0u, 4 * int64_t(T), s)); }
  }

  L.plan_only = 0;
  HIP_OK(hipEventRecord(ctx->ev[0], s));
  if (airpf::launch_forward(L, a, &plan) != hipSuccess) return AIRPF_E_DEVICE;
  HIP_OK(hipEventRecord(ctx->ev[1], s));

  double lz = 0.0;
  int kstatus = 0;
  HIP_OK(hipMemcpyAsync(&lz, a.out_logz, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&kstatus, a.status, sizeof(int), hipMemcpyDeviceToHost, s));
  if (trace) {
    if (a.tr_sstar) HIP_OK(hipMemcpyAsync(trace->sstar, a.tr_sstar, 4 * size_t(T), hipMemcpyDeviceToHost, s));
    if (a.tr_enf) HIP_OK(hipMemcpyAsync(trace->enf, a.tr_enf, 8 * size_t(T) * (S + 1), hipMemcpyDeviceToHost, s));
    if (a.tr_lpost) HIP_OK(hipMemcpyAsync(trace->lpost, a.tr_lpost, 8 * size_t(T) * m, hipMemcpyDeviceToHost, s));
    if (a.tr_anc) HIP_OK(hipMemcpyAsync(trace->anc, a.tr_anc, 4 * size_t(T - 1) * m * N, hipMemcpyDeviceToHost, s));
    if (a.tr_pi) HIP_OK(hipMemcpyAsync(trace->pi, a.tr_pi, 4 * size_t(T - 1) * m, hipMemcpyDeviceToHost, s));
    if (a.tr_digest) HIP_OK(hipMemcpyAsync(trace->digest, a.tr_digest, 16 * size_t(T), hipMemcpyDeviceToHost, s));
  }
  HIP_OK(hipStreamSynchronize(s));
  if (kstatus != 0) return AIRPF_E_DEVICE;
  float ms = 0.0f;
  HIP_OK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  ctx->last_kernel_ms = ms;
  *log_z_out = lz;
  return AIRPF_OK;
}

extern "C" airpf_status airpf_ctx_last_kernel_ms(airpf_ctx* ctx, double* ms) {
  if (!ctx || !ms) return AIRPF_E_INVALID_ARG;
  *ms = ctx->last_kernel_ms;
  return AIRPF_OK;
}

extern "C" airpf_status airpf_debug_eval(airpf_ctx* ctx, int32_t which, int64_t n, const double* in,
                                         const uint32_t* in_u32, double* out, double* out2, uint32_t* out_u32) {
  if (!ctx || n < 0 || which < 0 || which > 4) return AIRPF_E_INVALID_ARG;
  if (n == 0) return AIRPF_OK;
  const bool uses_in = which <= 2, uses_in32 = which >= 3, uses_out2 = which == 2 || which == 3;
  if ((uses_in && !in) || (uses_in32 && !in_u32) || (which <= 3 && !out) || (uses_out2 && !out2) ||
      (which == 4 && !out_u32))
    return AIRPF_E_INVALID_ARG;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const size_t n32 = which == 3 ? 2 * size_t(n) : 6 * size_t(n);
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
  if (which <= 3) HIP_OK(hipMemcpyAsync(out, ctx->dbg_out.p, 8 * size_t(n), hipMemcpyDeviceToHost, s));
  if (uses_out2) HIP_OK(hipMemcpyAsync(out2, ctx->dbg_out2.p, 8 * size_t(n), hipMemcpyDeviceToHost, s));
  if (which == 4) HIP_OK(hipMemcpyAsync(out_u32, ctx->dbg_out32.p, 16 * size_t(n), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return AIRPF_OK;
}
