// State-space models on the device: initial draw, mutation kernel K and the
// per-particle part of log g_n (Section 1.2's HMM; the concrete models are
// listed in include/airpf.h).  The particle arithmetic is done in the
// particles' own precision R (double, or binary32 with every parameter and
// derived constant rounded once to binary32 on the host and the observation
// rounded to binary32).  Operation order is part of the contract with the
// CPU checker (explicit fma only):
//   LG1  x_0 = z;  x' = fma(a, x, sx*z);  lw = -0.5*(r*r),
//        r = (y - x)/sy (double) or (y - x)*isy, isy = 1/sy (binary32)
//   SV   x_0 = fma(s0, z, mu);  x' = fma(phi, x - mu, fma(sigma, z, mu));
//        lw = fma(-(0.5*(y*y)), exp(-x), -0.5*x)
//   LGD  x_0[d] = sqrt(p0)*z_d;  x'[i] = sqrt(q)*z_i then fma(A[i][c], x[c], .)
//        over c;  e_i = y_i then fma(-H[i][c], x[c], .) over c;
//        ss = fma(e_i, e_i, ss) over i;  lw = -(ss*(1/(2r)))
//   BIN  z is the particle's raw 32-bit word (not a normal variate):
//        x_0 = bit 31 of z;  x' = 1 - x when bits 31..30 of z are zero,
//        else x;  lw = 0 when x == y, else -log 3
//   BCP  z is the particle's eight raw words; x = (log r, log(1 - r)) of a
//        rate r:  x_0 = beta(z);  x' = beta(z) when z_0 2^-32 < p, else x;
//        beta(z): ga = 0, ga -= log((z_i + 1/2) 2^-32) for i = 1..alpha;
//        gb likewise over i = alpha+1..alpha+beta;  ls = log(ga + gb);
//        x = (log ga - ls, log gb - ls);  lw = y_0 x_0 + (y_1 - y_0) x_1
//
// Derivatives for the score (plain double arithmetic, no bit-exactness
// contract): d lw/dx, d log g/d theta (the constant of log g included),
// and vector-Jacobian products of the mutation x' = F(x, z; theta) and of
// the initial draw.
#pragma once
#include <type_traits>

#include "dev_math.h"

namespace airpf {

constexpr int kMaxTheta = 64;
constexpr int kMaxDy = 8;

// Parameters of one problem, passed by value as a kernel argument.
struct ModelArgs {
  double th[kMaxTheta];
  double H[kMaxDy * 8];
  double s0, sq, sp0, hr;
  double ds0_dphi, ds0_dsig;  // SV: derivatives of the stationary sd
  // binary32 particles: the same parameters and constants rounded once
  float thf[kMaxTheta];
  float Hf[kMaxDy * 8];
  float s0f, sqf, sp0f, hrf, isyf;
  double log3;                // BIN: log 3 from the host
  int ab[2];                  // BCP: the integer Beta shapes (alpha, beta)
  int dy;
};

template <typename R> __device__ __forceinline__ constexpr bool is_f32() { return std::is_same<R, float>::value; }
template <typename R> __device__ __forceinline__ R rfma(R a, R b, R c) {
  if constexpr (is_f32<R>()) return fmaf(a, b, c); else return fma(a, b, c);
}
// parameter i, and entry i of H, in the particles' precision
template <typename R> __device__ __forceinline__ R par(const ModelArgs& p, int i) {
  if constexpr (is_f32<R>()) return p.thf[i]; else return p.th[i];
}
template <typename R> __device__ __forceinline__ R hpar(const ModelArgs& p, int i) {
  if constexpr (is_f32<R>()) return p.Hf[i]; else return p.H[i];
}

struct LG1 {
  static constexpr int DX = 1;
  static constexpr bool kWordNoise = false;     // N(0,1) noise
  static constexpr bool kThetaOuter = false;   // see LGD
  template <typename R>
  __device__ static void init(const ModelArgs&, const R* z, R* x) { x[0] = z[0]; }
  template <typename R>
  __device__ static void prop(const ModelArgs& p, const R* xp, const R* z, R* x) {
    x[0] = rfma<R>(par<R>(p, 0), xp[0], par<R>(p, 1) * z[0]);
  }
  template <typename R>
  __device__ static R logpot(const ModelArgs& p, const R* x, const double* y) {
    if constexpr (is_f32<R>()) {
      const float r = (static_cast<float>(y[0]) - x[0]) * p.isyf;
      return -0.5f * (r * r);
    } else {
      const double r = (y[0] - x[0]) / p.th[2];
      return -0.5 * (r * r);
    }
  }
  static constexpr int P = 3;
  __device__ static void dlogpot_dx(const ModelArgs& p, const double* x, const double* y, double* g) {
    const double sy = p.th[2];
    g[0] = (y[0] - x[0]) / (sy * sy);
  }
  __device__ static void dlogpot_dtheta(const ModelArgs& p, const double* x, const double* y, double w, double* acc) {
    const double sy = p.th[2], e = y[0] - x[0];
    acc[2] += w * (e * e / (sy * sy * sy) - 1.0 / sy);
  }
  __device__ static void prop_vjp_x(const ModelArgs& p, const double* lam, double* out) { out[0] = p.th[0] * lam[0]; }
  __device__ static void prop_vjp_theta(const ModelArgs&, const double* xp, const double* z, const double* lam,
                                        double* acc) {
    acc[0] += lam[0] * xp[0];
    acc[1] += lam[0] * z[0];
  }
  __device__ static void init_vjp_theta(const ModelArgs&, const double*, const double*, double*) {}
};

struct SV {
  static constexpr int DX = 1;
  static constexpr bool kWordNoise = false;     // N(0,1) noise
  static constexpr bool kThetaOuter = false;   // see LGD
  template <typename R>
  __device__ static void init(const ModelArgs& p, const R* z, R* x) {
    if constexpr (is_f32<R>()) x[0] = fmaf(p.s0f, z[0], p.thf[0]);
    else x[0] = fma(p.s0, z[0], p.th[0]);
  }
  template <typename R>
  __device__ static void prop(const ModelArgs& p, const R* xp, const R* z, R* x) {
    const R mu = par<R>(p, 0);
    x[0] = rfma<R>(par<R>(p, 1), xp[0] - mu, rfma<R>(par<R>(p, 2), z[0], mu));
  }
  template <typename R>
  __device__ static R logpot(const ModelArgs&, const R* x, const double* y) {
    const R yr = static_cast<R>(y[0]);
    const R h = R(0.5) * (yr * yr);
    return rfma<R>(-h, rexp(-x[0]), R(-0.5) * x[0]);
  }
  static constexpr int P = 3;
  __device__ static void dlogpot_dx(const ModelArgs&, const double* x, const double* y, double* g) {
    g[0] = -0.5 + 0.5 * y[0] * y[0] * dexp(-x[0]);
  }
  __device__ static void dlogpot_dtheta(const ModelArgs&, const double*, const double*, double, double*) {}
  __device__ static void prop_vjp_x(const ModelArgs& p, const double* lam, double* out) { out[0] = p.th[1] * lam[0]; }
  __device__ static void prop_vjp_theta(const ModelArgs& p, const double* xp, const double* z, const double* lam,
                                        double* acc) {
    acc[0] += lam[0] * (1.0 - p.th[1]);
    acc[1] += lam[0] * (xp[0] - p.th[0]);
    acc[2] += lam[0] * z[0];
  }
  __device__ static void init_vjp_theta(const ModelArgs& p, const double* z, const double* lam, double* acc) {
    acc[0] += lam[0];
    acc[1] += lam[0] * z[0] * p.ds0_dphi;
    acc[2] += lam[0] * z[0] * p.ds0_dsig;
  }
};

// The binary toy HMM of the exact-variance example (Section 4.1): a
// two-state chain that starts uniform and flips with probability 1/4 per
// step, observed through a channel that reports the state with probability
// 3/4.  A particle's noise is one raw 32-bit word per step (drawn with its
// own tag), so the states stay exactly 0 or 1 and the log-potential takes
// the two values 0 and -log 3 (the constant log(3/4) is added per island).
// No parameters; forward only.
struct BIN {
  static constexpr int DX = 1;
  static constexpr bool kWordNoise = true;
  static constexpr int kWords = 1;            // raw words per particle and step
  static constexpr uint32_t kTag = kTagBin;
  static constexpr bool kThetaOuter = false;
  static constexpr int P = 0;
  template <typename R>
  __device__ static void init(const ModelArgs&, const R* z, R* x) {
    x[0] = static_cast<R>(static_cast<uint32_t>(z[0]) >> 31);
  }
  template <typename R>
  __device__ static void prop(const ModelArgs&, const R* xp, const R* z, R* x) {
    x[0] = (static_cast<uint32_t>(z[0]) >> 30) == 0u ? R(1) - xp[0] : xp[0];
  }
  template <typename R>
  __device__ static R logpot(const ModelArgs& p, const R* x, const double* y) {
    return static_cast<double>(x[0]) == y[0] ? R(0) : static_cast<R>(-p.log3);
  }
};

// The Beta change-point model of the change-point experiment (Section 4.2):
// a rate r in (0, 1) that keeps its value from one step to the next with
// probability 1 - p and is otherwise drawn afresh from Beta(alpha, beta)
// (its initial law too), observed through counts y = (k, n) with g = r^k
// (1 - r)^(n - k).  The state is (log r, log(1 - r)); a Beta draw is the
// ratio of two sums of unit exponentials (integer shapes, alpha + beta <= 7),
// each a -log of a uniform from one of the particle's eight raw words (two
// Philox blocks, tag 6), word 0 deciding the change.  theta = (p); forward
// only, states in double.
struct BCP {
  static constexpr int DX = 2;
  static constexpr bool kWordNoise = true;
  static constexpr int kWords = 8;
  static constexpr uint32_t kTag = kTagBcp;
  static constexpr bool kThetaOuter = false;
  static constexpr int P = 1;
  __device__ static void beta(const ModelArgs& p, const double* z, double* x) {
    double ga = 0.0, gb = 0.0;
    for (int i = 1; i <= p.ab[0]; ++i) ga -= dlog((z[i] + 0.5) * 0x1p-32);
    for (int i = p.ab[0] + 1; i <= p.ab[0] + p.ab[1]; ++i) gb -= dlog((z[i] + 0.5) * 0x1p-32);
    const double ls = dlog(ga + gb);
    x[0] = dlog(ga) - ls;
    x[1] = dlog(gb) - ls;
  }
  template <typename R>
  __device__ static void init(const ModelArgs& p, const R* z, R* x) {
    static_assert(std::is_same<R, double>::value, "raw words and log rates are kept in double");
    beta(p, z, x);
  }
  template <typename R>
  __device__ static void prop(const ModelArgs& p, const R* xp, const R* z, R* x) {
    if (z[0] * 0x1p-32 < p.th[0]) {
      beta(p, z, x);
    } else {
      x[0] = xp[0];
      x[1] = xp[1];
    }
  }
  template <typename R>
  __device__ static R logpot(const ModelArgs&, const R* x, const double* y) {
    return y[0] * x[0] + (y[1] - y[0]) * x[1];
  }
};

template <int D>
struct LGD {
  static constexpr int DX = D;
  template <typename R>
  __device__ static void init(const ModelArgs& p, const R* z, R* x) {
    const R sp0 = is_f32<R>() ? R(p.sp0f) : R(p.sp0);
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = sp0 * z[d];
  }
  template <typename R>
  __device__ static void prop(const ModelArgs& p, const R* xp, const R* z, R* x) {
    const R sq = is_f32<R>() ? R(p.sqf) : R(p.sq);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      R acc = sq * z[i];
#pragma unroll
      for (int c = 0; c < D; ++c) acc = rfma<R>(par<R>(p, i * D + c), xp[c], acc);
      x[i] = acc;
    }
  }
  template <typename R>
  __device__ static R logpot(const ModelArgs& p, const R* x, const double* y) {
    R ss = R(0);
    for (int i = 0; i < p.dy; ++i) {
      R e = static_cast<R>(y[i]);
#pragma unroll
      for (int c = 0; c < D; ++c) e = rfma<R>(-hpar<R>(p, i * D + c), x[c], e);
      ss = rfma<R>(e, e, ss);
    }
    const R hr = is_f32<R>() ? R(p.hrf) : R(p.hr);
    return -(ss * hr);
  }
  // theta = A: the transition's theta-tangent contracted with the child's
  // adjoint is lam xp^T (an outer product), and g and x_0 do not depend on
  // theta, so a step's contribution of a slot is (sum over its children of
  // lam) xp^T, formed once per slot instead of once per child
  static constexpr bool kThetaOuter = true;
  static constexpr bool kWordNoise = false;
  static constexpr int P = D * D;
  __device__ static void dlogpot_dx(const ModelArgs& p, const double* x, const double* y, double* g) {
    const double inv_r = 2.0 * p.hr;
#pragma unroll
    for (int c = 0; c < D; ++c) g[c] = 0.0;
    for (int i = 0; i < p.dy; ++i) {
      double e = y[i];
#pragma unroll
      for (int c = 0; c < D; ++c) e -= p.H[i * D + c] * x[c];
#pragma unroll
      for (int c = 0; c < D; ++c) g[c] += p.H[i * D + c] * e * inv_r;
    }
  }
  __device__ static void dlogpot_dtheta(const ModelArgs&, const double*, const double*, double, double*) {}
  __device__ static void prop_vjp_x(const ModelArgs& p, const double* lam, double* out) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) acc += p.th[i * D + c] * lam[i];
      out[c] = acc;
    }
  }
  __device__ static void prop_vjp_theta(const ModelArgs&, const double* xp, const double*, const double* lam,
                                        double* acc) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[i * D + c] += lam[i] * xp[c];
  }
  __device__ static void init_vjp_theta(const ModelArgs&, const double*, const double*, double*) {}
};

}  // namespace airpf
