// State-space models on the device: initial draw, mutation kernel K and the
// per-particle part of log g_n (Section 1.2's HMM; the concrete models are
// listed in include/airpf.h).  Arithmetic is double precision; a state kept
// in binary32 is rounded once when produced, and every later use reads the
// rounded value.  Operation order is part of the contract with the CPU
// checker (explicit fma only):
//   LG1  x_0 = z;  x' = fma(a, x, sx*z);  lw = -0.5*(r*r), r = (y - x)/sy
//   SV   x_0 = fma(s0, z, mu);  x' = fma(phi, x - mu, fma(sigma, z, mu));
//        lw = fma(-(0.5*(y*y)), exp(-x), -0.5*x)
//   LGD  x_0[d] = sqrt(p0)*z_d;  x'[i] = sqrt(q)*z_i then fma(A[i][c], x[c], .)
//        over c;  e_i = y_i then fma(-H[i][c], x[c], .) over c;
//        ss = fma(e_i, e_i, ss) over i;  lw = -(ss*(1/(2r)))
//
// Derivatives for the score (plain double arithmetic, no bit-exactness
// contract): d lw/dx, d log g/d theta (the constant of log g included),
// and vector-Jacobian products of the mutation x' = F(x, z; theta) and of
// the initial draw.
#pragma once
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
  int dy;
};

template <typename Store>
__device__ __forceinline__ double round_store(double v) {
  return static_cast<double>(static_cast<Store>(v));
}

struct LG1 {
  static constexpr int DX = 1;
  static constexpr bool kThetaOuter = false;   // see LGD
  template <typename Store>
  __device__ static void init(const ModelArgs&, const double* z, double* x) { x[0] = round_store<Store>(z[0]); }
  template <typename Store>
  __device__ static void prop(const ModelArgs& p, const double* xp, const double* z, double* x) {
    x[0] = round_store<Store>(fma(p.th[0], xp[0], p.th[1] * z[0]));
  }
  __device__ static double logpot(const ModelArgs& p, const double* x, const double* y) {
    const double r = (y[0] - x[0]) / p.th[2];
    return -0.5 * (r * r);
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
  static constexpr bool kThetaOuter = false;   // see LGD
  template <typename Store>
  __device__ static void init(const ModelArgs& p, const double* z, double* x) {
    x[0] = round_store<Store>(fma(p.s0, z[0], p.th[0]));
  }
  template <typename Store>
  __device__ static void prop(const ModelArgs& p, const double* xp, const double* z, double* x) {
    const double mu = p.th[0];
    x[0] = round_store<Store>(fma(p.th[1], xp[0] - mu, fma(p.th[2], z[0], mu)));
  }
  __device__ static double logpot(const ModelArgs&, const double* x, const double* y) {
    const double h = 0.5 * (y[0] * y[0]);
    return fma(-h, dexp(-x[0]), -0.5 * x[0]);
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

template <int D>
struct LGD {
  static constexpr int DX = D;
  template <typename Store>
  __device__ static void init(const ModelArgs& p, const double* z, double* x) {
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = round_store<Store>(p.sp0 * z[d]);
  }
  template <typename Store>
  __device__ static void prop(const ModelArgs& p, const double* xp, const double* z, double* x) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double acc = p.sq * z[i];
#pragma unroll
      for (int c = 0; c < D; ++c) acc = fma(p.th[i * D + c], xp[c], acc);
      x[i] = round_store<Store>(acc);
    }
  }
  __device__ static double logpot(const ModelArgs& p, const double* x, const double* y) {
    double ss = 0.0;
    for (int i = 0; i < p.dy; ++i) {
      double e = y[i];
#pragma unroll
      for (int c = 0; c < D; ++c) e = fma(-p.H[i * D + c], x[c], e);
      ss = fma(e, e, ss);
    }
    return -(ss * p.hr);
  }
  // theta = A: the transition's theta-tangent contracted with the child's
  // adjoint is lam xp^T (an outer product), and g and x_0 do not depend on
  // theta, so a step's contribution of a slot is (sum over its children of
  // lam) xp^T, formed once per slot instead of once per child
  static constexpr bool kThetaOuter = true;
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
