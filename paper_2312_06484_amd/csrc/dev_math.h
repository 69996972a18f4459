// Device-side counter-based draws and elementary functions for gfx950.
//
// Contract shared (as a written specification, not as code) with the CPU
// checker, so that every integer decision of the filter -- fixed-point
// weights, ancestors, island selections -- comes out identical (runs with
// binary32 particles use the binary32 set further below):
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed lo, seed
//    hi), counter = (c0, island, step, tag << 24 | sub).
//  * exp, log and (cos, sin)(2 pi v) evaluated with correctly rounded IEEE
//    double operations only (fma, +, *, /, sqrt, rint): Cody-Waite reduction
//    with a two-part ln 2 and a degree-13 Taylor polynomial for exp; the
//    atanh series in s = (f-1)/(f+1) to s^23 for log; Taylor series of sin
//    and cos on [-pi/4, pi/4] after a quarter-turn reduction of v.
//  * Box-Muller: u1 = (w0 + 1/2) 2^-32, v = w1 2^-32, r = sqrt(-2 log u1),
//    (r cos 2 pi v, r sin 2 pi v).
// This file is compiled with -ffp-contract=off; fused operations are the
// explicit fma() calls.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace airpf {

enum : uint32_t { kTagNormal = 1, kTagSys = 2, kTagMult = 3, kTagIsl = 4, kTagBin = 5, kTagBcp = 6 };

struct Key { uint32_t k0, k1; };

__host__ __device__ inline Key make_key(uint64_t seed) {
  return Key{static_cast<uint32_t>(seed & 0xffffffffu), static_cast<uint32_t>(seed >> 32)};
}

// Philox4x32-10 bijection of the 128-bit counter (w) under the key.
__device__ __forceinline__ void philox4x32_10(uint32_t w[4], Key key) {
  uint32_t ka = key.k0, kb = key.k1;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = w[0] * 0xD2511F53u, hi0 = __umulhi(w[0], 0xD2511F53u);
    const uint32_t lo1 = w[2] * 0xCD9E8D57u, hi1 = __umulhi(w[2], 0xCD9E8D57u);
    const uint32_t n0 = hi1 ^ w[1] ^ ka;
    const uint32_t n2 = hi0 ^ w[3] ^ kb;
    w[0] = n0; w[1] = lo1; w[2] = n2; w[3] = lo0;
    ka += 0x9E3779B9u;
    kb += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void draw4(Key key, uint32_t c0, uint32_t island, uint32_t step,
                                      uint32_t tag, uint32_t sub, uint32_t w[4]) {
  w[0] = c0; w[1] = island; w[2] = step; w[3] = (tag << 24) | (sub & 0xffffffu);
  philox4x32_10(w, key);
}

// uniform on [0,1) from 53 bits of (hi, lo)
__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
  const uint64_t b = (static_cast<uint64_t>(hi) << 32) | lo;
  return static_cast<double>(b >> 11) * 0x1p-53;
}

// Uniform integer in [0, Q), Q >= 1: Lemire's multiply-and-reject on 64-bit
// candidates taken as (w0:w1), (w2:w3) of sub-blocks 0, 1, ..., at most 64
// sub-blocks (then the last candidate is used as is).  A candidate c is
// accepted iff the low word of c*Q is at least 2^64 mod Q; as that bound is
// below Q, the 64-bit remainder is only evaluated when the low word is below
// Q (probability Q/2^64).  `w0` is sub-block 0, drawn by the caller (it does
// not depend on Q).
__device__ inline uint64_t bounded_u64_from(const uint32_t w0[4], Key key, uint32_t c0, uint32_t island,
                                            uint32_t step, uint32_t tag, uint64_t Q) {
  uint64_t reject_below = 0;
  bool have_bound = false;
  uint64_t hi = 0;
  uint32_t w[4] = {w0[0], w0[1], w0[2], w0[3]};
  for (uint32_t sub = 0; sub < 64; ++sub) {
    if (sub > 0) draw4(key, c0, island, step, tag, sub, w);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t cand = (static_cast<uint64_t>(w[2 * h]) << 32) | w[2 * h + 1];
      hi = __umul64hi(cand, Q);
      const uint64_t lo = cand * Q;
      if (lo >= Q) return hi;
      if (!have_bound) { reject_below = (~Q + 1) % Q; have_bound = true; }   // 2^64 mod Q
      if (lo >= reject_below) return hi;
    }
  }
  return hi;
}

__device__ inline uint64_t bounded_u64(Key key, uint32_t c0, uint32_t island, uint32_t step, uint32_t tag, uint64_t Q) {
  uint32_t w[4];
  draw4(key, c0, island, step, tag, 0, w);
  return bounded_u64_from(w, key, c0, island, step, tag, Q);
}

// ---------------------------------------------------------------- exp / log

// Polynomial coefficients, evaluated by the compiler: 1/k! for k = 0..20
// (k! is exact in double for k <= 22, so each entry is 1/k! correctly
// rounded) and 1/(2i+1) for i = 0..11.
struct CoeffTables {
  double inv_fact[21];
  double inv_odd[12];
};
constexpr CoeffTables make_coeff_tables() {
  CoeffTables t{};
  double f = 1.0;
  for (int k = 0; k <= 20; ++k) {
    if (k > 0) f *= k;
    t.inv_fact[k] = 1.0 / f;
  }
  for (int i = 0; i < 12; ++i) t.inv_odd[i] = 1.0 / (2 * i + 1);
  return t;
}
constexpr CoeffTables kCoeff = make_coeff_tables();
template <int K> struct InvFact { static constexpr double value = kCoeff.inv_fact[K]; };
template <int I> struct InvOdd { static constexpr double value = kCoeff.inv_odd[I]; };

constexpr double kLn2Head = 0x1.62e42fee00000p-1;   // ln 2, 32 significant bits
constexpr double kLn2Tail = 0x1.a39ef35793c76p-33;  // ln 2 - head
constexpr double kLn2 = 0x1.62e42fefa39efp-1;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kTwoPi = 0x1.921fb54442d18p+2;

__device__ __forceinline__ double scale2(double p, int k) {  // p * 2^k, -1022 <= k <= 1023
  return p * __longlong_as_double(static_cast<long long>(k + 1023) << 52);
}

// Branch-free: every lane runs the same instructions and the special cases
// (NaN, overflow, underflow) are selected at the end.  p * 2^k is one
// correctly rounded scaling (v_ldexp_f64), which equals the reference's
// scaling by exact powers of two, including its two-step scaling into the
// subnormal range (one rounding either way).
__device__ inline double dexp(double x) {
  const double kd = rint(x * kInvLn2);
  const double r = fma(-kd, kLn2Tail, fma(-kd, kLn2Head, x));
  // e^r = 1 + (r + r^2 Q(r)), Q(r) = sum_{i=2}^{13} r^{i-2} / i! by Estrin's
  // scheme (adjacent pairs, then powers r^2, r^4, r^8); the leading 1 is
  // added last
  const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  const double q0 = fma(InvFact<3>::value, r, InvFact<2>::value);
  const double q1 = fma(InvFact<5>::value, r, InvFact<4>::value);
  const double q2 = fma(InvFact<7>::value, r, InvFact<6>::value);
  const double q3 = fma(InvFact<9>::value, r, InvFact<8>::value);
  const double q4 = fma(InvFact<11>::value, r, InvFact<10>::value);
  const double q5 = fma(InvFact<13>::value, r, InvFact<12>::value);
  const double s0 = fma(q1, r2, q0), s1 = fma(q3, r2, q2), s2 = fma(q5, r2, q4);
  const double Q = fma(s2, r8, fma(s1, r4, s0));
  const double p = 1.0 + fma(r2, Q, r);
  const int k = static_cast<int>(fmin(fmax(kd, -2000.0), 2000.0));
  double res = __builtin_ldexp(p, k);
  res = x > 0x1.62e42fefa39efp+9 ? __longlong_as_double(0x7ff0000000000000LL) : res;
  res = x < -0x1.74910d52d3051p+9 ? 0.0 : res;
  return x == x ? res : x;
}

// Branch-free like dexp: special inputs (NaN, negative, 0, +inf) selected at
// the end.
__device__ inline double dlog(double x0) {
  const bool sub = x0 < 0x1p-1022;
  const double x = sub ? x0 * 0x1p+54 : x0;
  const long long bits = __double_as_longlong(x);
  int e = static_cast<int>((bits >> 52) & 0x7ff) - 1023 - (sub ? 54 : 0);
  double f = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3ff0000000000000LL);
  const bool big = f > 0x1.6a09e667f3bcdp+0;
  f = big ? f * 0.5 : f;
  e += big ? 1 : 0;
  const double s = (f - 1.0) / (f + 1.0);
  const double z = s * s;
  // 2 atanh(s) = 2 (s + s z P(z)), P(z) = sum_{i=1}^{11} z^{i-1} / (2i+1) by
  // Estrin's scheme (adjacent pairs, then powers z^2, z^4, z^8)
  const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4;
  const double q0 = fma(InvOdd<2>::value, z, InvOdd<1>::value);
  const double q1 = fma(InvOdd<4>::value, z, InvOdd<3>::value);
  const double q2 = fma(InvOdd<6>::value, z, InvOdd<5>::value);
  const double q3 = fma(InvOdd<8>::value, z, InvOdd<7>::value);
  const double q4 = fma(InvOdd<10>::value, z, InvOdd<9>::value);
  const double s0 = fma(q1, z2, q0), s1 = fma(q3, z2, q2), s2 = fma(InvOdd<11>::value, z2, q4);
  const double P = fma(s2, z8, fma(s1, z4, s0));
  double t = fma(s * z, P, s);
  t = t + t;
  const double ed = static_cast<double>(e);
  double res = ed * kLn2Head + (ed * kLn2Tail + t);
  res = x0 == __longlong_as_double(0x7ff0000000000000LL) ? x0 : res;
  res = x0 == 0.0 ? -__longlong_as_double(0x7ff0000000000000LL) : res;
  return (x0 == x0 && x0 >= 0.0) ? res : __longlong_as_double(0x7ff8000000000000LL);
}

__device__ inline void cossin_2pi(double v, double& c, double& s) {
  const double q = rint(v * 4.0);
  const double th = (v - q * 0.25) * kTwoPi;
  const double z = th * th;
  // sin th = th sum_{i=0}^{9} (-1)^i z^i / (2i+1)!,  cos th = sum_{i=0}^{10} (-1)^i z^i / (2i)!,
  // both by Estrin's scheme
  const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4;
  const double a0 = fma(-InvFact<3>::value, z, 1.0);
  const double a1 = fma(-InvFact<7>::value, z, InvFact<5>::value);
  const double a2 = fma(-InvFact<11>::value, z, InvFact<9>::value);
  const double a3 = fma(-InvFact<15>::value, z, InvFact<13>::value);
  const double a4 = fma(-InvFact<19>::value, z, InvFact<17>::value);
  const double b0 = fma(a1, z2, a0), b1 = fma(a3, z2, a2);
  const double ps = fma(a4, z8, fma(b1, z4, b0));
  const double sn = th * ps;
  const double g0 = fma(-InvFact<2>::value, z, 1.0);
  const double g1 = fma(-InvFact<6>::value, z, InvFact<4>::value);
  const double g2 = fma(-InvFact<10>::value, z, InvFact<8>::value);
  const double g3 = fma(-InvFact<14>::value, z, InvFact<12>::value);
  const double g4 = fma(-InvFact<18>::value, z, InvFact<16>::value);
  const double h0 = fma(g1, z2, g0), h1 = fma(g3, z2, g2), h2 = fma(InvFact<20>::value, z2, g4);
  const double pc = fma(h2, z8, fma(h1, z4, h0));
  const int quad = static_cast<int>(q) & 3;
  const double a = (quad & 1) ? -sn : pc;   // cos(th + quad pi/2) for quad 0, 1
  const double b = (quad & 1) ? pc : sn;    // sin(th + quad pi/2) for quad 0, 1
  c = (quad & 2) ? -a : a;
  s = (quad & 2) ? -b : b;
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& z0, double& z1) {
  const double u1 = (static_cast<double>(wa) + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * dlog(u1));
  double c, s;
  cossin_2pi(static_cast<double>(wb) * 0x1p-32, c, s);
  z0 = r * c;
  z1 = r * s;
}

// normals 4g .. 4g+3 of (step, island)
__device__ __forceinline__ void normals4(Key key, uint32_t g, uint32_t island, uint32_t step, double z[4]) {
  uint32_t w[4];
  draw4(key, g, island, step, kTagNormal, 0, w);
  box_muller(w[0], w[1], z[0], z[1]);
  box_muller(w[2], w[3], z[2], z[3]);
}

// ---------------------------------------------------------------- binary32
// The same functions for binary32 particles, every operation a correctly
// rounded single-precision one (fmaf, +, *, /, sqrtf, rintf): Cody-Waite
// with a 15-bit ln 2 head (k ln2_head exact) and e^r = 1 + (r + r^2 Q(r)),
// Q of degree 5 (1/2! .. 1/7!); results below 2^-126 are 0 and the scaling
// 2^k is exact (k in [-125, 127]); log by 2 atanh(s) to s^9; sin to th^9 and
// cos to th^10 after the quarter-turn reduction.  Coefficients are the
// double tables above rounded once to binary32 (each equals the correctly
// rounded binary32 value of its rational).

constexpr float kLn2HeadF = 0x1.62e400p-1f;    // 15 significant bits
constexpr float kLn2TailF = 0x1.7f7d1cp-20f;   // ln 2 - head, rounded
constexpr float kInvLn2F = 0x1.715476p+0f;
constexpr float kTwoPiF = 0x1.921fb6p+2f;
template <int K> struct InvFactF { static constexpr float value = static_cast<float>(kCoeff.inv_fact[K]); };
template <int I> struct InvOddF { static constexpr float value = static_cast<float>(kCoeff.inv_odd[I]); };

__device__ inline float fexp(float x) {
  const float kf = rintf(x * kInvLn2F);
  const float r = fmaf(-kf, kLn2TailF, fmaf(-kf, kLn2HeadF, x));
  const float r2 = r * r, r4 = r2 * r2;
  const float q0 = fmaf(InvFactF<3>::value, r, InvFactF<2>::value);
  const float q1 = fmaf(InvFactF<5>::value, r, InvFactF<4>::value);
  const float q2 = fmaf(InvFactF<7>::value, r, InvFactF<6>::value);
  const float Q = fmaf(q2, r4, fmaf(q1, r2, q0));
  const float p = 1.0f + fmaf(r2, Q, r);
  const int k = static_cast<int>(fminf(fmaxf(kf, -200.0f), 200.0f));
  float res = __builtin_ldexpf(p, k);              // exact where it is kept
  res = kf > 127.0f ? __uint_as_float(0x7f800000u) : res;
  res = kf < -125.0f ? 0.0f : res;
  return x == x ? res : x;
}

__device__ inline float flog(float x0) {
  const bool sub = x0 < 0x1p-126f;
  const float x = sub ? x0 * 0x1p+24f : x0;
  const uint32_t bits = __float_as_uint(x);
  int e = static_cast<int>((bits >> 23) & 0xff) - 127 - (sub ? 24 : 0);
  float f = __uint_as_float((bits & 0x007fffffu) | 0x3f800000u);
  const bool big = f > 0x1.6a09e6p+0f;
  f = big ? f * 0.5f : f;
  e += big ? 1 : 0;
  const float s = (f - 1.0f) / (f + 1.0f);
  const float z = s * s;
  // 2 atanh(s) = 2 (s + s z P(z)), P(z) = 1/3 + z/5 + z^2/7 + z^3/9
  const float P = fmaf(fmaf(InvOddF<4>::value, z, InvOddF<3>::value), z * z,
                       fmaf(InvOddF<2>::value, z, InvOddF<1>::value));
  float t = fmaf(s * z, P, s);
  t = t + t;
  const float ef = static_cast<float>(e);
  float res = ef * kLn2HeadF + (ef * kLn2TailF + t);
  res = x0 == __uint_as_float(0x7f800000u) ? x0 : res;
  res = x0 == 0.0f ? __uint_as_float(0xff800000u) : res;
  return (x0 == x0 && x0 >= 0.0f) ? res : __uint_as_float(0x7fc00000u);
}

__device__ inline void fcossin_2pi(float v, float& c, float& s) {
  const float q = rintf(v * 4.0f);
  const float th = (v - q * 0.25f) * kTwoPiF;
  const float z = th * th, z2 = z * z;
  const float a0 = fmaf(-InvFactF<3>::value, z, 1.0f);
  const float a1 = fmaf(-InvFactF<7>::value, z, InvFactF<5>::value);
  const float sn = th * fmaf(fmaf(InvFactF<9>::value, z2, a1), z2, a0);
  const float g0 = fmaf(-InvFactF<2>::value, z, 1.0f);
  const float g1 = fmaf(-InvFactF<6>::value, z, InvFactF<4>::value);
  const float g2 = fmaf(-InvFactF<10>::value, z, InvFactF<8>::value);
  const float pc = fmaf(fmaf(g2, z2, g1), z2, g0);
  const int quad = static_cast<int>(q) & 3;
  const float a = (quad & 1) ? -sn : pc;
  const float b = (quad & 1) ? pc : sn;
  c = (quad & 2) ? -a : a;
  s = (quad & 2) ? -b : b;
}

// Box-Muller in binary32 on the same two words: u1 = fmaf((float)wa, 2^-32,
// 2^-33) in [2^-33, 1], v = (float)wb 2^-32 (the conversions round to
// nearest even)
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const float u1 = fmaf(static_cast<float>(wa), 0x1p-32f, 0x1p-33f);
  const float r = sqrtf(-2.0f * flog(u1));
  float c, s;
  fcossin_2pi(static_cast<float>(wb) * 0x1p-32f, c, s);
  z0 = r * c;
  z1 = r * s;
}

// normals 4g .. 4g+3 of (step, island) in binary32 arithmetic
__device__ __forceinline__ void normals4(Key key, uint32_t g, uint32_t island, uint32_t step, float z[4]) {
  uint32_t w[4];
  draw4(key, g, island, step, kTagNormal, 0, w);
  box_muller(w[0], w[1], z[0], z[1]);
  box_muller(w[2], w[3], z[2], z[3]);
}

// exp in the particles' precision
__device__ __forceinline__ double rexp(double x) { return dexp(x); }
__device__ __forceinline__ float rexp(float x) { return fexp(x); }

__device__ __forceinline__ uint64_t fmix64(uint64_t h) {
  h ^= h >> 33; h *= 0xff51afd7ed558ccdULL;
  h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ULL;
  h ^= h >> 33;
  return h;
}

// digest term of value v at (step, island, slot); slot 4095 tags island maps
__device__ __forceinline__ uint64_t digest_term(uint64_t step, uint64_t island, uint64_t slot, uint64_t v) {
  return fmix64(fmix64((step << 28) ^ (island << 12) ^ slot) ^ v);
}

}  // namespace airpf
