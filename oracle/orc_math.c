/*
 * AIRPF CPU oracle -- own double-precision exp, log and (cos, sin)(2 pi v).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Why these exist: ancestor indices and island pairings are integers decided
 * by floating point (the fixed-point weights and the pair-selection
 * probability).  For the GPU library and this oracle to take every such
 * decision identically, both evaluate the elementary functions with the same
 * sequence of correctly rounded IEEE-754 operations (+, -, *, /, sqrt, fma,
 * rint) instead of each platform's libm.  The methods are textbook:
 *   exp : Cody-Waite reduction x = k ln2 + r (two-part ln2), degree-13
 *         Taylor polynomial of e^r by Estrin's scheme, scaling by 2^k.
 *   log : x = 2^e f, f in [sqrt(2)/2, sqrt(2)], log f = 2 atanh(s) with
 *         s = (f-1)/(f+1), odd series in s to s^23.
 *   cos/sin(2 pi v): quadrant q = rint(4v), w = v - q/4 in [-1/8, 1/8],
 *         Taylor series of sin/cos at theta = 2 pi w, quadrant rotation.
 * Accuracy (checked in the tests against libm): a few ulp.
 *
 * This file must be compiled with -ffp-contract=off: every fused
 * multiply-add below is an explicit fma().
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include "orc.h"

static double bits_to_double(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t double_to_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }

/* 2^k as a double for -1022 <= k <= 1023 */
static double pow2i(int k) { return bits_to_double((uint64_t)(k + 1023) << 52); }

double orc_exp(double x) {
  if (x != x) return x;
  if (x > 0x1.62e42fefa39efp+9) return INFINITY;       /* > ln(DBL_MAX)      */
  if (x < -0x1.74910d52d3051p+9) return 0.0;           /* < ln(2^-1074) - .. */
  const double kd = rint(x * 0x1.71547652b82fep+0);    /* x / ln 2           */
  double r = fma(-kd, 0x1.62e42fee00000p-1, x);        /* ln2 high part      */
  r = fma(-kd, 0x1.a39ef35793c76p-33, r);              /* ln2 low part       */
  /* e^r = 1 + (r + r^2 Q(r)),  Q(r) = sum_{i=2}^{13} r^{i-2} / i!
     (Estrin: adjacent pairs in r, then combined with r^2, r^4, r^8; the
     leading 1 added last) */
  const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  const double q0 = fma(0x1.5555555555555p-3, r, 0x1.0000000000000p-1);   /* 1/3!, 1/2!   */
  const double q1 = fma(0x1.1111111111111p-7, r, 0x1.5555555555555p-5);   /* 1/5!, 1/4!   */
  const double q2 = fma(0x1.a01a01a01a01ap-13, r, 0x1.6c16c16c16c17p-10); /* 1/7!, 1/6!   */
  const double q3 = fma(0x1.71de3a556c734p-19, r, 0x1.a01a01a01a01ap-16); /* 1/9!, 1/8!   */
  const double q4 = fma(0x1.ae64567f544e4p-26, r, 0x1.27e4fb7789f5cp-22); /* 1/11!, 1/10! */
  const double q5 = fma(0x1.6124613a86d09p-33, r, 0x1.1eed8eff8d898p-29); /* 1/13!, 1/12! */
  const double s0 = fma(q1, r2, q0), s1 = fma(q3, r2, q2), s2 = fma(q5, r2, q4);
  const double Q = fma(s2, r8, fma(s1, r4, s0));
  const double p = 1.0 + fma(r2, Q, r);
  const int k = (int)kd;
  if (k > 1023) return (p * 2.0) * pow2i(k - 1);
  if (k < -1022) return (p * pow2i(k + 200)) * pow2i(-200);
  return p * pow2i(k);
}

double orc_log(double x) {
  if (x != x || x < 0.0) return NAN;
  if (x == 0.0) return -INFINITY;
  if (x == INFINITY) return INFINITY;
  int e = 0;
  if (x < 0x1p-1022) { x = x * 0x1p+54; e = -54; }     /* subnormal input    */
  uint64_t b = double_to_bits(x);
  e += (int)((b >> 52) & 0x7ff) - 1023;
  double f = bits_to_double((b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL);
  if (f > 0x1.6a09e667f3bcdp+0) { f = f * 0.5; e += 1; } /* f > sqrt(2)      */
  const double s = (f - 1.0) / (f + 1.0);
  const double z = s * s;
  /* 2 atanh(s) = 2 (s + s z P(z)),  P(z) = sum_{i=1}^{11} z^{i-1} / (2i+1)
     (Estrin: adjacent pairs in z, then combined with z^2, z^4, z^8) */
  const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4;
  const double q0 = fma(0x1.999999999999ap-3, z, 0x1.5555555555555p-2);   /* 1/5, 1/3     */
  const double q1 = fma(0x1.c71c71c71c71cp-4, z, 0x1.2492492492492p-3);   /* 1/9, 1/7     */
  const double q2 = fma(0x1.3b13b13b13b14p-4, z, 0x1.745d1745d1746p-4);   /* 1/13, 1/11   */
  const double q3 = fma(0x1.e1e1e1e1e1e1ep-5, z, 0x1.1111111111111p-4);   /* 1/17, 1/15   */
  const double q4 = fma(0x1.8618618618618p-5, z, 0x1.af286bca1af28p-5);   /* 1/21, 1/19   */
  const double s0 = fma(q1, z2, q0), s1 = fma(q3, z2, q2);
  const double s2 = fma(0x1.642c8590b2164p-5, z2, q4);                    /* 1/23         */
  const double P = fma(s2, z8, fma(s1, z4, s0));
  double t = fma(s * z, P, s);
  t = t + t;                                           /* 2 atanh(s)         */
  const double ed = (double)e;
  const double hi = ed * 0x1.62e42fee00000p-1;         /* exact              */
  const double lo = ed * 0x1.a39ef35793c76p-33;
  return hi + (lo + t);
}

void orc_cossin2pi(double v, double* c, double* s) {
  const double q = rint(v * 4.0);
  const double w = v - q * 0.25;                       /* |w| <= 1/8         */
  const double th = w * 0x1.921fb54442d18p+2;          /* 2 pi w             */
  const double z = th * th;
  /* sin th = th * sum_{i=0}^{9} (-1)^i z^i / (2i+1)!  and
     cos th = sum_{i=0}^{10} (-1)^i z^i / (2i)!, both by Estrin */
  const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4;
  const double a0 = fma(-0x1.5555555555555p-3, z, 1.0);                   /* -1/3!        */
  const double a1 = fma(-0x1.a01a01a01a01ap-13, z, 0x1.1111111111111p-7); /* -1/7!, 1/5!  */
  const double a2 = fma(-0x1.ae64567f544e4p-26, z, 0x1.71de3a556c734p-19); /* -1/11!, 1/9! */
  const double a3 = fma(-0x1.ae7f3e733b81fp-41, z, 0x1.6124613a86d09p-33); /* -1/15!, 1/13! */
  const double a4 = fma(-0x1.2f49b46814157p-57, z, 0x1.952c77030ad4ap-49); /* -1/19!, 1/17! */
  const double b0 = fma(a1, z2, a0), b1 = fma(a3, z2, a2);
  const double ps = fma(a4, z8, fma(b1, z4, b0));
  const double sn = th * ps;
  const double g0 = fma(-0x1.0000000000000p-1, z, 1.0);                   /* -1/2!        */
  const double g1 = fma(-0x1.6c16c16c16c17p-10, z, 0x1.5555555555555p-5); /* -1/6!, 1/4!  */
  const double g2 = fma(-0x1.27e4fb7789f5cp-22, z, 0x1.a01a01a01a01ap-16); /* -1/10!, 1/8! */
  const double g3 = fma(-0x1.93974a8c07c9dp-37, z, 0x1.1eed8eff8d898p-29); /* -1/14!, 1/12! */
  const double g4 = fma(-0x1.6827863b97d97p-53, z, 0x1.ae7f3e733b81fp-45); /* -1/18!, 1/16! */
  const double h0 = fma(g1, z2, g0), h1 = fma(g3, z2, g2);
  const double h2 = fma(0x1.e542ba4020225p-62, z2, g4);                   /* 1/20!        */
  const double pc = fma(h2, z8, fma(h1, z4, h0));
  const double cs = pc;
  /* angle = th + q pi/2 */
  const int quad = ((int)q) & 3;
  switch (quad) {
    case 0: *c = cs;  *s = sn;  break;
    case 1: *c = -sn; *s = cs;  break;
    case 2: *c = -cs; *s = -sn; break;
    default: *c = sn; *s = -cs; break;
  }
}

/* Box-Muller (Box & Muller 1958): two 32-bit words -> two N(0,1) values.
 * u1 = (wa + 1/2) 2^-32 in (0,1), v = wb 2^-32 in [0,1),
 * r = sqrt(-2 log u1), (z0, z1) = (r cos 2 pi v, r sin 2 pi v). */
void orc_boxmuller(uint32_t wa, uint32_t wb, double* z0, double* z1) {
  const double u1 = ((double)wa + 0.5) * 0x1p-32;
  const double v = (double)wb * 0x1p-32;
  const double r = sqrt(-2.0 * orc_log(u1));
  double c, s;
  orc_cossin2pi(v, &c, &s);
  *z0 = r * c;
  *z1 = r * s;
}

/* ------------------------------------------------------------------------
 * Binary32 counterparts, for runs whose particle arithmetic is single
 * precision (state, normals, model, weights).  Same methods with the
 * polynomials cut to single-precision accuracy, every operation a correctly
 * rounded IEEE binary32 +, -, *, /, sqrt, fmaf or rintf:
 *   expf : Cody-Waite with a 15-bit ln2 head (k ln2_hi exact for |k| < 512),
 *          e^r = 1 + (r + r^2 Q(r)), Q of degree 5 (1/2! .. 1/7!) by
 *          Estrin; the scaling 2^k is exact because results below 2^-126
 *          are returned as 0 (k < -125) and k > 127 overflows to +inf.
 *   logf : x = 2^e f, f in [sqrt(2)/2, sqrt(2)], 2 atanh(s) to s^9.
 *   cos/sin(2 pi v): quarter-turn reduction, sin to th^9, cos to th^10.
 * Box-Muller: u1 = fmaf((float)wa, 2^-32, 2^-33), v = (float)wb 2^-32
 * ((float) of a 32-bit word rounds to nearest even), r = sqrtf(-2 logf u1).
 * Accuracy against libm: within a couple of binary32 ulp (tests).
 * ------------------------------------------------------------------------ */

static float bits_to_float(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t float_to_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

float orc_expf(float x) {
  if (x != x) return x;
  const float kf = rintf(x * 0x1.715476p+0f);          /* x / ln 2           */
  float r = fmaf(-kf, 0x1.62e400p-1f, x);              /* ln2 head, 15 bits  */
  r = fmaf(-kf, 0x1.7f7d1cp-20f, r);                   /* ln2 tail           */
  const float r2 = r * r, r4 = r2 * r2;
  const float q0 = fmaf(0x1.555556p-3f, r, 0x1.000000p-1f);    /* 1/3!, 1/2! */
  const float q1 = fmaf(0x1.111112p-7f, r, 0x1.555556p-5f);    /* 1/5!, 1/4! */
  const float q2 = fmaf(0x1.a01a02p-13f, r, 0x1.6c16c2p-10f);  /* 1/7!, 1/6! */
  const float Q = fmaf(q2, r4, fmaf(q1, r2, q0));
  const float p = 1.0f + fmaf(r2, Q, r);
  if (kf > 127.0f) return INFINITY;
  if (kf < -125.0f) return 0.0f;
  return ldexpf(p, (int)kf);                           /* exact: normal range */
}

float orc_logf(float x) {
  if (x != x || x < 0.0f) return NAN;
  if (x == 0.0f) return -INFINITY;
  if (x == INFINITY) return INFINITY;
  int e = 0;
  if (x < 0x1p-126f) { x = x * 0x1p+24f; e = -24; }    /* subnormal input    */
  const uint32_t b = float_to_bits(x);
  e += (int)((b >> 23) & 0xff) - 127;
  float f = bits_to_float((b & 0x007fffffu) | 0x3f800000u);
  if (f > 0x1.6a09e6p+0f) { f = f * 0.5f; e += 1; }     /* f > sqrt(2)        */
  const float s = (f - 1.0f) / (f + 1.0f);
  const float z = s * s;
  /* 2 atanh(s) = 2 (s + s z P(z)), P(z) = 1/3 + z/5 + z^2/7 + z^3/9 (Estrin) */
  const float P = fmaf(fmaf(0x1.c71c72p-4f, z, 0x1.24924ap-3f), z * z,
                       fmaf(0x1.99999ap-3f, z, 0x1.555556p-2f));
  float t = fmaf(s * z, P, s);
  t = t + t;
  const float ef = (float)e;
  const float hi = ef * 0x1.62e400p-1f;                /* exact              */
  const float lo = ef * 0x1.7f7d1cp-20f;
  return hi + (lo + t);
}

void orc_cossin2pif(float v, float* c, float* s) {
  const float q = rintf(v * 4.0f);
  const float w = v - q * 0.25f;                       /* exact, |w| <= 1/8  */
  const float th = w * 0x1.921fb6p+2f;                 /* 2 pi w             */
  const float z = th * th, z2 = z * z;
  /* sin th = th (1 - z/3! + z^2/5! - z^3/7! + z^4/9!),
     cos th = 1 - z/2! + z^2/4! - z^3/6! + z^4/8! - z^5/10! (Estrin) */
  const float a0 = fmaf(-0x1.555556p-3f, z, 1.0f);                     /* -1/3!       */
  const float a1 = fmaf(-0x1.a01a02p-13f, z, 0x1.111112p-7f);          /* -1/7!, 1/5! */
  const float ps = fmaf(fmaf(0x1.71de3ap-19f, z2, a1), z2, a0);        /* 1/9!        */
  const float sn = th * ps;
  const float g0 = fmaf(-0x1.000000p-1f, z, 1.0f);                     /* -1/2!       */
  const float g1 = fmaf(-0x1.6c16c2p-10f, z, 0x1.555556p-5f);          /* -1/6!, 1/4! */
  const float g2 = fmaf(-0x1.27e4fcp-22f, z, 0x1.a01a02p-16f);         /* -1/10!, 1/8! */
  const float cs = fmaf(fmaf(g2, z2, g1), z2, g0);
  const int quad = ((int)q) & 3;
  switch (quad) {
    case 0: *c = cs;  *s = sn;  break;
    case 1: *c = -sn; *s = cs;  break;
    case 2: *c = -cs; *s = -sn; break;
    default: *c = sn; *s = -cs; break;
  }
}

void orc_boxmullerf(uint32_t wa, uint32_t wb, float* z0, float* z1) {
  const float u1 = fmaf((float)wa, 0x1p-32f, 0x1p-33f);   /* in [2^-33, 1]  */
  const float v = (float)wb * 0x1p-32f;                   /* in [0, 1]      */
  const float r = sqrtf(-2.0f * orc_logf(u1));
  float c, s;
  orc_cossin2pif(v, &c, &s);
  *z0 = r * c;
  *z1 = r * s;
}
