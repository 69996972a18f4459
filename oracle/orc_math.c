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
 *         Taylor polynomial of e^r by Horner's rule, scaling by 2^k.
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
  /* e^r = sum_{i=0}^{13} r^i / i!  (Horner) */
  double p = 0x1.6124613a86d09p-33;                    /* 1/13!              */
  p = fma(p, r, 0x1.1eed8eff8d898p-29);                /* 1/12!              */
  p = fma(p, r, 0x1.ae64567f544e4p-26);                /* 1/11!              */
  p = fma(p, r, 0x1.27e4fb7789f5cp-22);                /* 1/10!              */
  p = fma(p, r, 0x1.71de3a556c734p-19);                /* 1/9!               */
  p = fma(p, r, 0x1.a01a01a01a01ap-16);                /* 1/8!               */
  p = fma(p, r, 0x1.a01a01a01a01ap-13);                /* 1/7!               */
  p = fma(p, r, 0x1.6c16c16c16c17p-10);                /* 1/6!               */
  p = fma(p, r, 0x1.1111111111111p-7);                 /* 1/5!               */
  p = fma(p, r, 0x1.5555555555555p-5);                 /* 1/4!               */
  p = fma(p, r, 0x1.5555555555555p-3);                 /* 1/3!               */
  p = fma(p, r, 0x1.0000000000000p-1);                 /* 1/2!               */
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
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
  /* sum_{i=0}^{11} z^i / (2i+1)  (Horner) */
  double p = 0x1.642c8590b2164p-5;                     /* 1/23 */
  p = fma(p, z, 0x1.8618618618618p-5);                 /* 1/21 */
  p = fma(p, z, 0x1.af286bca1af28p-5);                 /* 1/19 */
  p = fma(p, z, 0x1.e1e1e1e1e1e1ep-5);                 /* 1/17 */
  p = fma(p, z, 0x1.1111111111111p-4);                 /* 1/15 */
  p = fma(p, z, 0x1.3b13b13b13b14p-4);                 /* 1/13 */
  p = fma(p, z, 0x1.745d1745d1746p-4);                 /* 1/11 */
  p = fma(p, z, 0x1.c71c71c71c71cp-4);                 /* 1/9  */
  p = fma(p, z, 0x1.2492492492492p-3);                 /* 1/7  */
  p = fma(p, z, 0x1.999999999999ap-3);                 /* 1/5  */
  p = fma(p, z, 0x1.5555555555555p-2);                 /* 1/3  */
  p = fma(p, z, 1.0);
  double t = s * p;
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
  /* sin th = th * sum_{i=0}^{9} (-1)^i z^i / (2i+1)! */
  double ps = -0x1.2f49b46814157p-57;
  ps = fma(ps, z, 0x1.952c77030ad4ap-49);
  ps = fma(ps, z, -0x1.ae7f3e733b81fp-41);
  ps = fma(ps, z, 0x1.6124613a86d09p-33);
  ps = fma(ps, z, -0x1.ae64567f544e4p-26);
  ps = fma(ps, z, 0x1.71de3a556c734p-19);
  ps = fma(ps, z, -0x1.a01a01a01a01ap-13);
  ps = fma(ps, z, 0x1.1111111111111p-7);
  ps = fma(ps, z, -0x1.5555555555555p-3);
  ps = fma(ps, z, 1.0);
  const double sn = th * ps;
  /* cos th = sum_{i=0}^{10} (-1)^i z^i / (2i)! */
  double pc = 0x1.e542ba4020225p-62;
  pc = fma(pc, z, -0x1.6827863b97d97p-53);
  pc = fma(pc, z, 0x1.ae7f3e733b81fp-45);
  pc = fma(pc, z, -0x1.93974a8c07c9dp-37);
  pc = fma(pc, z, 0x1.1eed8eff8d898p-29);
  pc = fma(pc, z, -0x1.27e4fb7789f5cp-22);
  pc = fma(pc, z, 0x1.a01a01a01a01ap-16);
  pc = fma(pc, z, -0x1.6c16c16c16c17p-10);
  pc = fma(pc, z, 0x1.5555555555555p-5);
  pc = fma(pc, z, -0x1.0000000000000p-1);
  pc = fma(pc, z, 1.0);
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
