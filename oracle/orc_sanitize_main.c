/*
 * Driver for the sanitised build of the AIRPF CPU oracle.
 * TEST INFRASTRUCTURE ONLY (see orc.h): tests/test_oracle_sanitized.py builds
 * the oracle's sources with this main under AddressSanitizer and
 * UndefinedBehaviorSanitizer (gcc, host code) and runs it; any out-of-bounds
 * access, leak, misaligned or overflowing operation in the manual indexing of
 * the oracle's m*N*dx*P arrays aborts the run.  Every entry point is
 * exercised over sizes that reach the edges of that indexing: one island,
 * one particle, ragged N, the largest N, a single observation, both
 * internal resampling schemes, both particle precisions, the 8-D model with
 * 64 score tangents, replay of a recorded genealogy, the bootstrap filter.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

double orc_airpf_run(const orc_problem* P, const orc_opts* O, orc_trace* tr);
double orc_airpf_score(const orc_problem* P, const orc_opts* O, orc_trace* tr, double* gpw, double* gps);
double orc_airpf_frozen(const orc_problem* P, const orc_opts* O, orc_trace* tr, double* fS, double* flw);
double orc_bpf_run(const orc_problem* P, int32_t k, int32_t f32, int32_t* anc_out);

static int fails = 0;

static void check(int ok, const char* what) {
  if (!ok) { fprintf(stderr, "FAILED: %s\n", what); ++fails; }
}

/* options the later cases set: r of the interactions, adaptive threshold */
static int g_arity = 2;
static double g_ess = 0.0;

static void case_run(int kind, int dx, int dy, int m, int N, int T, double tau, int scheme, int f32) {
  double theta[64], consts[3 + 64];
  int dth = 3;
  if (kind == ORC_LG1) { theta[0] = 0.9; theta[1] = 1.0; theta[2] = 1.0; }
  else if (kind == ORC_SV) { theta[0] = -1.0; theta[1] = 0.95; theta[2] = 0.3; }
  else if (kind == ORC_BIN) { theta[0] = 0.0; dth = 1; }
  else if (kind == ORC_BCP) { theta[0] = 0.1; dth = 1; consts[0] = 2.0; consts[1] = 5.0; }
  else {
    dth = dx * dx;
    for (int i = 0; i < dth; ++i) theta[i] = (i % (dx + 1) == 0) ? 0.5 : 0.05;
    consts[0] = 0.5; consts[1] = 1.0; consts[2] = 1.0;
    for (int i = 0; i < dx * dy; ++i) consts[3 + i] = 0.3 * ((i % 5) - 2);
  }
  double* y = malloc(sizeof(double) * (size_t)T * dy);
  for (int i = 0; i < T * dy; ++i) y[i] = kind == ORC_BIN ? (double)(i % 2) : sin(0.7 * i);
  if (kind == ORC_BCP)
    for (int i = 0; i < T; ++i) { y[2 * i] = (double)(i % 7); y[2 * i + 1] = 20.0; }
  orc_problem P = {kind, dx, dy, dth, theta, consts, y, T, m, N, 12345};
  orc_opts O = {tau, scheme, f32, 0, 0, g_ess, g_arity};
  const int S = (int)round(log2((double)m));
  const size_t mN = (size_t)m * N;
  orc_trace tr = {0};
  tr.sstar = calloc((size_t)T, sizeof(int32_t));
  tr.enf = calloc((size_t)T * (S + 1), sizeof(double));
  tr.lpost = calloc((size_t)T * m, sizeof(double));
  tr.anc = calloc((size_t)T * mN, sizeof(int32_t));
  tr.pi = calloc((size_t)T * m, sizeof(int32_t));
  tr.digest = calloc((size_t)2 * T, sizeof(uint64_t));
  tr.x = calloc((size_t)T * mN * dx, sizeof(double));
  tr.logz_inc = calloc((size_t)T, sizeof(double));
  tr.fmean = calloc((size_t)T * m, sizeof(double));
  tr.lpre = calloc((size_t)T * m, sizeof(double));
  const double lz = orc_airpf_run(&P, &O, &tr);
  check(lz == lz, "run returned NaN");
  if (kind != ORC_BIN && kind != ORC_BCP) {
    double gpw[64], gps[64];
    const double lz2 = orc_airpf_score(&P, &O, NULL, gpw, gps);
    check(lz2 == lz, "score's log Zhat differs from the run's");
    if (scheme == 0) {
      orc_opts R = O;
      R.replay = 1;
      double* fS = calloc(mN, sizeof(double));
      double* flw = calloc(mN, sizeof(double));
      const double F = orc_airpf_frozen(&P, &R, &tr, fS, flw);
      check(F == F, "frozen returned NaN");
      free(fS);
      free(flw);
    }
  }
  if (m == 1) {
    int32_t* anc = calloc((size_t)T * N, sizeof(int32_t));
    const double ll = orc_bpf_run(&P, 0, f32, anc);
    check(ll == ll, "bootstrap filter returned NaN");
    free(anc);
  }
  free(tr.sstar); free(tr.enf); free(tr.lpost); free(tr.anc); free(tr.pi); free(tr.digest);
  free(tr.x); free(tr.logz_inc); free(tr.fmean); free(tr.lpre); free(y);
}

int main(void) {
  const int kinds[3] = {ORC_LG1, ORC_SV, ORC_LGD};
  for (int f32 = 0; f32 <= 1; ++f32)
    for (int scheme = 0; scheme <= 1; ++scheme)
      for (int ki = 0; ki < 3; ++ki) {
        const int kind = kinds[ki];
        const int dx = kind == ORC_LGD ? 3 : 1, dy = kind == ORC_LGD ? 2 : 1;
        case_run(kind, dx, dy, 1, 1, 4, 0.3, scheme, f32);
        case_run(kind, dx, dy, 1, 37, 5, 0.3, scheme, f32);
        case_run(kind, dx, dy, 4, 1, 6, 2.0, scheme, f32);
        case_run(kind, dx, dy, 8, 33, 1, 0.3, scheme, f32);
        case_run(kind, dx, dy, 16, 5, 7, 0.7, scheme, f32);
        case_run(kind, dx, dy, 2, 2048, 2, 0.9, scheme, f32);
      }
  case_run(ORC_LGD, 8, 4, 4, 9, 3, 0.6, 0, 1);       /* 64 tangents of vec(A) */
  case_run(ORC_LGD, 8, 8, 2, 3, 2, 2.0, 1, 0);
  case_run(ORC_BIN, 1, 1, 4, 2, 5, 2.0, 1, 0);        /* the exact-variance toy */
  case_run(ORC_BIN, 1, 1, 1, 8, 5, 0.3, 0, 0);
  case_run(ORC_BCP, 2, 2, 8, 16, 12, 0.5, 0, 0);      /* Beta change points */
  case_run(ORC_BCP, 2, 2, 4, 5, 9, 2.0, 1, 0);
  g_ess = 0.6;                                         /* adaptive internal resampling */
  case_run(ORC_SV, 1, 1, 16, 37, 9, 0.7, 0, 0);
  case_run(ORC_LGD, 3, 2, 4, 6, 5, 2.0, 0, 1);
  g_ess = 0.0;
  g_arity = 4;                                         /* groups of four islands */
  case_run(ORC_LG1, 1, 1, 64, 7, 9, 0.9, 0, 0);
  case_run(ORC_LGD, 3, 2, 16, 5, 6, 2.0, 1, 1);
  g_arity = 16;
  case_run(ORC_SV, 1, 1, 256, 3, 5, 0.95, 0, 0);
  g_arity = 2;
  if (fails) return 1;
  printf("sanitised oracle run: ok\n");
  return 0;
}
