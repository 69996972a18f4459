/*
 * AIRPF CPU oracle -- a textbook bootstrap particle filter (Gordon, Salmond
 * and Smith 1993), kept apart from orc_airpf.c on purpose.  Section 2 notes
 * that AIRPF with m = 1 is a single BPF, and with interactions switched off
 * (tau <= 1/m) it is m independent BPFs (IBPF, Section 3); the tests check
 * the AIRPF code against this one on the same random draws.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * It reads the same draws (island label k in the counter) and the same
 * fixed-point weights, but counts offspring per particle instead of
 * searching ancestors per slot: particle i gets every slot j with
 * M C_{i-1} <= U + j Q < M C_i, i.e. j in [ceil((M C_{i-1} - U)/Q),
 * ceil((M C_i - U)/Q)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"
#include "orc_models.h"

/* #{j >= 0 : U + j Q < B} for B >= 0 */
static int64_t slots_below(uint64_t B, uint64_t U, uint64_t Q) {
  if (B <= U) return 0;
  return (int64_t)((B - U + Q - 1) / Q);
}

double orc_bpf_run(const orc_problem* P, int32_t k, int32_t f32, int32_t* anc_out) {
  if (P->N < 1 || P->N > 2048 || P->T < 1 || P->dx < 1 || P->dx > ORC_MAX_DX ||
      P->dy < 1 || P->dy > ORC_MAX_DY)
    return NAN;
  const int32_t N = P->N, dx = P->dx, dy = P->dy;
  orc_model Mo;
  orc_model_setup(&Mo, P, f32);
  const int nd = orc_model_noise_dim(&Mo);
  double* x = malloc(sizeof(double) * N * dx);
  double* xn = malloc(sizeof(double) * N * dx);
  double* lw = malloc(sizeof(double) * N);
  uint64_t* q = malloc(sizeof(uint64_t) * N);
  int32_t* a = malloc(sizeof(int32_t) * N);
  double* z = malloc(sizeof(double) * N * nd);
  orc_model_noise(&Mo, P->seed, 0, k, N, z);
  for (int32_t j = 0; j < N; ++j) orc_model_init(&Mo, z + j * nd, x + j * dx);
  double ll = 0.0;
  const double cst = Mo.c_log - 40.0 * log(2.0) - log((double)N);
  for (int64_t n = 0; n < P->T; ++n) {
    for (int32_t j = 0; j < N; ++j) {
      double v = orc_model_logpot(&Mo, x + j * dx, P->y + n * dy);
      if (v != v) v = -INFINITY;
      lw[j] = v;
    }
    double mx;
    orc_model_quantise(&Mo, lw, N, q, &mx);
    uint64_t Q = 0;
    for (int32_t j = 0; j < N; ++j) Q += q[j];
    if (Q == 0) { ll = -INFINITY; break; }
    ll = ll + ((mx + orc_log((double)Q)) + cst);
    if (n == P->T - 1) break;
    const uint64_t U = orc_bounded(P->seed, 0, (uint32_t)k, (uint32_t)n, TAG_SYS, Q);
    uint64_t Cprev = 0;
    for (int32_t i = 0; i < N; ++i) {
      const uint64_t C = Cprev + q[i];
      const int64_t lo = slots_below((uint64_t)N * Cprev, U, Q);
      int64_t hi = slots_below((uint64_t)N * C, U, Q);
      if (hi > N) hi = N;
      for (int64_t j = lo; j < hi; ++j) a[j] = i;
      Cprev = C;
    }
    if (anc_out) memcpy(anc_out + n * N, a, sizeof(int32_t) * N);
    orc_model_noise(&Mo, P->seed, n + 1, k, N, z);
    for (int32_t j = 0; j < N; ++j) orc_model_prop(&Mo, x + a[j] * dx, z + j * nd, xn + j * dx);
    double* t = x; x = xn; xn = t;
  }
  free(x); free(xn); free(lw); free(q); free(a); free(z);
  return ll;
}
