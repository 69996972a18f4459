/* AIRPF CPU oracle -- model interface.  TEST INFRASTRUCTURE ONLY (see orc.h). */
#ifndef ORC_MODELS_H
#define ORC_MODELS_H
#include "orc.h"

typedef struct {
  int kind, dx, dy, P, f32;
  double th[ORC_MAX_P];
  /* binary32 runs: every parameter and derived constant rounded to binary32
     once (derived constants computed in double first) */
  float thf[ORC_MAX_P], Hf[ORC_MAX_DX * ORC_MAX_DY];
  float s0f, sqf, sp0f, hrf, isyf;
  double c_log;                 /* additive constant of log g per step     */
  double s0;                    /* SV: stationary sd                       */
  double q, r, p0, sq, sp0, hr; /* LGD noise scales                        */
  double H[ORC_MAX_DX * ORC_MAX_DY];
  double log3;                  /* BIN                                     */
  int ab[2];                    /* BCP: integer Beta shapes (alpha, beta)  */
} orc_model;

void orc_model_setup(orc_model* M, const orc_problem* P, int f32);
int orc_model_noise_dim(const orc_model* M);
void orc_model_noise(const orc_model* M, uint64_t seed, int64_t n, int32_t k,
                     int32_t N, double* z);
void orc_model_init(const orc_model* M, const double* z, double* x);
void orc_model_prop(const orc_model* M, const double* xp, const double* z, double* x);
double orc_model_logpot(const orc_model* M, const double* x, const double* y);
void orc_model_quantise(const orc_model* M, const double* lw, int32_t N, uint64_t* q, double* mx);
void orc_model_init_tangent(const orc_model* M, const double* z, double* dx0);
void orc_model_prop_tangent(const orc_model* M, const double* xp, const double* dxp,
                            const double* z, double* dx);
void orc_model_logpot_tangent(const orc_model* M, const double* x, const double* dx,
                              const double* y, double* dlw);
#endif
