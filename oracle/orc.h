/*
 * AIRPF CPU oracle -- internal header.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing under oracle/ is part of the product
 * path: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the HIP library; both sides
 * are written independently from the same written contract (Philox counter
 * layout, own double-precision exp/log/sincos, fixed-point resampling rule,
 * island-decision rule), which is restated in the comments below.
 *
 * Paper: K. Heine, "Augmented Island Resampling Particle Filters for Particle
 * Markov Chain Monte Carlo" (arXiv:2312.06484).  The filter itself is
 * Algorithm 1 of Section 2; the marginal-likelihood estimate is the
 * gamma^N_n(1) definition that follows it.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

enum { ORC_LG1 = 0, ORC_SV = 1, ORC_LGD = 2, ORC_BIN = 3, ORC_BCP = 4 };
enum { TAG_NORMAL = 1, TAG_SYS = 2, TAG_MULT = 3, TAG_ISL = 4, TAG_BIN = 5, TAG_BCP = 6 };
#define ORC_MAX_DX 8
#define ORC_MAX_DY 8
#define ORC_MAX_P 64

typedef struct {
  int32_t kind, dx, dy, d_theta;
  const double* theta;   /* d_theta values                                  */
  const double* consts;  /* LGD: q, r, p0, H[dy*dx] row-major; else unused   */
  const double* y;       /* T*dy observations, row-major                     */
  int64_t T;
  int32_t m, N;          /* m islands (power of two), N particles per island */
  uint64_t seed;
} orc_problem;

typedef struct {
  double tau;            /* ENF threshold; <= 1/m never interacts           */
  int32_t scheme;        /* 0 systematic, 1 multinomial                     */
  int32_t f32;           /* 1: binary32 particles: state, normals, model and
                            weights in single precision (island log-weights
                            and log Zhat stay double)                        */
  int32_t replay;        /* 1: ancestors, island maps, stage counts read
                            from the trace instead of being drawn            */
  int32_t exact_weights; /* 1: island weights from the unquantised sum       */
  double ess_frac;       /* 0: every island resamples internally at every
                            step.  rho > 0: adaptive internal resampling, an
                            island resamples iff its ESS < rho N (ESS from the
                            fixed-point weights truncated to 20 bits), else
                            its particles keep their weights                 */
  int32_t arity;         /* r of the interactions, m = r^(S_r): 0 or 2 the
                            pairs of Algorithm 1; 4, 8, ... (powers of two)
                            groups of r islands per stage                     */
} orc_opts;

typedef struct {
  int32_t* sstar;        /* [T]          interacting stages per step         */
  double* enf;           /* [T*(S+1)]    ENF_{n,s}, NaN when not evaluated   */
  double* lpost;         /* [T*m]        island log-weights after weighting  */
  int32_t* anc;          /* [T*m*N]      within-island ancestors             */
  int32_t* pi;           /* [T*m]        composite island source map         */
  uint64_t* digest;      /* [2*T]        ancestor / island-map digests       */
  double* x;             /* [T*m*N*dx]   state entering each weighting       */
  double* logz_inc;      /* [T]          log Zhat_{n+1} - log Zhat_n         */
  double* fmean;         /* [T*m]        island k's weighted mean of the first
                            state coordinate after the weighting:
                            sum_i q_i x_i / Q, summed in particle order     */
  double* lpre;          /* [T*m]        island log-weights entering each
                            weighting (after the previous step's stages)     */
} orc_trace;

/* ---- counter-based RNG (orc_rng.c) ---- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
              uint32_t tag, uint32_t sub, uint32_t w[4]);
double orc_u53(uint32_t hi, uint32_t lo);
uint64_t orc_bounded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t tag, uint64_t Q);
void orc_island_normals(uint64_t seed, int64_t n, int32_t k, int64_t count,
                        double* z);
void orc_island_normalsf(uint64_t seed, int64_t n, int32_t k, int64_t count,
                         double* z);

/* ---- own double-precision elementary functions (orc_math.c) ---- */
double orc_exp(double x);
double orc_log(double x);
void orc_cossin2pi(double v, double* c, double* s);
void orc_boxmuller(uint32_t wa, uint32_t wb, double* z0, double* z1);
/* binary32 counterparts (runs with single-precision particle arithmetic) */
float orc_expf(float x);
float orc_logf(float x);
void orc_cossin2pif(float v, float* c, float* s);
void orc_boxmullerf(uint32_t wa, uint32_t wb, float* z0, float* z1);

/* ---- fixed-point resampling (orc_airpf.c) ---- */
void orc_quantise(const double* lw, int32_t N, uint64_t* q, double* mx);
void orc_systematic(const uint64_t* q, int32_t N, uint64_t U, int32_t* anc);

uint64_t orc_fmix64(uint64_t h);
uint64_t orc_digest_term(int64_t n, int64_t k, int64_t j, int64_t v);

#endif
