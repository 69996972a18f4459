/*
 * AIRPF CPU oracle -- Algorithm 1 (Section 2) run sequentially, step by step.
 * TEST INFRASTRUCTURE ONLY (see orc.h): loaded by the tests, the smoke check
 * and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * One filter step n, in the order of Algorithm 1:
 *   1. ENF_{n,0} of the island weights W_{n,0} (traced, not used).
 *   2. Island weighting ("marginal likelihood estimation" line):
 *        W^k_{n,1} = W^k_{n,0} M^-1 sum_i g_n(xi^{k,i}).
 *      In log form L_k += log(M^-1 sum_i g_n), evaluated on fixed-point
 *      weights: mx = max_i lw_i, q_i = floor(2^40 exp(lw_i - mx)),
 *      Q = sum_i q_i (exact, uint64),
 *        L_k += (mx + log Q) + (c - 40 log 2 - log M).
 *      The same q drive the internal resampling, so the filter is exactly the
 *      AIRPF of the (negligibly) quantised potential.
 *   3. log Zhat: gamma^N_n(1) = m^-1 sum_k W^k_{n,0}; the stages preserve
 *      sum_k W (the columns of every alpha sum to one, Theorem 1's proof),
 *      so log Zhat after the last weighting is logsumexp_k L_k - log m.
 *   4. Stop after the weighting of the last observation.
 *   5. Internal resampling of every island from its g-weighted empirical
 *      measure.  Systematic (default): U uniform on the integers [0, Q),
 *      t_j = U + j Q, ancestor a(j) = min{i : M C_i > t_j}, C the inclusive
 *      prefix sum of q.  Multinomial: a(j) = min{i : C_i > U_j}, U_j iid.
 *   6. Stages s = 1..S (S = log2 m), each exactly as the stage loop of
 *      Algorithm 1: ENF_{n,s} = (m^-1 sum W)^2 / (m^-1 sum W^2); interact
 *      (alpha_s = A_s) iff ENF < tau, else alpha_s = I.  A_s pairs island k
 *      with p = k xor 2^(s-1) (0-based; the Kronecker structure
 *      I (x) (1/2)1_2 (x) I of the interaction matrices).  Interacting:
 *        W'_k = W'_p = (W_k + W_p)/2         (the normaliser line),
 *        block k := block p with probability W_p / (W_k + W_p), drawn
 *        independently for every island, else block k is kept.
 *      r-ary interactions (Section 2 allows m = r^S for any r >= 2; here r
 *      a power of two): S_r = log_r m stages, A_s = I (x) (1/r)1_r (x)
 *      I_{r^(s-1)}, so stage s groups the r islands whose base-r digits
 *      agree except digit s-1.  Interacting: every member's new weight is
 *      the group mean (r/2 pair means, then pair means of those, in digit
 *      order), and block k := block of member d with probability
 *      W_d / sum W: the first d whose running sum of exp(L_d - max L)
 *      exceeds u times the total, u island k's uniform of the stage (the
 *      last live member if rounding leaves none).
 *   7. Mutation into step n+1 (the final-stage line), also when m = 1 or
 *      when no stage interacted: x_{n+1}^{k,j} ~ K(block pi(k) slot j, .),
 *      where pi(k) is the original island whose (internally resampled)
 *      block island k holds after the stages.
 *
 * Readings where the text is silent: strict "<" in the ENF test; pair
 * probability 1/(1 + exp(L_k - L_p)) with a dead partner never taken and a
 * dead island always taking a live partner; a dead island (all weights
 * zero) resamples to the identity; NaN log-potentials count as -inf.
 *
 * Score (forward-mode tangents, decisions frozen, quantisation read as the
 * identity so weights are exp(lw) exactly):
 *   PATHWISE  : d/dtheta of F = logsumexp_k L^ex_k - log m along the frozen
 *               genealogy, with L^ex the exact-weight island log-weights;
 *   PATHSPACE : sum over final particles of their normalised final weight
 *               times the total derivative of the path's summed log g.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"
#include "orc_models.h"

uint64_t orc_fmix64(uint64_t h) {
  h ^= h >> 33; h *= 0xff51afd7ed558ccdULL;
  h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ULL;
  h ^= h >> 33;
  return h;
}

/* digest term of value v at (step n, island k, slot j); j = 4095 marks the
 * island-map digest.  Digests are wrap-around sums of terms, so their value
 * does not depend on summation order. */
uint64_t orc_digest_term(int64_t n, int64_t k, int64_t j, int64_t v) {
  const uint64_t key = ((uint64_t)n << 28) ^ ((uint64_t)k << 12) ^ (uint64_t)j;
  return orc_fmix64(orc_fmix64(key) ^ (uint64_t)v);
}

static double nan_to_ninf(double v) { return (v != v) ? -INFINITY : v; }

void orc_quantise(const double* lw, int32_t N, uint64_t* q, double* mx_out) {
  double mx = -INFINITY;
  for (int32_t i = 0; i < N; ++i) if (lw[i] > mx) mx = lw[i];
  *mx_out = mx;
  for (int32_t i = 0; i < N; ++i) {
    if (mx == -INFINITY) { q[i] = 0; continue; }
    const double e = orc_exp(lw[i] - mx);
    q[i] = (uint64_t)(e * 0x1p40);
  }
}

void orc_systematic(const uint64_t* q, int32_t N, uint64_t U, int32_t* anc) {
  uint64_t Q = 0;
  for (int32_t i = 0; i < N; ++i) Q += q[i];
  int32_t i = 0;
  uint64_t C = q[0];                                   /* C_i inclusive */
  for (int32_t j = 0; j < N; ++j) {
    const uint64_t t = U + (uint64_t)j * Q;
    while ((uint64_t)N * C <= t) { ++i; C += q[i]; }
    anc[j] = i;
  }
}

static void multinomial(const uint64_t* q, int32_t N, uint64_t seed, int64_t n,
                        int32_t k, uint64_t Q, int32_t* anc) {
  for (int32_t j = 0; j < N; ++j) {
    const uint64_t U = orc_bounded(seed, (uint32_t)j, (uint32_t)k, (uint32_t)n, TAG_MULT, Q);
    int32_t i = 0;
    uint64_t C = q[0];
    while (C <= U) { ++i; C += q[i]; }
    anc[j] = i;
  }
}

static double enf_of(const double* L, int32_t m) {
  double Lmax = -INFINITY;
  for (int32_t k = 0; k < m; ++k) if (L[k] > Lmax) Lmax = L[k];
  if (Lmax == -INFINITY) return NAN;
  double s1 = 0.0, s2 = 0.0;
  for (int32_t k = 0; k < m; ++k) {
    const double W = orc_exp(L[k] - Lmax);
    s1 += W;
    s2 += W * W;
  }
  const double a = s1 / (double)m, b = s2 / (double)m;
  return (a * a) / b;
}

/* probability that island with log-weight Lk takes its partner's block */
static double prob_partner(double Lk, double Lp) {
  if (Lp == -INFINITY) return 0.0;
  if (Lk == -INFINITY) return 1.0;
  return 1.0 / (1.0 + orc_exp(Lk - Lp));
}

/* the member of island k's r-group that island k's stage draw u selects:
   W_d / sum W by a running sum of exp(L_d - max); all dead: k's own digit */
static int32_t pick_in_group(const double* L, int32_t base, int32_t b, int32_t r, int32_t own, double u) {
  double hi = -INFINITY;
  for (int32_t d = 0; d < r; ++d) if (L[base + d * b] > hi) hi = L[base + d * b];
  if (hi == -INFINITY) return own;
  double tot = 0.0;
  for (int32_t d = 0; d < r; ++d) tot += orc_exp(L[base + d * b] - hi);
  const double t = u * tot;
  double run = 0.0;
  int32_t last = own;
  for (int32_t d = 0; d < r; ++d) {
    const double w = orc_exp(L[base + d * b] - hi);
    run += w;
    if (w > 0.0) last = d;
    if (t < run) return d;
  }
  return last;
}

/* log((W_k + W_p)/2), symmetric in its arguments */
static double pair_mean(double a, double b) {
  const double hi = a > b ? a : b, lo = a > b ? b : a;
  if (hi == -INFINITY) return -INFINITY;
  double t = orc_exp(lo - hi);
  t = 1.0 + t;
  t = orc_log(t);
  return (hi + t) - 0x1.62e42fefa39efp-1;
}

/* log of the mean of the r group members' weights: pair means of
   neighbours in digit order, then of those, up to one value (gv: r slots) */
static double group_mean(const double* L, int32_t base, int32_t b, int32_t r, double* gv) {
  for (int32_t d = 0; d < r; ++d) gv[d] = L[base + d * b];
  for (int32_t w = r; w > 1; w >>= 1)
    for (int32_t i = 0; i < w / 2; ++i) gv[i] = pair_mean(gv[2 * i], gv[2 * i + 1]);
  return gv[0];
}

static double lse(const double* L, int64_t m) {
  double Lmax = -INFINITY;
  for (int64_t k = 0; k < m; ++k) if (L[k] > Lmax) Lmax = L[k];
  if (Lmax == -INFINITY) return -INFINITY;
  double s = 0.0;
  for (int64_t k = 0; k < m; ++k) s += orc_exp(L[k] - Lmax);
  return Lmax + orc_log(s);
}

typedef struct {
  double* grad_pathwise;    /* [P] or NULL */
  double* grad_pathspace;   /* [P] or NULL */
  double* final_S;          /* [m*N] path sums of full log g, or NULL */
  double* final_logw;       /* [m*N] unnormalised final log-weights, or NULL */
} orc_score_out;

static int ilog2(int32_t m) { int s = 0; while ((1 << s) < m) ++s; return s; }

/* returns 0 on success; *logz quantised-weight log Zhat, *logz_ex exact-weight */
static int airpf_core(const orc_problem* P, const orc_opts* O, orc_trace* tr,
                      orc_score_out* so, double* logz, double* logz_ex) {
  *logz = NAN;
  if (logz_ex) *logz_ex = NAN;
  /* sizes the fixed-point rule supports: N C_i <= N^2 2^40 < 2^64 needs N <= 2^11 */
  if (P->m < 1 || (P->m & (P->m - 1)) != 0 || P->N < 1 || P->N > 2048 || P->T < 1 ||
      P->dx < 1 || P->dx > ORC_MAX_DX || P->dy < 1 || P->dy > ORC_MAX_DY ||
      P->d_theta > ORC_MAX_P || (O->replay && (!tr || !tr->anc || !tr->pi || !tr->sstar)))
    return -1;
  const int32_t m = P->m, N = P->N, dx = P->dx, dy = P->dy;
  const int64_t T = P->T;
  const int S = ilog2(m);
  /* r-ary interactions: r = 2^rb, m = r^Sr */
  const int32_t r = O->arity == 0 ? 2 : O->arity;
  if (r < 2 || (r & (r - 1)) != 0 || r > 65536) return -1;
  const int rb = ilog2(r);
  if (S % rb != 0) return -1;
  const int Sr = S / rb;
  orc_model M;
  orc_model_setup(&M, P, O->f32);
  const int nd = orc_model_noise_dim(&M);
  const int Pn = P->d_theta;
  const int want_score = so && (so->grad_pathwise || so->grad_pathspace);
  const int want_paths = so && (so->final_S || so->final_logw);
  const int64_t mN = (int64_t)m * N;

  double* x = malloc(sizeof(double) * mN * dx);
  double* xn = malloc(sizeof(double) * mN * dx);
  double* lw = malloc(sizeof(double) * mN);
  uint64_t* q = malloc(sizeof(uint64_t) * mN);
  uint64_t* Qk = malloc(sizeof(uint64_t) * m);
  int32_t* anc = malloc(sizeof(int32_t) * mN);
  double* L = malloc(sizeof(double) * m);
  double* Lx = malloc(sizeof(double) * m);
  double* Lpre = malloc(sizeof(double) * m);
  double* Lnew = malloc(sizeof(double) * m);
  double* Lxnew = malloc(sizeof(double) * m);
  int32_t* pi = malloc(sizeof(int32_t) * m);
  int32_t* pinew = malloc(sizeof(int32_t) * m);
  int32_t* src = malloc(sizeof(int32_t) * m);
  double* z = malloc(sizeof(double) * (size_t)N * nd);
  double *dX = NULL, *dXn = NULL, *Sp = NULL, *Spn = NULL, *dL = NULL, *dLn = NULL,
         *dlw = NULL, *Sf = NULL, *Sfn = NULL;
  if (want_score) {
    dX = calloc((size_t)mN * dx * Pn, sizeof(double));
    dXn = calloc((size_t)mN * dx * Pn, sizeof(double));
    Sp = calloc((size_t)mN * Pn, sizeof(double));
    Spn = calloc((size_t)mN * Pn, sizeof(double));
    dL = calloc((size_t)m * Pn, sizeof(double));
    dLn = calloc((size_t)m * Pn, sizeof(double));
    dlw = calloc((size_t)mN * Pn, sizeof(double));
  }
  if (want_paths) {
    Sf = calloc((size_t)mN, sizeof(double));
    Sfn = calloc((size_t)mN, sizeof(double));
  }
  const double cst_q = M.c_log - 40.0 * log(2.0) - log((double)N);
  /* adaptive internal resampling (ess_frac > 0): a particle's carried
     weight lc = log of its fixed-point weight at the last weighting (0 right
     after a resampling), an island's carried normaliser dq = log Q - log N of
     that weighting (0 after a resampling); both travel with the block */
  const int adapt = O->ess_frac > 0.0;
  const double logN = log((double)N);
  double* lc = calloc((size_t)mN, sizeof(double));
  double* lcn = calloc((size_t)mN, sizeof(double));
  double* dq = calloc((size_t)m, sizeof(double));
  double* dqn = calloc((size_t)m, sizeof(double));
  int* resamp = malloc(sizeof(int) * m);
  double* gv = malloc(sizeof(double) * r);
  const double cst_x = M.c_log - log((double)N);

  /* Initialisation: W^k_{0,0} = 1, xi^k_{0,0} ~ pi_0^{(x)M} */
  for (int32_t k = 0; k < m; ++k) {
    orc_model_noise(&M, P->seed, 0, k, N, z);
    for (int32_t j = 0; j < N; ++j) {
      const int64_t id = (int64_t)k * N + j;
      orc_model_init(&M, z + (size_t)j * nd, x + id * dx);
      if (want_score) orc_model_init_tangent(&M, z + (size_t)j * nd, dX + id * dx * Pn);
    }
    L[k] = 0.0;
    Lx[k] = 0.0;
  }

  double out_logz = 0.0, out_logz_ex = 0.0;
  int dead = 0;
  for (int64_t n = 0; n < T; ++n) {
    const double* yn = P->y + n * dy;
    if (tr && tr->enf) tr->enf[n * (S + 1)] = enf_of(L, m);
    if (tr && tr->x) memcpy(tr->x + n * mN * dx, x, sizeof(double) * mN * dx);
    if (tr && tr->lpre) memcpy(tr->lpre + n * m, L, sizeof(double) * m);
    const double lse_pre = lse(L, m);
    for (int32_t k = 0; k < m; ++k) Lpre[k] = Lx[k];

    /* island weighting */
    for (int32_t k = 0; k < m; ++k) {
      double* lwk = lw + (int64_t)k * N;
      for (int32_t j = 0; j < N; ++j)
        lwk[j] = nan_to_ninf(orc_model_logpot(&M, x + ((int64_t)k * N + j) * dx, yn));
      if (adapt)
        for (int32_t j = 0; j < N; ++j) lwk[j] = lc[(int64_t)k * N + j] + lwk[j];
      double mx;
      orc_model_quantise(&M, lwk, N, q + (int64_t)k * N, &mx);
      uint64_t Q = 0;
      double se = 0.0;
      for (int32_t j = 0; j < N; ++j) {
        Q += q[(int64_t)k * N + j];
        if (mx != -INFINITY) se += orc_exp(lwk[j] - mx);
      }
      Qk[k] = Q;
      if (tr && tr->fmean) {
        /* the island's estimate of the filtering mean of x (first coordinate) */
        double num = 0.0;
        for (int32_t j = 0; j < N; ++j) num += (double)q[(int64_t)k * N + j] * x[((int64_t)k * N + j) * dx];
        tr->fmean[n * m + k] = (Q == 0) ? NAN : num / (double)Q;
      }
      L[k] = (Q == 0) ? -INFINITY : L[k] + ((mx + orc_log((double)Q)) + cst_q);
      Lx[k] = (mx == -INFINITY) ? -INFINITY : Lx[k] + ((mx + orc_log(se)) + cst_x);
      if (adapt) {
        /* the carried normaliser: Algorithm 1's island weight update with the
           particles' incoming weights q_prev / Q_prev instead of 1 / N */
        if (Q != 0) L[k] = L[k] - dq[k];
        if (mx != -INFINITY) Lx[k] = Lx[k] - dq[k];
        /* the ESS of the island's weights, from the weights truncated to
           their top 20 of 40 bits (exact integer sums) */
        uint64_t Qt = 0, S2 = 0;
        for (int32_t j = 0; j < N; ++j) {
          const uint64_t qt = q[(int64_t)k * N + j] >> 20;
          Qt += qt;
          S2 += qt * qt;
        }
        resamp[k] = Q != 0 && S2 != 0 && (double)Qt * (double)Qt < O->ess_frac * (double)N * (double)S2;
      }
      if (want_score) {
        double* dLk = dL + (int64_t)k * Pn;
        for (int32_t j = 0; j < N; ++j) {
          const int64_t id = (int64_t)k * N + j;
          orc_model_logpot_tangent(&M, x + id * dx, dX + id * dx * Pn, yn, dlw + id * Pn);
          const double wj = (mx == -INFINITY) ? 0.0 : orc_exp(lwk[j] - mx) / se;
          for (int p = 0; p < Pn; ++p) {
            dLk[p] += wj * dlw[id * Pn + p];
            Sp[id * Pn + p] += dlw[id * Pn + p];
          }
        }
      }
      if (want_paths)
        for (int32_t j = 0; j < N; ++j) Sf[(int64_t)k * N + j] += lwk[j] + M.c_log;
    }
    if (tr && tr->lpost) memcpy(tr->lpost + n * m, L, sizeof(double) * m);
    const double lse_post = lse(L, m);
    if (tr && tr->logz_inc) tr->logz_inc[n] = lse_post - lse_pre;
    out_logz = lse_post - log((double)m);
    out_logz_ex = lse(Lx, m) - log((double)m);
    if (lse_post == -INFINITY) { dead = 1; }

    if (n == T - 1 || dead) {
      if (want_score) {
        /* final weights W^{k,i} ~ W^k_{T-1,0} g(xi^{k,i}) (exact) */
        double gmax = -INFINITY;
        for (int32_t k = 0; k < m; ++k)
          for (int32_t j = 0; j < N; ++j) {
            const double v = Lpre[k] + lw[(int64_t)k * N + j];
            if (v > gmax) gmax = v;
          }
        double tot = 0.0;
        for (int64_t id = 0; id < mN; ++id) {
          const double v = Lpre[id / N] + lw[id];
          if (gmax != -INFINITY) tot += exp(v - gmax);
        }
        double Lxmax = -INFINITY;
        for (int32_t k = 0; k < m; ++k) if (Lx[k] > Lxmax) Lxmax = Lx[k];
        double totk = 0.0;
        for (int32_t k = 0; k < m; ++k) if (Lxmax != -INFINITY) totk += exp(Lx[k] - Lxmax);
        for (int p = 0; p < Pn; ++p) {
          double gps = 0.0, gpw = 0.0;
          for (int64_t id = 0; id < mN; ++id) {
            const double v = Lpre[id / N] + lw[id];
            if (gmax != -INFINITY && v != -INFINITY) gps += exp(v - gmax) / tot * Sp[id * Pn + p];
          }
          for (int32_t k = 0; k < m; ++k)
            if (Lx[k] != -INFINITY) gpw += exp(Lx[k] - Lxmax) / totk * dL[(int64_t)k * Pn + p];
          if (so->grad_pathspace) so->grad_pathspace[p] = gps;
          if (so->grad_pathwise) so->grad_pathwise[p] = gpw;
        }
      }
      if (want_paths)
        for (int64_t id = 0; id < mN; ++id) {
          if (so->final_S) so->final_S[id] = Sf[id];
          if (so->final_logw) so->final_logw[id] = Lpre[id / N] + lw[id] + M.c_log;
        }
      if (tr && tr->sstar) tr->sstar[n] = 0;
      break;
    }

    /* internal resampling */
    for (int32_t k = 0; k < m; ++k) {
      int32_t* ak = anc + (int64_t)k * N;
      if (O->replay) {
        memcpy(ak, tr->anc + n * mN + (int64_t)k * N, sizeof(int32_t) * N);
      } else if (Qk[k] == 0 || (adapt && !resamp[k])) {
        for (int32_t j = 0; j < N; ++j) ak[j] = j;
      } else if (O->scheme == 1) {
        multinomial(q + (int64_t)k * N, N, P->seed, n, k, Qk[k], ak);
      } else {
        const uint64_t U = orc_bounded(P->seed, 0, (uint32_t)k, (uint32_t)n, TAG_SYS, Qk[k]);
        orc_systematic(q + (int64_t)k * N, N, U, ak);
      }
    }

    /* filter interaction: stages s = 1..Sr (Sr = S for pairs) */
    for (int32_t k = 0; k < m; ++k) pi[k] = k;
    int sstar = 0;
    for (int s = 1; s <= Sr; ++s) {
      const double enf = enf_of(L, m);
      if (tr && tr->enf) tr->enf[n * (S + 1) + s] = enf;
      const int interact = O->replay ? (s <= tr->sstar[n]) : (enf < O->tau);
      if (!interact) continue;          /* alpha_s = I: weights and blocks unchanged */
      sstar = s;
      if (rb > 1) {
        /* groups of r: the members of island k's group are base + d b */
        const int32_t b = 1 << ((s - 1) * rb);
        for (int32_t k = 0; k < m; ++k) {
          const int32_t own = (k / b) % r, base = k - own * b;
          if (!O->replay) {
            uint32_t w[4];
            orc_draw(P->seed, (uint32_t)s, (uint32_t)k, (uint32_t)n, TAG_ISL, 0, w);
            src[k] = base + b * pick_in_group(L, base, b, r, own, orc_u53(w[0], w[1]));
          } else {
            src[k] = k;
          }
          pinew[k] = pi[src[k]];
          Lnew[k] = group_mean(L, base, b, r, gv);
          Lxnew[k] = group_mean(Lx, base, b, r, gv);
          if (want_score) {
            double hi = -INFINITY, tot = 0.0;
            for (int32_t d = 0; d < r; ++d) if (Lx[base + d * b] > hi) hi = Lx[base + d * b];
            for (int pp = 0; pp < Pn; ++pp) dLn[(int64_t)k * Pn + pp] = 0.0;
            for (int32_t d = 0; d < r; ++d) {
              const int32_t l = base + d * b;
              const double wl = (hi == -INFINITY) ? 1.0 : exp(Lx[l] - hi);
              tot += wl;
              for (int pp = 0; pp < Pn; ++pp) dLn[(int64_t)k * Pn + pp] += wl * dL[(int64_t)l * Pn + pp];
            }
            for (int pp = 0; pp < Pn; ++pp) dLn[(int64_t)k * Pn + pp] /= tot;
          }
        }
      } else {
      const int32_t b = 1 << (s - 1);
      for (int32_t k = 0; k < m; ++k) {
        const int32_t p = k ^ b;
        if (!O->replay) {
          uint32_t w[4];
          orc_draw(P->seed, (uint32_t)s, (uint32_t)k, (uint32_t)n, TAG_ISL, 0, w);
          const double u = orc_u53(w[0], w[1]);
          src[k] = (u < prob_partner(L[k], L[p])) ? p : k;
        } else {
          src[k] = k;
        }
        pinew[k] = pi[src[k]];
        Lnew[k] = pair_mean(L[k], L[p]);
        Lxnew[k] = pair_mean(Lx[k], Lx[p]);
        if (want_score) {
          const double hi = Lx[k] > Lx[p] ? Lx[k] : Lx[p];
          const double wk = (hi == -INFINITY) ? 0.5 : exp(Lx[k] - hi);
          const double wp = (hi == -INFINITY) ? 0.5 : exp(Lx[p] - hi);
          for (int pp = 0; pp < Pn; ++pp)
            dLn[(int64_t)k * Pn + pp] = (wk * dL[(int64_t)k * Pn + pp] + wp * dL[(int64_t)p * Pn + pp]) / (wk + wp);
        }
      }
      }  /* pairs */
      memcpy(pi, pinew, sizeof(int32_t) * m);
      memcpy(L, Lnew, sizeof(double) * m);
      memcpy(Lx, Lxnew, sizeof(double) * m);
      if (want_score) memcpy(dL, dLn, sizeof(double) * m * Pn);
    }
    if (O->replay) memcpy(pi, tr->pi + n * m, sizeof(int32_t) * m);
    if (tr && tr->sstar) tr->sstar[n] = sstar;
    if (tr && tr->anc && !O->replay) memcpy(tr->anc + n * mN, anc, sizeof(int32_t) * mN);
    if (tr && tr->pi && !O->replay) memcpy(tr->pi + n * m, pi, sizeof(int32_t) * m);
    if (tr && tr->digest) {
      uint64_t da = 0, dp = 0;
      for (int32_t k = 0; k < m; ++k) {
        for (int32_t j = 0; j < N; ++j) da += orc_digest_term(n, k, j, anc[(int64_t)k * N + j]);
        dp += orc_digest_term(n, k, 4095, pi[k]);
      }
      dp += (uint64_t)sstar * 0x9E3779B97F4A7C15ULL;
      tr->digest[2 * n] = da;
      tr->digest[2 * n + 1] = dp;
    }

    /* carried weights after the internal step: 0 after a resampling, else
       the log of the fixed-point weight */
    if (adapt)
      for (int32_t k = 0; k < m; ++k)
        for (int32_t j = 0; j < N; ++j) {
          const int64_t id = (int64_t)k * N + j;
          lc[id] = resamp[k] ? 0.0 : orc_log((double)q[id]);
          if (j == 0) dq[k] = resamp[k] ? 0.0 : orc_log((double)Qk[k]) - logN;
        }

    /* mutation into step n+1 */
    for (int32_t k = 0; k < m; ++k) {
      orc_model_noise(&M, P->seed, n + 1, k, N, z);
      const int32_t sk = pi[k];
      if (adapt) dqn[k] = dq[sk];
      for (int32_t j = 0; j < N; ++j) {
        const int64_t par = (int64_t)sk * N + anc[(int64_t)sk * N + j];
        const int64_t id = (int64_t)k * N + j;
        orc_model_prop(&M, x + par * dx, z + (size_t)j * nd, xn + id * dx);
        if (adapt) lcn[id] = lc[par];
        if (want_score) {
          orc_model_prop_tangent(&M, x + par * dx, dX + par * dx * Pn, z + (size_t)j * nd,
                                 dXn + id * dx * Pn);
          memcpy(Spn + id * Pn, Sp + par * Pn, sizeof(double) * Pn);
        }
        if (want_paths) Sfn[id] = Sf[par];
      }
    }
    { double* t = x; x = xn; xn = t; }
    if (adapt) {
      double* t = lc; lc = lcn; lcn = t;
      t = dq; dq = dqn; dqn = t;
    }
    if (want_score) {
      double* t = dX; dX = dXn; dXn = t;
      t = Sp; Sp = Spn; Spn = t;
    }
    if (want_paths) { double* t = Sf; Sf = Sfn; Sfn = t; }
  }

  *logz = out_logz;
  if (logz_ex) *logz_ex = out_logz_ex;
  free(x); free(xn); free(lw); free(q); free(Qk); free(anc); free(L); free(Lx);
  free(Lpre); free(Lnew); free(Lxnew); free(pi); free(pinew); free(src); free(z);
  free(dX); free(dXn); free(Sp); free(Spn); free(dL); free(dLn); free(dlw);
  free(Sf); free(Sfn);
  free(lc); free(lcn); free(dq); free(dqn); free(resamp); free(gv);
  return 0;
}

/* ---------------- exported entry points ---------------- */

double orc_airpf_run(const orc_problem* P, const orc_opts* O, orc_trace* tr) {
  double lz = NAN;
  airpf_core(P, O, tr, NULL, &lz, NULL);
  return lz;
}

/* forward-mode score; returns log Zhat (quantised) and both gradients */
double orc_airpf_score(const orc_problem* P, const orc_opts* O, orc_trace* tr,
                       double* grad_pathwise, double* grad_pathspace) {
  orc_score_out so = {grad_pathwise, grad_pathspace, NULL, NULL};
  double lz = NAN;
  airpf_core(P, O, tr, &so, &lz, NULL);
  return lz;
}

/* frozen estimator: with O->replay the genealogy comes from tr; returns the
 * exact-weight log Zhat (the pathwise F) and, if asked, per final particle
 * the path sum of log g and the unnormalised final log-weight. */
double orc_airpf_frozen(const orc_problem* P, const orc_opts* O, orc_trace* tr,
                        double* final_S, double* final_logw) {
  orc_score_out so = {NULL, NULL, final_S, final_logw};
  double lz = NAN, lzx = NAN;
  airpf_core(P, O, tr, &so, &lz, &lzx);
  return lzx;
}
