/*
 * AIRPF CPU oracle -- the state-space models (Section 1.2, the HMM (1) with
 * latent kernel K, observation density g_n = G(., y_n), initial law pi_0).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Double-precision runs use the forms below in double arithmetic.  Runs with
 * binary32 particles (f32) evaluate the same model in single precision:
 * parameters and derived constants rounded to binary32 once (the derived
 * ones computed in double first), observations rounded to binary32, normals
 * from the binary32 Box-Muller, every operation a binary32 one, and the
 * quantised weight q = (uint64)(expf(lw - mx) * 2^40) with the difference
 * taken in binary32.  Each formula is written in the exact operation order
 * the GPU library follows (explicit fma where fused, no contraction
 * elsewhere); binary32 forms differ only where noted.
 *
 *   LG1  theta = (a, sx, sy):  x_0 = z;  x' = fma(a, x, sx*z);
 *        log g = -(1/2) r^2 + c,  r = (y - x)/sy,  c = -log sy - log(2 pi)/2
 *        (binary32: r = (y - x) * isy with isy = 1/sy rounded).
 *   SV   theta = (mu, phi, sigma), s0 = sigma / sqrt(1 - phi^2):
 *        x_0 = fma(s0, z, mu);  x' = fma(phi, x - mu, fma(sigma, z, mu));
 *        log g = fma(-h, exp(-x), -x/2) + c,  h = y^2/2,  c = -log(2 pi)/2.
 *   LGD  theta = vec(A) (dx x dx, row-major); consts q, r, p0, H (dy x dx);
 *        x_0[d] = sqrt(p0) z_d;
 *        x'[i] = acc, acc = sqrt(q) z_i, then acc = fma(A[i][c], x[c], acc)
 *                for c = 0..dx-1;
 *        e_i = y_i, then e_i = fma(-H[i][c], x[c], e_i) for c = 0..dx-1;
 *        ss = 0, ss = fma(e_i, e_i, ss) for i = 0..dy-1;
 *        log g = -(ss * (1/(2r))) + c,  c = -(dy/2) log(2 pi r).
 *   BIN  the binary toy HMM of the exact-variance experiment (Section 4.1):
 *        x in {0,1}, x_0 = w >> 31, flip iff (w >> 30) == 0 (prob 1/4),
 *        g = 3/4 if y == x else 1/4, written as log g = l + log(3/4) with
 *        l = 0 (match) or l = -log 3.
 *   BCP  the Beta change-point model of the change-point experiment (Section
 *        4.2): a rate x in (0,1), x_0 ~ Beta(alpha, beta), x' = x with
 *        probability 1 - p, else a fresh Beta(alpha, beta) draw; theta = (p),
 *        consts = (alpha, beta), positive integers with alpha + beta <= 7;
 *        y_n = (k_n, n_n) counts, g = x^k (1-x)^(n-k) (the binomial
 *        likelihood without its data-only coefficient).  The state is
 *        (log x, log(1-x)).  A particle's step uses the eight words of two
 *        Philox blocks (counters 2j and 2j+1, tag 6): word 0 decides the
 *        change (u0 = w0 2^-32 < p), words 1..alpha+beta give the uniforms
 *        u_i = (w_i + 1/2) 2^-32 of the draw
 *          ga = 0, ga -= log(u_i) for i = 1..alpha;
 *          gb = 0, gb -= log(u_i) for i = alpha+1..alpha+beta;
 *          ls = log(ga + gb);  x = (log(ga) - ls, log(gb) - ls)
 *        (a sum of k unit exponentials is Gamma(k, 1), and Ga / (Ga + Gb) is
 *        Beta(alpha, beta)); log is the oracle's own orc_log.
 *        lw = y_0 * x_0 + (y_1 - y_0) * x_1, no constant.
 * The per-particle part (without c) is what gets quantised; c is added once
 * per island and step.  Constants c, s0, sqrt(q), sqrt(p0), 1/(2r) and log 3
 * come from the host libm.
 */
#include <math.h>
#include <stdint.h>
#include "orc.h"
#include "orc_models.h"

void orc_model_setup(orc_model* M, const orc_problem* P, int f32) {
  M->kind = P->kind; M->dx = P->dx; M->dy = P->dy; M->P = P->d_theta;
  M->f32 = (P->kind == ORC_BIN || P->kind == ORC_BCP) ? 0 : f32;   /* word-driven models: double only */
  for (int i = 0; i < P->d_theta && i < ORC_MAX_P; ++i) {
    M->th[i] = P->theta[i];
    M->thf[i] = (float)P->theta[i];
  }
  const double LOG2PI = log(2.0 * M_PI);
  switch (P->kind) {
    case ORC_LG1:
      M->c_log = -log(M->th[2]) - 0.5 * LOG2PI;
      M->isyf = (float)(1.0 / M->th[2]);
      break;
    case ORC_SV:
      M->s0 = M->th[2] / sqrt(1.0 - M->th[1] * M->th[1]);
      M->s0f = (float)M->s0;
      M->c_log = -0.5 * LOG2PI;
      break;
    case ORC_LGD: {
      const double q = P->consts[0], r = P->consts[1], p0 = P->consts[2];
      M->q = q; M->r = r; M->p0 = p0;
      M->sq = sqrt(q); M->sp0 = sqrt(p0); M->hr = 1.0 / (2.0 * r);
      M->sqf = (float)M->sq; M->sp0f = (float)M->sp0; M->hrf = (float)M->hr;
      for (int i = 0; i < P->dy * P->dx; ++i) {
        M->H[i] = P->consts[3 + i];
        M->Hf[i] = (float)M->H[i];
      }
      M->c_log = -(0.5 * (double)P->dy) * log(2.0 * M_PI * r);
      break;
    }
    case ORC_BIN:
      M->c_log = log(0.75);
      M->log3 = log(3.0);
      break;
    case ORC_BCP:
      M->c_log = 0.0;
      M->ab[0] = (int)P->consts[0];
      M->ab[1] = (int)P->consts[1];
      break;
  }
}

/* a Beta(alpha, beta) draw from words w[1..alpha+beta] as (log x, log(1-x)) */
static void bcp_beta(const orc_model* M, const double* w, double* x) {
  double ga = 0.0, gb = 0.0;
  for (int i = 1; i <= M->ab[0]; ++i) ga -= orc_log((w[i] + 0.5) * 0x1p-32);
  for (int i = M->ab[0] + 1; i <= M->ab[0] + M->ab[1]; ++i) gb -= orc_log((w[i] + 0.5) * 0x1p-32);
  const double ls = orc_log(ga + gb);
  x[0] = orc_log(ga) - ls;
  x[1] = orc_log(gb) - ls;
}

/* number of N(0,1) (or BIN words) one particle consumes per step */
int orc_model_noise_dim(const orc_model* M) {
  return M->kind == ORC_BIN ? 1 : (M->kind == ORC_BCP ? 8 : M->dx);
}

/* noise for particles 0..N-1 of (step n, island k): z[j*dim + d] */
void orc_model_noise(const orc_model* M, uint64_t seed, int64_t n, int32_t k,
                     int32_t N, double* z) {
  if (M->kind == ORC_BIN) {
    for (int32_t j = 0; j < N; ++j) {
      uint32_t w[4];
      orc_draw(seed, (uint32_t)j, (uint32_t)k, (uint32_t)n, TAG_BIN, 0, w);
      z[j] = (double)w[0];
    }
  } else if (M->kind == ORC_BCP) {
    for (int32_t j = 0; j < N; ++j) {
      uint32_t w[4];
      for (int b = 0; b < 2; ++b) {
        orc_draw(seed, (uint32_t)(2 * j + b), (uint32_t)k, (uint32_t)n, TAG_BCP, 0, w);
        for (int i = 0; i < 4; ++i) z[8 * j + 4 * b + i] = (double)w[i];
      }
    }
  } else if (M->f32) {
    orc_island_normalsf(seed, n, k, (int64_t)N * M->dx, z);
  } else {
    orc_island_normals(seed, n, k, (int64_t)N * M->dx, z);
  }
}

void orc_model_init(const orc_model* M, const double* z, double* x) {
  if (M->f32 && M->kind != ORC_BIN && M->kind != ORC_BCP) {
    switch (M->kind) {
      case ORC_LG1: x[0] = (double)(float)z[0]; break;
      case ORC_SV: x[0] = (double)fmaf(M->s0f, (float)z[0], M->thf[0]); break;
      case ORC_LGD:
        for (int d = 0; d < M->dx; ++d) x[d] = (double)(M->sp0f * (float)z[d]);
        break;
    }
    return;
  }
  switch (M->kind) {
    case ORC_LG1: x[0] = z[0]; break;
    case ORC_SV: x[0] = fma(M->s0, z[0], M->th[0]); break;
    case ORC_LGD:
      for (int d = 0; d < M->dx; ++d) x[d] = M->sp0 * z[d];
      break;
    case ORC_BIN: x[0] = (double)(((uint32_t)z[0]) >> 31); break;
    case ORC_BCP: bcp_beta(M, z, x); break;
  }
}

void orc_model_prop(const orc_model* M, const double* xp, const double* z, double* x) {
  if (M->f32 && M->kind != ORC_BIN && M->kind != ORC_BCP) {
    switch (M->kind) {
      case ORC_LG1:
        x[0] = (double)fmaf(M->thf[0], (float)xp[0], M->thf[1] * (float)z[0]);
        break;
      case ORC_SV: {
        const float mu = M->thf[0], phi = M->thf[1], sig = M->thf[2];
        x[0] = (double)fmaf(phi, (float)xp[0] - mu, fmaf(sig, (float)z[0], mu));
        break;
      }
      case ORC_LGD: {
        const int dx = M->dx;
        for (int i = 0; i < dx; ++i) {
          float acc = M->sqf * (float)z[i];
          for (int c = 0; c < dx; ++c) acc = fmaf(M->thf[i * dx + c], (float)xp[c], acc);
          x[i] = (double)acc;
        }
        break;
      }
    }
    return;
  }
  switch (M->kind) {
    case ORC_LG1: x[0] = fma(M->th[0], xp[0], M->th[1] * z[0]); break;
    case ORC_SV: {
      const double mu = M->th[0], phi = M->th[1], sig = M->th[2];
      x[0] = fma(phi, xp[0] - mu, fma(sig, z[0], mu));
      break;
    }
    case ORC_LGD: {
      const int dx = M->dx;
      for (int i = 0; i < dx; ++i) {
        double acc = M->sq * z[i];
        for (int c = 0; c < dx; ++c) acc = fma(M->th[i * dx + c], xp[c], acc);
        x[i] = acc;
      }
      break;
    }
    case ORC_BIN: {
      const uint32_t w = (uint32_t)z[0];
      x[0] = ((w >> 30) == 0) ? 1.0 - xp[0] : xp[0];
      break;
    }
    case ORC_BCP:
      if (z[0] * 0x1p-32 < M->th[0]) {
        bcp_beta(M, z, x);
      } else {
        x[0] = xp[0];
        x[1] = xp[1];
      }
      break;
  }
}

/* per-particle part of log g_n(x) (the model constant c is not included) */
double orc_model_logpot(const orc_model* M, const double* x, const double* y) {
  if (M->f32 && M->kind != ORC_BIN && M->kind != ORC_BCP) {
    switch (M->kind) {
      case ORC_LG1: {
        const float r = ((float)y[0] - (float)x[0]) * M->isyf;
        return (double)(-0.5f * (r * r));
      }
      case ORC_SV: {
        const float yf = (float)y[0], xf = (float)x[0];
        const float h = 0.5f * (yf * yf);
        return (double)fmaf(-h, orc_expf(-xf), -0.5f * xf);
      }
      case ORC_LGD: {
        const int dx = M->dx, dy = M->dy;
        float ss = 0.0f;
        for (int i = 0; i < dy; ++i) {
          float e = (float)y[i];
          for (int c = 0; c < dx; ++c) e = fmaf(-M->Hf[i * dx + c], (float)x[c], e);
          ss = fmaf(e, e, ss);
        }
        return (double)(-(ss * M->hrf));
      }
    }
    return NAN;
  }
  switch (M->kind) {
    case ORC_LG1: {
      const double r = (y[0] - x[0]) / M->th[2];
      return -0.5 * (r * r);
    }
    case ORC_SV: {
      const double h = 0.5 * (y[0] * y[0]);
      return fma(-h, orc_exp(-x[0]), -0.5 * x[0]);
    }
    case ORC_LGD: {
      const int dx = M->dx, dy = M->dy;
      double ss = 0.0;
      for (int i = 0; i < dy; ++i) {
        double e = y[i];
        for (int c = 0; c < dx; ++c) e = fma(-M->H[i * dx + c], x[c], e);
        ss = fma(e, e, ss);
      }
      return -(ss * M->hr);
    }
    case ORC_BIN: return (x[0] == y[0]) ? 0.0 : -M->log3;
    case ORC_BCP: return y[0] * x[0] + (y[1] - y[0]) * x[1];
  }
  return NAN;
}

/* fixed-point weights of one island: mx = max lw, q_i = floor(2^40 exp(lw_i - mx))
 * (binary32 runs: the difference and the exponential in binary32) */
void orc_model_quantise(const orc_model* M, const double* lw, int32_t N, uint64_t* q, double* mx_out) {
  if (!M->f32) { orc_quantise(lw, N, q, mx_out); return; }
  float mx = -INFINITY;
  for (int32_t i = 0; i < N; ++i) if ((float)lw[i] > mx) mx = (float)lw[i];
  *mx_out = (double)mx;
  for (int32_t i = 0; i < N; ++i) {
    if (mx == -INFINITY) { q[i] = 0; continue; }
    const float e = orc_expf((float)lw[i] - mx);
    q[i] = (uint64_t)(e * 0x1p40f);
  }
}

/* ---------------- derivatives (score), plain double arithmetic ---------------- */

/* d x_0 / d theta_p for the initial draw: dx0[d*P + p] */
void orc_model_init_tangent(const orc_model* M, const double* z, double* dx0) {
  const int P = M->P, dx = M->dx;
  for (int i = 0; i < dx * P; ++i) dx0[i] = 0.0;
  if (M->kind == ORC_SV) {
    const double phi = M->th[1], sig = M->th[2];
    const double om = 1.0 - phi * phi;
    dx0[0] = 1.0;                                        /* d/d mu    */
    dx0[1] = z[0] * sig * phi / (om * sqrt(om));         /* d/d phi   */
    dx0[2] = z[0] / sqrt(om);                            /* d/d sigma */
  }
}

/* tangent of the mutation x = F(xp, z): dx[d*P+p] = sum_c dF_d/dxp_c dxp[c*P+p] + dF_d/dtheta_p */
void orc_model_prop_tangent(const orc_model* M, const double* xp, const double* dxp,
                            const double* z, double* dx) {
  const int P = M->P, dxn = M->dx;
  switch (M->kind) {
    case ORC_LG1:
      for (int p = 0; p < P; ++p) dx[p] = M->th[0] * dxp[p];
      dx[0] += xp[0];
      dx[1] += z[0];
      break;
    case ORC_SV: {
      const double mu = M->th[0], phi = M->th[1];
      for (int p = 0; p < P; ++p) dx[p] = phi * dxp[p];
      dx[0] += 1.0 - phi;
      dx[1] += xp[0] - mu;
      dx[2] += z[0];
      break;
    }
    case ORC_LGD:
      for (int i = 0; i < dxn; ++i) {
        for (int p = 0; p < P; ++p) {
          double acc = 0.0;
          for (int c = 0; c < dxn; ++c) acc += M->th[i * dxn + c] * dxp[c * P + p];
          dx[i * P + p] = acc;
        }
        for (int c = 0; c < dxn; ++c) dx[i * P + i * dxn + c] += xp[c];
      }
      break;
    default:
      for (int i = 0; i < dxn * P; ++i) dx[i] = 0.0;
  }
}

/* total derivative of the full log g_n (constant included) along a tangent:
 * dlw[p] = sum_d dlogg/dx_d * dx[d*P+p] + dlogg/dtheta_p */
void orc_model_logpot_tangent(const orc_model* M, const double* x, const double* dx,
                              const double* y, double* dlw) {
  const int P = M->P, dxn = M->dx;
  switch (M->kind) {
    case ORC_LG1: {
      const double sy = M->th[2];
      const double res = y[0] - x[0];
      const double gx = res / (sy * sy);
      for (int p = 0; p < P; ++p) dlw[p] = gx * dx[p];
      dlw[2] += res * res / (sy * sy * sy) - 1.0 / sy;
      break;
    }
    case ORC_SV: {
      const double gx = -0.5 + 0.5 * y[0] * y[0] * exp(-x[0]);
      for (int p = 0; p < P; ++p) dlw[p] = gx * dx[p];
      break;
    }
    case ORC_LGD: {
      const int dy = M->dy;
      double g[ORC_MAX_DX] = {0};
      for (int i = 0; i < dy; ++i) {
        double e = y[i];
        for (int c = 0; c < dxn; ++c) e -= M->H[i * dxn + c] * x[c];
        for (int c = 0; c < dxn; ++c) g[c] += M->H[i * dxn + c] * e / M->r;
      }
      for (int p = 0; p < P; ++p) {
        double acc = 0.0;
        for (int c = 0; c < dxn; ++c) acc += g[c] * dx[c * P + p];
        dlw[p] = acc;
      }
      break;
    }
    default:
      for (int p = 0; p < P; ++p) dlw[p] = 0.0;
  }
}
