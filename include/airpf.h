/*
 * airpf.h -- C ABI of the MI355X (gfx950) AIRPF library.
 *
 * The augmented island resampling particle filter (Algorithm 1 of Heine,
 * "Augmented Island Resampling Particle Filters for Particle Markov Chain
 * Monte Carlo", arXiv:2312.06484, Section 2) run on one GPU: m = 2^S
 * islands of N particles each (the paper's filters of M particles), internal
 * resampling every step, and S butterfly interaction stages switched on
 * adaptively by the effective number of filters (ENF < tau).  A call returns
 * the marginal-likelihood estimate log Zhat = log gamma^N_T(1) (the estimator
 * defined after Algorithm 1, unbiased by Theorem 1), which a particle
 * marginal Metropolis-Hastings step consumes once per iteration.
 *
 * Problem statement (Section 1.2): a parameterised hidden Markov model
 * X_0 ~ pi_0, X_n | X_{n-1} ~ K(X_{n-1}, .), Y_n | X_n ~ G(X_n, .) with
 * observations y_0 .. y_{T-1} fixed; the estimate is of
 * p(y_0..y_{T-1} | theta) = gamma_T(1).
 *
 * Conventions
 *   - N is the number of particles PER ISLAND (the paper's M); m is the
 *     number of islands and must be a power of two; 1 <= N <= 2048;
 *     m <= 65536 on one device (larger m: AIRPF_E_UNSUPPORTED).
 *   - Arrays are plain host pointers unless a flag says otherwise; the
 *     library copies what it needs and keeps no pointer after returning.
 *   - The context owns all device workspaces; they grow on demand and are
 *     reused by later calls on the same context.  One context per host
 *     thread; calls on one context are serialised on its stream.
 *   - Every call is deterministic: the same inputs, seed and options give
 *     bit-identical outputs.  All random numbers are Philox4x32-10 draws at
 *     fixed counters: key = seed, counter = (c0, island, step, tag << 24 | sub).
 *   - Errors: every function returns an airpf_status.  On
 *     AIRPF_E_DOMAIN (theta outside its support) *log_z_out is -inf; on other
 *     errors outputs are set to NaN where they exist.  A run in which every
 *     island's weight vanishes is a valid estimate: AIRPF_OK, log Zhat = -inf.
 *   - Observations are checked for NaN and infinities: host arrays before
 *     anything is launched, device-resident ones (AIRPF_FLAG_Y_ON_DEVICE)
 *     by the kernels as they read them; either way such a call returns
 *     AIRPF_E_INVALID_ARG with NaN outputs (per item in a batch).
 *   - Tiling never changes a result.  Environment switches, read at each
 *     call, only change how the work is laid out: AIRPF_MAX_BLOCKS=<n> caps
 *     the blocks of a single-problem launch, AIRPF_PIPELINE=0 switches off
 *     the pipelined forward kernel (worker waves beside a control wave),
 *     AIRPF_TILER="alpha,beta" sets the batch tiler's cost ratio beta/alpha.
 *     AIRPF_WORKSPACE_CAP=<bytes> caps every device buffer a context grows
 *     (a call that needs more returns AIRPF_E_NOMEM, as a failed allocation
 *     does).
 */
#ifndef AIRPF_H
#define AIRPF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AIRPF_OK = 0,
  AIRPF_E_INVALID_ARG = 1, /* bad size, NaN/Inf input, wrong d_theta, null pointer */
  AIRPF_E_DOMAIN = 2,      /* theta outside the model's parameter space */
  AIRPF_E_NOMEM = 3,       /* device workspace could not be allocated */
  AIRPF_E_DEVICE = 4,      /* a HIP call or a kernel failed */
  AIRPF_E_UNSUPPORTED = 5, /* valid request the library does not implement */
  AIRPF_E_TOO_LARGE = 6    /* airpf_run_noalloc: the workspace exceeds the fixed scratch */
} airpf_status;

/* State-space models (concrete instances of the HMM of Section 1.2).
 *  AIRPF_LG1  x_0 ~ N(0,1), x' = a x + sx e, y = x + sy v;  theta = (a, sx, sy),
 *             sx > 0, sy > 0.  d_x = d_y = 1, no constants.
 *  AIRPF_SV   x_0 ~ N(mu, sigma^2/(1-phi^2)), x' = mu + phi (x - mu) + sigma e,
 *             y = exp(x/2) v;  theta = (mu, phi, sigma), |phi| < 1, sigma > 0.
 *  AIRPF_LGD  x_0 ~ N(0, p0 I), x' = A x + sqrt(q) e, y = H x + sqrt(r) v;
 *             theta = vec(A) row-major (d_x^2 entries); consts =
 *             (q, r, p0, H row-major d_y x d_x), q, r, p0 > 0;
 *             d_x in {2, 3, 4, 8}, 1 <= d_y <= 8.
 *  AIRPF_BIN  the binary toy HMM of the exact-variance example (Section 4.1):
 *             x_0 uniform on {0, 1}, x' = 1 - x with probability 1/4,
 *             g(y | x) = 3/4 if y == x else 1/4 (observations 0 or 1; any
 *             other value never matches);  no parameters (d_theta = 0, theta
 *             may be NULL), d_x = d_y = 1.  Forward only (airpf_run,
 *             airpf_run_noalloc); its states are 0/1 and always kept in
 *             double (the precision option has no effect).  airpf_score and
 *             airpf_run_batch return AIRPF_E_UNSUPPORTED.
 *  AIRPF_BCP  the Beta change-point model of the change-point experiment
 *             (Section 4.2): a rate r_0 ~ Beta(alpha, beta); r' = r with
 *             probability 1 - p, else a fresh Beta(alpha, beta) draw;
 *             y_n = (k_n, n_n) counts (row-major, d_y = 2) with
 *             g = r^k (1 - r)^(n - k) (no binomial coefficient: a constant of
 *             the data).  theta = (p), 0 <= p <= 1 (else AIRPF_E_DOMAIN);
 *             consts = (alpha, beta), integers >= 1 with alpha + beta <= 7;
 *             d_x = 2 (the state is (log r, log(1 - r))).  Forward only, as
 *             AIRPF_BIN (states in double; score and batch UNSUPPORTED). */
typedef enum { AIRPF_LG1 = 0, AIRPF_SV = 1, AIRPF_LGD = 2, AIRPF_BIN = 3, AIRPF_BCP = 4 } airpf_model_kind;

typedef struct {
  int32_t kind;          /* airpf_model_kind */
  int32_t dx, dy;        /* state and observation dimensions */
  const double* consts;  /* model constants (AIRPF_LGD, AIRPF_BCP), host memory */
  int32_t n_consts;
} airpf_model;

typedef enum { AIRPF_SYSTEMATIC = 0, AIRPF_MULTINOMIAL = 1 } airpf_resampling;
typedef enum { AIRPF_FP32 = 0, AIRPF_FP64 = 1 } airpf_precision;
typedef enum { AIRPF_PATHSPACE = 0, AIRPF_PATHWISE = 1 } airpf_score_mode;

#define AIRPF_FLAG_Y_ON_DEVICE 1u /* y is a device pointer (already resident in HBM) */
#define AIRPF_FLAG_AUTOTUNE 2u    /* airpf_run_batch: measure the tiler's cost ratio for this
                                     batch shape (see airpf_run_batch) */

typedef struct {
  double tau;         /* ENF threshold of the adaptation line of Algorithm 1:
                         stage s interacts iff ENF_{n,s} < tau.  tau <= 1/m never
                         interacts (independent filters), tau > 1 always does. */
  int32_t resampling; /* airpf_resampling of the internal (within-island) step:
                         AIRPF_SYSTEMATIC everywhere; AIRPF_MULTINOMIAL (slot j
                         takes the first particle whose cumulative fixed-point
                         weight exceeds its own uniform draw on [0, Q)) in
                         airpf_run, airpf_run_batch and airpf_score (the
                         reverse pass sorts each step's slots by ancestor);
                         any other value is AIRPF_E_INVALID_ARG */
  int32_t precision;  /* precision of the particles: AIRPF_FP64 everything in
                         double; AIRPF_FP32 binary32 state, normals, model
                         and fixed-point weights (own single-precision exp,
                         log, sin/cos, Box-Muller on the same draws), island
                         log-weights and log Zhat in double either way */
  int32_t score_mode; /* airpf_score_mode (airpf_score, airpf_run_batch with scores) */
  int32_t ckpt_every; /* checkpoint interval of the score's recomputation (0: auto) */
  uint32_t flags;     /* AIRPF_FLAG_* */
  double resample_ess; /* 0: every island resamples internally at every step
                          (Algorithm 1).  rho > 0: adaptive internal
                          resampling (the remark after Algorithm 1 that the
                          analysis does not need a resampling at every step):
                          an island resamples (systematically) iff the ESS of
                          its fixed-point weights, truncated to their top 20
                          of 40 bits, is below rho * N; otherwise its
                          particles carry their weights into the next
                          weighting, and the island weight is updated with
                          those incoming weights.  airpf_run only (double
                          states, systematic; score, batch and
                          airpf_run_noalloc return AIRPF_E_UNSUPPORTED);
                          negative or NaN: AIRPF_E_INVALID_ARG */
  int32_t arity;       /* r of the island interactions (Section 2 allows
                          m = r^S for any r >= 2): 0 or 2, the pairs of
                          Algorithm 1; 4, 8, 16, ... (powers of two, m a
                          power of r): S / log2(r) stages, stage s grouping
                          the r islands whose base-r digits differ only in
                          digit s-1 (A_s = I (x) (1/r)1_r (x) I); when it
                          interacts every member takes the group mean
                          weight and each island's block is drawn from its
                          group with probability W_d / sum W (the first
                          member whose running sum of exp(L_d - max L)
                          exceeds u times the total, u the island's uniform
                          of the stage).  The ENF of stage s is that of the
                          weights after the stages below.  airpf_run and
                          airpf_run_noalloc (the score and the batch return
                          AIRPF_E_UNSUPPORTED); other values, or m not a
                          power of r: AIRPF_E_INVALID_ARG */
} airpf_options;

/* Optional per-call trace, host arrays (any may be NULL). */
typedef struct {
  int32_t* sstar;    /* [T] interacting stages per step (0 at the last step) */
  double* enf;       /* [T*(S+1)] ENF_{n,s}; entries not evaluated are NaN */
  double* lpost;     /* [T*m] island log-weights after each weighting */
  int32_t* anc;      /* [(T-1)*m*N] within-island ancestors */
  int32_t* pi;       /* [(T-1)*m] island source map after the stages */
  uint64_t* digest;  /* [2*T] order-free digests of ancestors and island maps */
  double* fmean;     /* [T*m] island k's estimate of the filtering mean of the first
                        state coordinate after step n's weighting, sum_i q_i x_i / Q
                        with the fixed-point weights q (the filter's estimate of
                        E[x_n | y_0..y_n] is sum_k exp(lpost_k) fmean_k / sum_k exp(lpost_k)) */
} airpf_trace;

typedef struct airpf_ctx airpf_ctx;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t, or NULL for the default stream). */
airpf_status airpf_ctx_create(int device, void* hip_stream, airpf_ctx** out);
airpf_status airpf_ctx_destroy(airpf_ctx* ctx);

/* Forward filter: *log_z_out = log Zhat(theta).
 *   theta [d_theta] host; y [T*dy] row-major (host, or device with
 *   AIRPF_FLAG_Y_ON_DEVICE); m islands (power of two), N per island. */
airpf_status airpf_run(airpf_ctx* ctx, const airpf_model* model, const double* theta,
                       int32_t d_theta, const double* y, int64_t T, int32_t m, int32_t N,
                       uint64_t seed, const airpf_options* opt, double* log_z_out,
                       airpf_trace* trace);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): airpf_run
 * without a trace, whose workspaces (resampled states, island tree, ENF
 * records, barrier flags, the uploaded observations when y is on the host)
 * are carved from a fixed device array of 64 MiB that the library holds on
 * every device it runs on until the process ends.  The call makes no
 * hipMalloc, hipFree or other allocating call; the context must have been
 * created beforehand (airpf_ctx_create resolves the array's address on its
 * device).  A request whose workspace exceeds the array returns
 * AIRPF_E_TOO_LARGE (*log_z_out NaN), e.g. m*N*d_x*bytes-per-state above
 * about 32 MiB.  Calls on one device share the array: calls that overlap in
 * time on one device (several contexts or streams) race; calls serialised on
 * one stream do not.  Results are bit-identical to airpf_run's. */
airpf_status airpf_run_noalloc(airpf_ctx* ctx, const airpf_model* model, const double* theta,
                               int32_t d_theta, const double* y, int64_t T, int32_t m, int32_t N,
                               uint64_t seed, const airpf_options* opt, double* log_z_out);

/* Score: *log_z_out = log Zhat(theta) (the same value airpf_run returns for
 * the same arguments) and grad_out[d_theta] = an estimate of
 * d log Z / d theta with the noise and every discrete decision of the run
 * held fixed and the fixed-point weights read as exact (the derivative is
 * not part of the paper; it is the score a gradient-based PMCMC proposal
 * consumes).  opt->score_mode picks the estimator:
 *   AIRPF_PATHSPACE  the final-weight average over final particles of the
 *                    derivative of the summed log g along each particle's
 *                    ancestral path (consistent for d log Z / d theta);
 *   AIRPF_PATHWISE   the derivative of the run's own log Zhat (the
 *                    estimator of Algorithm 1's gamma^N_T(1)) with the
 *                    ancestors, island maps and stage counts fixed.
 * opt->ckpt_every = K: the forward pass keeps a checkpoint every K steps and
 * the reverse pass recomputes the particle history one segment of K steps at
 * a time (K = 0: the whole history is kept when it fits the workspace
 * budget, otherwise K = ceil(sqrt(T))).  Supported: N <= 1024 (LG1, SV),
 * N <= 512 (LGD); any other score_mode is AIRPF_E_INVALID_ARG.  grad_out is
 * host memory.  A run in
 * which every island's weight vanishes returns AIRPF_OK, log Zhat = -inf and
 * a zero score (no reverse pass is made; airpf_run_batch does the same per
 * problem). */
airpf_status airpf_score(airpf_ctx* ctx, const airpf_model* model, const double* theta,
                         int32_t d_theta, const double* y, int64_t T, int32_t m, int32_t N,
                         uint64_t seed, const airpf_options* opt, double* log_z_out,
                         double* grad_out, airpf_trace* trace);

/* One problem of a batch: its own parameter, data, sizes and seed. */
typedef struct {
  const double* theta;   /* [d_theta], host */
  int32_t d_theta;
  const double* y;       /* [T*dy], host (device with AIRPF_FLAG_Y_ON_DEVICE) */
  int64_t T;
  int32_t m, N;          /* islands (power of two), particles per island */
  uint64_t seed;
} airpf_problem;

/* Batched multi-theta call (e.g. the proposals of many PMMH chains): every
 * problem of the batch runs in ONE cooperative persistent launch, each on a
 * sub-grid of blocks of its own chosen by the library's tiler (the slowest
 * problem's modelled time is minimised under the device's co-residency);
 * with want_score the reverse passes are batched too, segment by segment.
 * All problems share `model` and `opt`; T, m, N, theta and seed may differ.
 * Outputs: log_z_out[B]; grad_out[B*d_theta] (packed in problem order) when
 * want_score; item_status[B] per problem (an invalid problem is reported
 * there and skipped, the others still run).  Each item's results are
 * bit-identical to the same problem run alone with airpf_run / airpf_score.
 * The call's return value is AIRPF_OK unless the batch as a whole failed.
 * Tiling: a problem's time is modelled as steps * (1 + r * passes) (a pass
 * is one round of island work of a block); with AIRPF_FLAG_AUTOTUNE in
 * opt->flags the library times the tilings of several r on the first (up to)
 * 32 steps of every problem, for four and for eight particles per lane when
 * a forward-only systematic batch of a one-dimensional model allows both
 * (islands of at most 1024 particles), keeps the fastest and caches it in
 * the context for batches of the same shape (model, precision, score,
 * resampling, and every problem's T, m, N), so only the first such call
 * pays for the probes; with the environment variable AIRPF_TUNE_CACHE
 * naming a file, the measured choices are also appended there and read
 * back by later processes (one text line "<shape key, hex> <ratio>
 * <particles per lane>" per measurement).
 * Tiling never changes results. */
airpf_status airpf_run_batch(airpf_ctx* ctx, const airpf_model* model, int32_t B,
                             const airpf_problem* probs, const airpf_options* opt,
                             int32_t want_score, double* log_z_out, double* grad_out,
                             airpf_status* item_status);

const char* airpf_status_str(airpf_status s);

/* Device time, in milliseconds, of the filter kernel of the last successful
 * call on this context: HIP events recorded on the context's stream right
 * before and after the persistent launch. */
airpf_status airpf_ctx_last_kernel_ms(airpf_ctx* ctx, double* ms);

/* Diagnostics used by the tests: evaluate the library's own device
 * implementations of exp, log, (cos, sin)(2 pi v), Box-Muller and Philox on
 * host arrays of length n (outputs host).  `which`: 0 exp, 1 log, 2 cossin
 * (out2 gets sin), 3 Box-Muller of word pairs (in_u32 pairs, out/out2),
 * 4 Philox (in_u32 = 6 words per item: key0, key1, c0..c3; out_u32 4 per
 * item); 5, 6, 7, 8: the binary32 exp, log, cossin and Box-Muller (inputs
 * rounded to binary32, results widened to double). */
airpf_status airpf_debug_eval(airpf_ctx* ctx, int32_t which, int64_t n, const double* in,
                              const uint32_t* in_u32, double* out, double* out2,
                              uint32_t* out_u32);

#ifdef __cplusplus
}
#endif
#endif
