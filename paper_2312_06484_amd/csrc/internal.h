// Internal interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_models.h"

namespace airpf {

// copies of the pipelined kernel's level-1 record ring: every block writes
// its record into each copy and reads the copy of its own XCD (blocks are
// dealt to the eight XCDs round-robin), so the polls of the 256 blocks are
// spread over eight sets of lines instead of converging on one
constexpr int kRingCopies = 8;
constexpr int kRingSlots = 5;               // steps of level-1 records the ring holds

// Kernel argument block of the persistent forward launch (one problem).
struct FwdArgs {
  ModelArgs mp;
  const double* y;            // [T*dy]
  int64_t T;
  int m, N, S, TP, c, lc, G, dy;
  uint64_t seed;
  double tau, cst_q;
  int shortcut_all;           // tau > 1: every stage interacts
  int no_interaction;         // tau <= 1/(2m): no stage can interact (ENF >= 1/m)
  int res_lds;                // 1: a block also keeps its resampled states in LDS (one copy per step parity)
  int multinomial;            // internal resampling: 0 systematic, 1 multinomial (N independent draws)
  void* x1[2];                // Store*, resampled blocks, [m*N*DX] particle-major
  double* tree[2];            // [2m] pair-mean tree of island log-weights
  double* part[2];            // [(lc+1)*3*G] per level: the blocks' ENF records (E, a, b)
  unsigned* bar;              // [G] grid-barrier flags, zero before the launch
  int* status;                // [1] 0 ok, 1 barrier timed out
  double* ring;               // pipelined kernel: [kRingCopies][kRingSlots][E, a, b][G] level-1 ENF records, NaN before the launch
  int check_y;                // 1: the observations came from the caller's device memory unchecked
  int* bad_y;                 // [1] set to 1 when such an observation is NaN or infinite
  double* out_logz;           // [1]
  int32_t* tr_sstar;
  double* tr_enf;
  double* tr_lpost;
  int32_t* tr_anc;
  int32_t* tr_pi;
  unsigned long long* tr_digest;
  double* tr_fmean;           // [T*m] island weighted means of x[0] after each weighting
  // adaptive internal resampling (ess_frac > 0; the serial kernel of its own):
  // an island resamples iff the ESS of its 20-bit-truncated fixed-point
  // weights is below ess_frac * N; otherwise its particles carry log q (lc1)
  // and the island log Q - log N (dq1) into the next weighting; both by step
  // parity, [m*N] and [m]
  double ess_frac;
  double log_N;
  // r-ary interactions, r = 2^arity_log2 (0 or 1: the pairs of Algorithm 1):
  // stage t groups the r islands that differ only in base-r digit t-1
  int arity_log2;
  double* lc1[2];
  double* dq1[2];
  // ---- what the score needs (all optional) ----
  int64_t n0, n1;             // steps [n0, n1) of this launch (0, T for a plain run)
  int replay_pi;              // 1: island maps from tr_pi, no cascade, no island weights
  const int32_t* sstar_in;    // replay (optional): s* of each step; the barrier before step n
                              // is a block barrier when s*_{n-1} and s*_{n-2} are <= log2 c
  int64_t ck_every;           // checkpoint interval K (0: none)
  void* ck_x;                 // Store*, [ceil(T/K)][m*N*DX] state entering step c*K
  double* ck_L;               // [ceil(T/K)][m] island log-weights entering step c*K
  int ck_in;                  // 1: step n0 starts from checkpoint n0/K (else n0 == 0: initial draw)
  double* tr_lpre;            // [T*m] island log-weights entering each weighting
  void* rec_x;                // Store*, [(n1-n0)][m*N*DX] state entering each weighting
  uint16_t* rec_anc;          // [(n1-n0)][m*N] within-island ancestors
};


// Kernel argument block of the reverse (adjoint) launch over steps
// [n_lo, n_hi), processed from n_hi - 1 down to n_lo.
struct BwdArgs {
  ModelArgs mp;
  const double* y;
  int64_t T;
  int m, N, S, TP, c, lc, G, dy;
  uint64_t seed;
  double log_mN, c_log;       // log(m N) and the constant of log g
  double log_N;               // log N
  int pathwise;               // seed: 0 path-space (descendants' final weights), 1 pathwise (island weights)
  int multinomial;            // 1: a step's ancestors are in no slot order (multinomial internal
                              // resampling); the slots are sorted by ancestor before the runs are taken
  double* nu[2];              // pathwise: [m] d log Zhat / d (island log-weight after step n's weighting), by step parity
  const double* logz;         // [1] log Zhat of the forward run (device)
  int64_t n_lo, n_hi;
  const void* rec_x;          // Store*, [(n_hi-n_lo)][m*N*DX], index n - n_lo
  const uint16_t* rec_anc;    // [(n_hi-n_lo)][m*N]
  const int32_t* pi_all;      // [T*m] island source maps
  const int32_t* sstar_all;   // [T] interacting stages
  const double* lpre_all;     // [T*m] island log-weights entering each weighting
  void* lam[2];               // Store*, [m*N*DX] adjoint of the state, by step parity
  void* del[2];               // Store*, [m*N] descendant final-weight mass, by step parity
  double* gisl;               // [m*P] per-island gradient sums (accumulated across launches)
  unsigned* bar;
  int* status;
};

struct FwdLaunch {
  int kind, dx, fp64;
  int num_cus, max_blocks;
  int plan_only;
  hipStream_t stream;
};

struct FwdPlan {
  int ppt, tp, G, c;
  size_t smem;
};

hipError_t launch_forward(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan);
// max_blocks_out != nullptr: only report how many blocks can be co-resident
hipError_t launch_backward(const FwdLaunch& L, const BwdArgs& a, int* max_blocks_out);
hipError_t launch_island_grad_sum(const double* gisl, int m, int P, double* out, hipStream_t st);
hipError_t fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t st);

// ---- batched launches: one cooperative grid, block b runs local block
// bmap[b].y of problem bmap[b].x ----
struct BatchLaunch {
  int kind, dx, fp64;
  int n_max;                  // largest N of the batch
  int ppt = 0;                // forward: particles per lane of every item (forward_ppt of the batch)
  int num_cus;
  size_t smem;                // dynamic LDS per block
  int blocks;                 // total blocks
  const void* probs;          // device array of FwdArgs or BwdArgs
  const int2* bmap;           // device [blocks]
  hipStream_t stream;
  int plain = 0;              // forward: every item plain (no traces, records, replay or checkpoints)
  int multinomial = 0;        // forward: multinomial internal resampling (every item's FwdArgs says so too)
};
int forward_ppt(int kind, int dx, int n_max, bool plain);
// dynamic LDS of a forward block with c islands of a G-block problem, plus
// `resident` bytes of LDS-resident resampled states (forward_resident_bytes)
size_t forward_smem(int fp64, int ppt, int dx, int c, int G, size_t resident, int multinomial = 0);
// LDS for both parity copies of a block's resampled states, or 0 when they
// exceed the budget kResidentBudget (the states then come from HBM only)
size_t forward_resident_bytes(int fp64, int dx, int c, int N);
constexpr size_t kResidentBudget = 32768;
hipError_t forward_batch_capacity(const BatchLaunch& L, int* blocks);   // co-resident blocks at L.smem
hipError_t launch_forward_batch(const BatchLaunch& L);
int backward_ppt(int kind, int dx, int n_max);                          // 0: unsupported
size_t backward_smem(int fp64, int ppt, int dx);
hipError_t backward_batch_capacity(const BatchLaunch& L, int* blocks);
hipError_t launch_backward_batch(const BatchLaunch& L);
hipError_t launch_debug_eval(int which, int64_t n, const double* in, const uint32_t* in_u32, double* out,
                             double* out2, uint32_t* out_u32, hipStream_t st);

}  // namespace airpf
