// Internal interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_models.h"

namespace airpf {

// Kernel argument block of the persistent forward launch (one problem).
struct FwdArgs {
  ModelArgs mp;
  const double* y;            // [T*dy]
  int64_t T;
  int m, N, S, TP, c, lc, G, dy;
  uint64_t seed;
  double tau, cst_q;
  int shortcut_all;
  void* x1[2];                // Store*, resampled blocks, [m*N*DX] particle-major
  double* tree[2];            // [2m] pair-mean tree of island log-weights
  double* part[2];            // [(lc+1)*G] per-block log sum exp(2 LT) per level
  unsigned* bar;              // [G] grid-barrier flags, zero before the launch
  int* status;                // [1] 0 ok, 1 barrier timed out
  double* out_logz;           // [1]
  int32_t* tr_sstar;
  double* tr_enf;
  double* tr_lpost;
  int32_t* tr_anc;
  int32_t* tr_pi;
  unsigned long long* tr_digest;
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
hipError_t fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t st);
hipError_t launch_debug_eval(int which, int64_t n, const double* in, const uint32_t* in_u32, double* out,
                             double* out2, uint32_t* out_u32, hipStream_t st);

}  // namespace airpf
