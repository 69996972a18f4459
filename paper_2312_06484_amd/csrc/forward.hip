// Host side of the AIRPF forward launches: dispatch on the model to the
// per-model translation units (forward_models_*.hip), the batched-launch
// queries, and small helper kernels.  The kernel itself is in forward_impl.h.
#include "forward_impl.h"

namespace airpf {

hipError_t launch_forward(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  switch (L.kind) {
    case 0: return fwd_launch_lg1(L, a, plan);
    case 1: return fwd_launch_sv(L, a, plan);
    case 3: return fwd_launch_bin(L, a, plan);
    case 4: return fwd_launch_bcp(L, a, plan);
    case 2:
      switch (L.dx) {
        case 2: return fwd_launch_lgd2(L, a, plan);
        case 3: return fwd_launch_lgd3(L, a, plan);
        case 4: return fwd_launch_lgd4(L, a, plan);
        case 8: return fwd_launch_lgd8(L, a, plan);
      }
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ batched launches

int forward_ppt(int kind, int dx, int n, bool plain) {
  const int DX = kind == 2 ? dx : 1;
  // a forward-only batch of a 1-D model whose teams would span two waves
  // takes eight particles per lane instead (teams inside one wave; results
  // do not depend on it): 294 -> 255 ms on the 64-proposal SV batch.  With
  // scores the recorded variants lose occupancy at eight, so they keep four.
  if (plain && DX == 1 && n > 256 && n <= 1024) return 8;
  if (DX % 4 == 0) {
    if (n <= 256) return 1;
    if (n <= 512) return 2;
  } else if (DX % 2 == 0) {
    if (n <= 512) return 2;
  }
  return n <= 1024 ? 4 : 8;
}

size_t forward_smem(int fp64, int ppt, int dx, int c, int G, size_t resident, int multinomial) {
  // multinomial draws also keep each team's cumulative weights (16-byte aligned)
  return fwd_smem_bytes(fp64 ? 8 : 4, ppt, dx, c, G) + resident +
         (multinomial ? 16 + 8 * size_t(kBlock) * ppt : 0);
}

size_t forward_resident_bytes(int fp64, int dx, int c, int N) { return fwd_res_bytes(fp64 ? 8 : 4, dx, c, N); }

static hipError_t batch_fwd(const BatchLaunch& L, int* cap) {
  switch (L.kind) {
    case 0: return fwd_batch_lg1(L, cap);
    case 1: return fwd_batch_sv(L, cap);
    case 2:
      switch (L.dx) {
        case 2: return fwd_batch_lgd2(L, cap);
        case 3: return fwd_batch_lgd3(L, cap);
        case 4: return fwd_batch_lgd4(L, cap);
        case 8: return fwd_batch_lgd8(L, cap);
      }
  }
  return hipErrorInvalidValue;
}

hipError_t forward_batch_capacity(const BatchLaunch& L, int* blocks) { return batch_fwd(L, blocks); }

hipError_t launch_forward_batch(const BatchLaunch& L) { return batch_fwd(L, nullptr); }

// ------------------------------------------------------------ small helpers

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

hipError_t fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  int64_t blocks = (n_words + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  fill_u32_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st>>>(static_cast<uint32_t*>(p), v, n_words);
  return hipGetLastError();
}

__global__ void debug_eval_kernel(int which, int64_t n, const double* in, const uint32_t* in_u32, double* out,
                                  double* out2, uint32_t* out_u32) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  switch (which) {
    case 0: out[i] = dexp(in[i]); break;
    case 1: out[i] = dlog(in[i]); break;
    case 2: { double c, s; cossin_2pi(in[i], c, s); out[i] = c; out2[i] = s; break; }
    case 3: { double z0, z1; box_muller(in_u32[2 * i], in_u32[2 * i + 1], z0, z1); out[i] = z0; out2[i] = z1; break; }
    case 4: {
      uint32_t w[4] = {in_u32[6 * i + 2], in_u32[6 * i + 3], in_u32[6 * i + 4], in_u32[6 * i + 5]};
      philox4x32_10(w, Key{in_u32[6 * i], in_u32[6 * i + 1]});
      for (int r = 0; r < 4; ++r) out_u32[4 * i + r] = w[r];
      break;
    }
    // binary32 counterparts (inputs and outputs widened to double)
    case 5: out[i] = fexp(static_cast<float>(in[i])); break;
    case 6: out[i] = flog(static_cast<float>(in[i])); break;
    case 7: { float c, s; fcossin_2pi(static_cast<float>(in[i]), c, s); out[i] = c; out2[i] = s; break; }
    case 8: { float z0, z1; box_muller(in_u32[2 * i], in_u32[2 * i + 1], z0, z1); out[i] = z0; out2[i] = z1; break; }
  }
}

hipError_t launch_debug_eval(int which, int64_t n, const double* in, const uint32_t* in_u32, double* out,
                             double* out2, uint32_t* out_u32, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  debug_eval_kernel<<<dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st>>>(which, n, in, in_u32, out,
                                                                                       out2, out_u32);
  return hipGetLastError();
}

}  // namespace airpf
