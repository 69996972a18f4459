// Forward kernels of LG1, SV (instantiated here, one translation unit per model group).
#include "forward_impl.h"

namespace airpf {

hipError_t fwd_launch_lg1(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<LG1>(L, a, plan);
}
hipError_t fwd_batch_lg1(const BatchLaunch& L, int* cap) { return fwd_batch_model<LG1>(L, cap); }

hipError_t fwd_launch_sv(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<SV>(L, a, plan);
}
hipError_t fwd_batch_sv(const BatchLaunch& L, int* cap) { return fwd_batch_model<SV>(L, cap); }

}  // namespace airpf
