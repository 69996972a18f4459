// Forward kernels of the word-driven models: the binary toy HMM and the Beta
// change-point model (their own translation unit).
#include "forward_impl.h"

namespace airpf {

hipError_t fwd_launch_bin(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<BIN>(L, a, plan);
}

hipError_t fwd_launch_bcp(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<BCP>(L, a, plan);
}

}  // namespace airpf
