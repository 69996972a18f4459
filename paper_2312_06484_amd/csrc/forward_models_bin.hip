// Forward kernels of the binary toy HMM (its own translation unit).
#include "forward_impl.h"

namespace airpf {

hipError_t fwd_launch_bin(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<BIN>(L, a, plan);
}

}  // namespace airpf
