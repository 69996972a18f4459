// Forward kernels of LGD<4> (instantiated here, one translation unit per model group).
#include "forward_impl.h"

namespace airpf {

hipError_t fwd_launch_lgd4(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<LGD<4>>(L, a, plan);
}
hipError_t fwd_batch_lgd4(const BatchLaunch& L, int* cap) { return fwd_batch_model<LGD<4>>(L, cap); }

}  // namespace airpf
