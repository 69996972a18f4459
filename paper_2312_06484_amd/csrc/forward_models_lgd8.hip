// Forward kernels of LGD<8> (instantiated here, one translation unit per model group).
#include "forward_impl.h"

namespace airpf {

hipError_t fwd_launch_lgd8(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<LGD<8>>(L, a, plan);
}
hipError_t fwd_batch_lgd8(const BatchLaunch& L, int* cap) { return fwd_batch_model<LGD<8>>(L, cap); }

}  // namespace airpf
