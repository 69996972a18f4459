// Forward kernels of LGD<2>, LGD<3> (instantiated here, one translation unit per model group).
#include "forward_impl.h"

namespace airpf {

hipError_t fwd_launch_lgd2(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<LGD<2>>(L, a, plan);
}
hipError_t fwd_batch_lgd2(const BatchLaunch& L, int* cap) { return fwd_batch_model<LGD<2>>(L, cap); }

hipError_t fwd_launch_lgd3(const FwdLaunch& L, const FwdArgs& a, FwdPlan* plan) {
  return fwd_launch_model<LGD<3>>(L, a, plan);
}
hipError_t fwd_batch_lgd3(const BatchLaunch& L, int* cap) { return fwd_batch_model<LGD<3>>(L, cap); }

}  // namespace airpf
