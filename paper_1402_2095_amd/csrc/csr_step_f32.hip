// FP32-state instantiations of the fused sparse step.
#include "csr_step.hpp"

namespace fth {
template <>
int launch_csr_step<float>(const StepArgs<float>& a, const StepLaunch& L, int k, void* stream) {
    return a.tpart != nullptr ? launch_csr_step_traced<float>(a, L, k, stream)
                              : launch_csr_step_impl<float, false>(a, L, k, stream);
}
}  // namespace fth
