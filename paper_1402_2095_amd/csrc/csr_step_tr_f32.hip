// FP32-state instantiations of the fused sparse step with trace partials.
#include "csr_step.hpp"

namespace fth {
template <>
int launch_csr_step_traced<float>(const StepArgs<float>& a, const StepLaunch& L, int k, void* stream) {
    return launch_csr_step_impl<float, true>(a, L, k, stream);
}
}  // namespace fth
