// FP32-state instantiations of the fused sparse step.
#include "csr_step.hpp"

namespace fth {
template <>
int launch_csr_step<float>(const StepArgs<float>& a, const StepLaunch& L, int k, void* stream) {
    return launch_csr_step_impl<float>(a, L, k, stream);
}
}  // namespace fth
