// FP64-state instantiations of the fused sparse step with trace partials.
#include "csr_step.hpp"

namespace fth {
template <>
int launch_csr_step_traced<double>(const StepArgs<double>& a, const StepLaunch& L, int k, void* stream) {
    return launch_csr_step_impl<double, true>(a, L, k, stream);
}
}  // namespace fth
