// FP32-state instantiations of the fused sparse step.
#include "csr_step.hpp"

namespace fth {
template <>
int launch_csr_step<float>(const CsrStepArgs<float>& a, int ns, int rpt, int k, int block,
                           int64_t pair_tiles, void* stream) {
    return launch_csr_step_impl<float>(a, ns, rpt, k, block, pair_tiles, stream);
}
}  // namespace fth
