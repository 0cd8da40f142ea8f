// FP64-state instantiations of the fused sparse step (the plain FP64 form).
#include "csr_step.hpp"

namespace fth {
template <>
int launch_csr_step<double>(const StepArgs<double>& a, const StepLaunch& L, int k, void* stream) {
    return a.tpart != nullptr ? launch_csr_step_traced<double>(a, L, k, stream)
                              : launch_csr_step_impl<double, false>(a, L, k, stream);
}

namespace dev {
__global__ void advance_kernel(int64_t* step_base, int64_t k) { step_base[0] += k; }
}  // namespace dev

int launch_advance(int64_t* step_base, int64_t k, void* stream) {
    hipLaunchKernelGGL(dev::advance_kernel, dim3(1), dim3(1), 0, static_cast<hipStream_t>(stream), step_base, k);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace fth
