// FP32 instantiations of the persistent small-system kernel.
#include "small_dense.hpp"

namespace fth {
template <>
int launch_small_dense<float>(const StepArgs<float>& a, const StepLaunch& L, int K, size_t lds_bytes, void* stream) {
    return launch_small_dense_impl<float>(a, L, K, lds_bytes, stream);
}
}  // namespace fth
