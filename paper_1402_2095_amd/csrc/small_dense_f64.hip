// FP64 instantiations of the persistent small-system kernel.
#include "small_dense.hpp"

namespace fth {
template <>
int launch_small_dense<double>(const StepArgs<double>& a, const StepLaunch& L, int K, size_t lds_bytes,
                               void* stream) {
    return launch_small_dense_impl<double>(a, L, K, lds_bytes, stream);
}
}  // namespace fth
