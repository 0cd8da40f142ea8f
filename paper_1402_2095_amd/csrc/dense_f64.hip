// FP64 dense force GEMM (plain FP64 form) and the FP64 dense epilogue.
#include "dense.hpp"

namespace fth {

int launch_gemm_f64(const DenseGemmArgs& g, void* stream) {
    if (g.rows_pad % 64 != 0 || g.kslice % 16 != 0 || g.kslice * g.ksplit != g.rows_pad) return -3;
    const int64_t grid = (g.rows_pad / 64) * g.ksplit;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    switch (g.R) {
        case 16: hipLaunchKernelGGL(dev::gemm_f64_kernel<1>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        case 32: hipLaunchKernelGGL(dev::gemm_f64_kernel<2>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        case 64: hipLaunchKernelGGL(dev::gemm_f64_kernel<4>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        case 128: hipLaunchKernelGGL(dev::gemm_f64_kernel<8>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        default: return -2;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <>
int launch_dense_epilogue<double>(const StepArgs<double>& a, const StepLaunch& L, int k, void* stream) {
    return launch_dense_epilogue_impl<double>(a, L, k, stream);
}

}  // namespace fth
