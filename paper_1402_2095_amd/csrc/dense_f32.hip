// Split-BF16x3 dense force GEMM, the bf16 split kernels and the FP32 dense
// epilogue instantiations.
#include "dense.hpp"

namespace fth {
namespace dev {

__global__ void split_bf16_kernel(const float* __restrict__ m, uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                  int64_t count) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x) {
        const float x = m[i];
        const uint16_t h = bf16_bits(x);
        hi[i] = h;
        lo[i] = bf16_bits(x - bf16_value(h));
    }
}

__global__ void qt_from_q_kernel(const float* __restrict__ q, uint16_t* __restrict__ qt, int64_t N, int32_t R) {
    const int64_t total = N * R;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
        put_qt(qt, t / R, t % R, R, q[t]);
}

}  // namespace dev

int launch_gemm_bf16x3(const DenseGemmArgs& g, void* stream) {
    if (g.rows_pad % 128 != 0 || g.kslice % 64 != 0 || g.kslice * g.ksplit != g.rows_pad) return -3;
    const int64_t grid = (g.rows_pad / 128) * g.ksplit;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    switch (g.R) {
        case 16: hipLaunchKernelGGL(dev::gemm_bf16x3_kernel<1>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        case 32: hipLaunchKernelGGL(dev::gemm_bf16x3_kernel<2>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        case 64: hipLaunchKernelGGL(dev::gemm_bf16x3_kernel<4>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        case 128: hipLaunchKernelGGL(dev::gemm_bf16x3_kernel<8>, dim3(unsigned(grid)), dim3(256), 0, s, g); break;
        default: return -2;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_split_bf16(const float* m, uint16_t* hi, uint16_t* lo, int64_t count, void* stream) {
    hipLaunchKernelGGL(dev::split_bf16_kernel, dim3(4096), dim3(256), 0, static_cast<hipStream_t>(stream), m, hi, lo,
                       count);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_qt_from_q(const float* q, uint16_t* qt, int64_t N, int64_t rows_pad, int32_t R, void* stream) {
    (void)rows_pad;
    hipLaunchKernelGGL(dev::qt_from_q_kernel, dim3(2048), dim3(256), 0, static_cast<hipStream_t>(stream), q, qt, N, R);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <>
int launch_dense_epilogue<float>(const StepArgs<float>& a, const StepLaunch& L, int k, void* stream) {
    return launch_dense_epilogue_impl<float>(a, L, k, stream);
}

}  // namespace fth
