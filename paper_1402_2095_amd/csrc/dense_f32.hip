// Split-BF16x3 dense force GEMM, the bf16 split kernels and the FP32 dense
// epilogue instantiations.
#include "dense.hpp"

namespace fth {
namespace dev {

// M (FP32, [P][P] row-major) -> bf16 hi/lo parts in the GEMM's tiled
// layout; one 16-byte output unit (8 consecutive k of one row, one part)
// per iteration.
__global__ void split_bf16_tiled_kernel(const float* __restrict__ m, u32x4* __restrict__ mt, int64_t P) {
    const int64_t total = P * P / 4;  // P^2 elements x 2 parts x 2 bytes / 16 bytes
    const int64_t KB = P / 64;
    for (int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
        const int l = int(o & 63), u = int((o >> 6) & 7), w = int((o >> 9) & 3);
        const int64_t tile = o >> 11;
        const int64_t row = (tile / KB) * 128 + 32 * w + 16 * (u >> 2) + (l & 15);
        const int64_t k = (tile % KB) * 64 + 16 * (l >> 4) + 8 * (u & 1);
        const bool lo = ((u >> 1) & 1) != 0;
        const float* src = m + row * P + k;
        uint32_t word[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t two = 0;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const float x = src[2 * t + e];
                const uint16_t h = bf16_bits(x);
                const uint16_t part = lo ? bf16_bits(x - bf16_value(h)) : h;
                two |= uint32_t(part) << (16 * e);
            }
            word[t] = two;
        }
        mt[o] = u32x4{word[0], word[1], word[2], word[3]};
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

int launch_split_bf16_tiled(const float* m, void* mt, int64_t P, void* stream) {
    if (P % 128 != 0) return -3;
    hipLaunchKernelGGL(dev::split_bf16_tiled_kernel, dim3(4096), dim3(256), 0, static_cast<hipStream_t>(stream), m,
                       static_cast<dev::u32x4*>(mt), P);
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
