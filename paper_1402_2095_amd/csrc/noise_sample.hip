// Device evaluation of the thermostat's noise stream at arbitrary
// (dof, replica, step, component) points, for validation of the generator.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/fth.h"
#include "noise.hpp"

namespace fth {
namespace dev {

template <typename Real>
__global__ void noise_sample_kernel(uint32_t k0, uint32_t k1, uint32_t stream, int64_t count,
                                    const uint32_t* __restrict__ i, const uint32_t* __restrict__ r,
                                    const uint32_t* __restrict__ n, const uint32_t* __restrict__ j,
                                    double* __restrict__ out, uint32_t* __restrict__ raw) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= count) return;
    Real z[1];
    normals<Real, 1>(k0, k1, stream, i[k], n[k], j[k], r[k], z);
    out[k] = double(z[0]);
    if (raw != nullptr) {
        const Block4 b = philox4x32_10(i[k], n[k], (j[k] << 16) | (r[k] >> 2), stream, k0, k1);
        for (int w = 0; w < 4; ++w) raw[4 * k + w] = b.w[w];
    }
}

}  // namespace dev
}  // namespace fth

extern "C" fth_status fth_noise_sample(uint64_t seed, uint32_t stream, int64_t count, const uint32_t* i,
                                       const uint32_t* r, const uint32_t* n, const uint32_t* j, int32_t precision,
                                       double* out, uint32_t* raw) {
    if (count < 0 || (count > 0 && (!i || !r || !n || !j || !out))) return FTH_EINVAL;
    if (precision != FTH_FP64 && precision != FTH_FP32) return FTH_EINVAL;
    if (count == 0) return FTH_OK;
    for (int64_t k = 0; k < count; ++k)
        if (j[k] >= 65536u || r[k] >= (1u << 18)) return FTH_EINVAL;
    const size_t c = size_t(count);
    uint32_t* d_in = nullptr;
    double* d_out = nullptr;
    uint32_t* d_raw = nullptr;
    fth_status st = FTH_OK;
    if (hipMalloc(&d_in, 4 * c * sizeof(uint32_t)) != hipSuccess || hipMalloc(&d_out, c * sizeof(double)) != hipSuccess ||
        (raw && hipMalloc(&d_raw, 4 * c * sizeof(uint32_t)) != hipSuccess)) {
        st = FTH_ENOMEM;
    } else {
        const uint32_t* src[4] = {i, r, n, j};
        for (int a = 0; a < 4 && st == FTH_OK; ++a)
            if (hipMemcpy(d_in + a * c, src[a], c * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) st = FTH_EDEVICE;
        if (st == FTH_OK) {
            const unsigned grid = unsigned((count + 255) / 256);
            if (precision == FTH_FP64)
                hipLaunchKernelGGL(fth::dev::noise_sample_kernel<double>, dim3(grid), dim3(256), 0, nullptr,
                                   uint32_t(seed), uint32_t(seed >> 32), stream, count, d_in, d_in + c, d_in + 2 * c,
                                   d_in + 3 * c, d_out, d_raw);
            else
                hipLaunchKernelGGL(fth::dev::noise_sample_kernel<float>, dim3(grid), dim3(256), 0, nullptr,
                                   uint32_t(seed), uint32_t(seed >> 32), stream, count, d_in, d_in + c, d_in + 2 * c,
                                   d_in + 3 * c, d_out, d_raw);
            if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) st = FTH_EDEVICE;
        }
        if (st == FTH_OK && hipMemcpy(out, d_out, c * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) st = FTH_EDEVICE;
        if (st == FTH_OK && raw && hipMemcpy(raw, d_raw, 4 * c * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
            st = FTH_EDEVICE;
    }
    if (d_in) (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    if (d_raw) (void)hipFree(d_raw);
    return st;
}
