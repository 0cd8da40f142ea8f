// Trace estimators (sum_i <q_i^2>, <q^T M q>, sum_i <p_i^2>): every step
// kernel leaves one partial per row tile and step; once per chunk these are
// summed per step in a fixed order and folded into the trace accumulators in
// step order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "row_update.hpp"

namespace fth {
namespace dev {

// One workgroup per step k: sum the W tile partials, clear them.
__global__ __launch_bounds__(256) void trace_reduce_kernel(double* __restrict__ tpart, double* __restrict__ tsum,
                                                           int W) {
    __shared__ double red[16 * 3];
    const int64_t k = blockIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = int(threadIdx.x); t < W; t += int(blockDim.x)) {
        double* p = tpart + (k * W + t) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] += p[c];
            p[c] = 0.0;
        }
    }
    workgroup_sum3(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) tsum[k * 3 + c] = v[c];
}

// Block averaging of the per-step trace values, in step order.
__global__ void trace_fold_kernel(const double* __restrict__ tsum, int K, int ntr, double* blk, double* s1,
                                  double* s2, const int64_t* step_base, int64_t shift, int64_t burn_in,
                                  int64_t block_len) {
    if (threadIdx.x != 0) return;
    const int64_t n0 = step_base[0] + shift;
    for (int k = 0; k < K; ++k) {
        const int64_t n = n0 + k;
        if (n < burn_in) continue;
        const bool close = ((n - burn_in + 1) % block_len) == 0;
        for (int c = 0; c < ntr; ++c) acc_update(blk, s1, s2, c, tsum[k * 3 + c], close);
    }
}

}  // namespace dev

int launch_trace_fold(double* tpart, double* tsum, int K, int W, int ntr, double* blk, double* s1, double* s2,
                      const int64_t* step_base, int64_t shift, int64_t burn_in, int64_t block_len, void* stream) {
    if (K <= 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(dev::trace_reduce_kernel, dim3(unsigned(K)), dim3(256), 0, st, tpart, tsum, W);
    hipLaunchKernelGGL(dev::trace_fold_kernel, dim3(1), dim3(64), 0, st, tsum, K, ntr, blk, s1, s2, step_base, shift,
                       burn_in, block_len);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fth
