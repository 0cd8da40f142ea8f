// Dense force for few replicas (R in {1, 2, 4, 8}): F = M q_n as R matrix-vector
// products, streamed row by row.  With so few right-hand sides the work is one
// pass over M per step, bound by HBM; the matrix cores' 16-column tiles would
// compute mostly zero columns, so the products use plain FMAs in the state
// precision.
//
// Layouts: M row-major Real [N][ld], ld = N rounded up to 4 with zero columns;
// q_n [ld][R] (the context's q buffers, zero rows past N).  Wave w of workgroup
// b owns rows ROWS (4 b + w) + (0 .. ROWS-1).  Lane l walks the columns
// 4 l + 256 m, loading 4 entries of each of its rows and the 4 matching rows of
// q_n per pass, and keeps one partial sum per (row, replica); the wave then adds
// the 64 lanes' partials in a fixed butterfly, so the result does not depend on
// scheduling.  The sums are written as the single K slice the dense epilogue
// reads (part [1][ld][R]).
#include "dense.hpp"

namespace fth {
namespace dev {

template <typename Real, int R>
__global__ __launch_bounds__(256) void dense_gemv_kernel(const DenseGemmArgs g, const Real* __restrict__ M, int64_t N,
                                                         int64_t ld) {
    constexpr int ROWS = (sizeof(Real) == 8 && R == 8) ? 4 : 8;
    constexpr int VW = 4;
    const int lane = threadIdx.x & 63;
    const int64_t row0 = (int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6)) * ROWS;
    if (row0 >= N) return;  // the whole wave; no barrier follows
    const int64_t n = g.step_base[0] + g.k;
    const Real* __restrict__ q = static_cast<const Real*>((n & 1) ? g.q1 : g.q0);
    Real* part = static_cast<Real*>(g.part);
    // rows past N (in the last wave) repeat row N - 1 and are not stored
    const Real* mrow[ROWS];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) mrow[rr] = M + min(row0 + rr, N - 1) * ld;
    Real acc[ROWS][R];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[rr][r] = Real(0);
    for (int64_t j = int64_t(lane) * VW; j < ld; j += 64 * VW) {
        // q_n rows j .. j+3: 4 R consecutive values
        Vec<Real, 4> qv[R];
#pragma unroll
        for (int u = 0; u < R; ++u) qv[u] = load_vec<Real, 4>(q + j * R + 4 * u);
        Vec<Real, 4> mv[ROWS];
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) mv[rr] = load_vec<Real, 4>(mrow[rr] + j);
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr)
#pragma unroll
            for (int c = 0; c < VW; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = c * R + r;  // element (j + c, r) of the 4 R loaded
                    acc[rr][r] = fmaR(mv[rr].v[c], qv[e >> 2].v[e & 3], acc[rr][r]);
                }
    }
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            Real v = acc[rr][r];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
            if (lane == 0 && row0 + rr < N) part[(row0 + rr) * R + r] = v;
        }
}

template <typename Real, int R>
int launch_gemv_r(const DenseGemmArgs& g, const Real* M, int64_t N, int64_t ld, void* stream) {
    constexpr int ROWS = (sizeof(Real) == 8 && R == 8) ? 4 : 8;
    const int64_t waves = (N + ROWS - 1) / ROWS;
    const int64_t grid = (waves + 3) / 4;
    if (grid > 0x7FFFFFFF) return -3;
    hipLaunchKernelGGL((dense_gemv_kernel<Real, R>), dim3(unsigned(grid)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), g, M, N, ld);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dev

template <typename Real>
int launch_dense_gemv(const DenseGemmArgs& g, const Real* M, int64_t N, int64_t ld, void* stream) {
    if (ld % 4 != 0 || ld < N || g.rows_pad < ld) return -4;
    switch (g.R) {
        case 1: return dev::launch_gemv_r<Real, 1>(g, M, N, ld, stream);
        case 2: return dev::launch_gemv_r<Real, 2>(g, M, N, ld, stream);
        case 4: return dev::launch_gemv_r<Real, 4>(g, M, N, ld, stream);
        case 8: return dev::launch_gemv_r<Real, 8>(g, M, N, ld, stream);
        default: return -2;
    }
}

template int launch_dense_gemv<float>(const DenseGemmArgs&, const float*, int64_t, int64_t, void*);
template int launch_dense_gemv<double>(const DenseGemmArgs&, const double*, int64_t, int64_t, void*);

}  // namespace fth
