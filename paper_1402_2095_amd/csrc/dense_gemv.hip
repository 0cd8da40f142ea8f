// Dense force for few replicas (R in {1, 2, 4, 8}): F = M q_n as R matrix-vector
// products, streamed row by row.  With so few right-hand sides the work is one
// pass over M per step, bound by HBM; the matrix cores' 16-column tiles would
// compute mostly zero columns, so the products use plain FMAs in the state
// precision.
//
// Layouts: M row-major Real [N][ld], ld = N rounded up to 4 with zero columns;
// q_n [ld][R] (the context's q buffers, zero rows past N).  Wave w of workgroup
// b owns rows ROWS (4 b + w) + (0 .. ROWS-1).  The four waves walk the columns
// together, 256 per pass: from 4 replicas on, the pass's 256 rows of q_n are
// staged once in LDS for all four (read from L2 by every wave, they cost more
// than M itself at R = 8); lane l takes columns 4 l .. 4 l + 3 of the pass, loads 4 entries of each of its
// rows, and keeps one partial sum per (row, replica); the wave then adds the 64
// lanes' partials in a fixed butterfly, so the result does not depend on
// scheduling.  The sums are written as the single K slice the dense epilogue
// reads (part [1][ld][R]).
#include "dense.hpp"

namespace fth {
namespace dev {

template <typename Real, int R>
__global__ __launch_bounds__(256) void dense_gemv_kernel(const DenseGemmArgs g, const Real* __restrict__ M, int64_t N,
                                                         int64_t ld) {
    constexpr int ROWS = 8;
    constexpr int VW = 4;
    constexpr int CH = 64 * VW;          // columns per pass
    constexpr int QV = CH / 4 * R;       // 4-value vectors of q_n per pass
    // From 4 replicas on, q_n read from L2 by every wave costs as much as M itself, so the
    // pass's rows are staged once in LDS for the four waves; with 1 or 2 replicas each lane
    // reads its own (fewer bytes than the barrier per pass costs).
    constexpr bool STAGE = R >= 4;
    __shared__ Vec<Real, 4> qs[STAGE ? 2 : 1][STAGE ? QV : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t row0 = (int64_t(blockIdx.x) * 4 + (tid >> 6)) * ROWS;
    const bool live = row0 < N;  // a wave past the last row still stages q_n and meets the barriers
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
    // ROWS rows' partial sums from columns j .. j+3, with the lane's 4 R values of q_n at qv
    auto accumulate = [&](int64_t j, const Vec<Real, 4>* qv) {
        Vec<Real, 4> mv[ROWS];
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) mv[rr] = load_vec<Real, 4>(mrow[rr] + j);
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr)
#pragma unroll
            for (int c = 0; c < VW; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = c * R + r;  // element (j + c, r) of the lane's 4 R values
                    acc[rr][r] = fmaR(mv[rr].v[c], qv[e >> 2].v[e & 3], acc[rr][r]);
                }
    };
    if constexpr (STAGE) {
        // vector x of a pass starting at column j0 holds q_n elements [4x, 4x + 4) of rows
        // j0 .. j0 + CH - 1, i.e. from row j0 + 4x / R on (ld is a multiple of 4)
        auto stage = [&](int buf, int64_t j0) {
            for (int x = tid; x < QV; x += 256)
                if (j0 + 4 * x / R < ld) qs[buf][x] = load_vec<Real, 4>(q + j0 * R + 4 * x);
        };
        const int64_t npass = (ld + CH - 1) / CH;
        stage(0, 0);
        __syncthreads();
        for (int64_t p = 0; p < npass; ++p) {
            const int64_t j0 = p * CH, j = j0 + int64_t(lane) * VW;
            if (p + 1 < npass) stage(int((p + 1) & 1), j0 + CH);  // last read before the previous barrier
            if (live && j < ld) accumulate(j, &qs[p & 1][lane * R]);
            __syncthreads();
        }
    } else {
        if (!live) return;
        for (int64_t j = int64_t(lane) * VW; j < ld; j += CH) {
            Vec<Real, 4> qv[R];  // q_n rows j .. j+3: 4 R consecutive values
#pragma unroll
            for (int u = 0; u < R; ++u) qv[u] = load_vec<Real, 4>(q + j * R + 4 * u);
            accumulate(j, qv);
        }
    }
    if (!live) return;
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
    constexpr int ROWS = 8;
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
