// Dense force F = -M q_n as a GEMM on the matrix cores, and the epilogue
// that applies the GLE step to its result.
//
// Split form (FTH_FP32_BF16X3): M (FP32) is split once into bf16 hi/lo
// parts with M = M_hi + M_lo + O(2^-17 |M|); q_n is split likewise each step
// by the previous epilogue.  The force uses three bf16 products with FP32
// accumulation on v_mfma_f32_16x16x32_bf16:
//     M q ~ M_hi q_hi + M_hi q_lo + M_lo q_hi     (the M_lo q_lo term, ~2^-16
//                                                  relative, is dropped)
// FP64 form (FTH_FP64): v_mfma_f64_16x16x4_f64 on M and q_n directly.
//
// Work split: the output rows are cut into row blocks and the K dimension
// into ksplit slices (a power of two <= 8); workgroup b takes K slice
// b mod ksplit and row block b / ksplit.  The hardware deals workgroups
// round-robin over the 8 XCDs, so the workgroups of K slice s run on the
// XCDs x with x mod ksplit = s, and the q_n slice they stream stays in
// those XCDs' L2.  Each workgroup writes FP32
// (FP64) partial sums part[ks][row][col]; the epilogue adds the ksplit
// partials in slice order, so the result does not depend on scheduling.
//
// Operand layouts (one wave, verified on gfx950):
//   16x16x32 bf16: lane l holds A[l%16][8(l/16)+t], B[8(l/16)+t][l%16],
//                  and D[4(l/16)+e][l%16], t < 8, e < 4.
//   16x16x4  f64 : lane l holds A[l%16][l/16], B[l/16][l%16],
//                  and D[4e+l/16][l%16], e < 4.
// In the split form M_hi and M_lo are kept together in a tiled layout,
// written once by the split kernel, in which every load of a wave is 1 KB
// of contiguous memory: for row block rb (128 rows) and k-step kb (64 k)
// one 32 KB tile holds, per wave w and load slot u < 8, the 64 lanes'
// 16-byte A fragments side by side,
//     mt[((rb * rows_pad / 64 + kb) * 4 + w) * 8 + u][lane],
// slot u carrying part (u >> 1) & 1 (0: hi, 1: lo) of row
// 128 rb + 32 w + 16 (u >> 2) + lane % 16 at k = 64 kb + 16 (lane / 16) +
// 8 (u & 1) + (0..7).  The k-steps of one K slice are consecutive tiles,
// so a workgroup streams one contiguous run of memory.  (Row-major, each
// load instruction touched 16 rows 32 KB apart and M streamed at about
// half the rate.)  In the FP64 form M is row-major, so an A fragment is
// 4 contiguous doubles of one row.  The bf16 B fragment needs 8 consecutive k of one column, so q_n is
// kept as qt[k/8][col][hi|lo][k%8] (written by the epilogue): a k-step of
// 64 is one contiguous 256*R-byte chunk, staged through LDS and shared by
// the four waves.  The f64 B fragment is one element, so q_n [k][col] is
// staged as is; within a k-step of 16, lane group g handles k = 4g + t at
// substep t, which makes each lane's A data 4 contiguous doubles.
#pragma once

#include <hip/hip_runtime.h>

#include "csr_step.hpp"

namespace fth {
namespace dev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// qt[k/8][r][0][k%8] = hi(q[k][r]), qt[k/8][r][1][k%8] = lo(q[k][r]) for k < N.
__device__ __forceinline__ void put_qt(uint16_t* qt, int64_t k, int64_t r, int32_t R, float x) {
    const uint16_t h = bf16_bits(x);
    uint16_t* base = qt + ((k >> 3) * R + r) * 16 + (k & 7);
    base[0] = h;
    base[8] = bf16_bits(x - bf16_value(h));
}


// Copy of one staged chunk: thread t moves elements t, t + 256, ... (< COUNT).
// Written as compile-time recursion so the register arrays are never indexed
// at run time (which would put them in scratch memory).
template <typename T, int COUNT, int PER, int U = 0>
__device__ __forceinline__ void gather_chunk(T (&dst)[PER], const T* __restrict__ src) {
    if constexpr (U < PER) {
        const int idx = int(threadIdx.x) + 256 * U;
        if (COUNT % 256 == 0 || idx < COUNT) dst[U] = src[idx];
        gather_chunk<T, COUNT, PER, U + 1>(dst, src);
    }
}
template <typename T, int COUNT, int PER, int U = 0>
__device__ __forceinline__ void scatter_chunk(T* __restrict__ dst, const T (&src)[PER]) {
    if constexpr (U < PER) {
        const int idx = int(threadIdx.x) + 256 * U;
        if (COUNT % 256 == 0 || idx < COUNT) dst[idx] = src[U];
        scatter_chunk<T, COUNT, PER, U + 1>(dst, src);
    }
}

// ------------------------------------------------------ split-BF16x3 GEMM
// A k-step covers 64 consecutive k: one 32 KB tile of M (hi and lo parts)
// and one 32 KB chunk of q_n, both fetched one k-step ahead.  M is read once
// per step, so its loads are non-temporal (they do not evict q_n from L2).  Inside a
// k-step the k order is permuted (a sum may be taken in any order): lane
// group g owns k = 16 g + 8 t + (0..7) in substep t = 0, 1, so its B
// fragment is q-chunk block 2 g + t.
template <int RT>
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_kernel(const DenseGemmArgs g) {
    constexpr int R = 16 * RT;
    constexpr int BM = 128;  // rows per workgroup: 4 waves x 32
    constexpr int KS = 64;   // k per step
    constexpr int CHUNK = (KS / 8) * R * 2;  // 16-byte units per staged k-step: [8][R][hi|lo]
    __shared__ u32x4 qs[2][CHUNK];

    const int ks = blockIdx.x % g.ksplit;
    const int64_t rb = blockIdx.x / g.ksplit;
    const int64_t m0 = rb * BM;
    const int64_t kbeg = int64_t(ks) * g.kslice;
    const int nsteps = int(g.kslice / KS);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const int64_t P = g.rows_pad;
    const u32x4* qsrc = reinterpret_cast<const u32x4*>(g.qt);
    constexpr int TILE = 4 * 8 * 64;  // 16-byte units per (row block, k-step) tile
    // this wave's slots of the first tile of the K slice (rows m0 + 32 w + lr and + 16)
    const u32x4* mt = static_cast<const u32x4*>(g.m_hi) + (rb * (P / KS) + kbeg / KS) * TILE + w * (8 * 64) + l;

    f32x4 acc[2][RT];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    constexpr int PER_THREAD = (CHUNK + 255) / 256;
    u32x4 rq[PER_THREAD];
    u32x4 ra[8];  // [row 0/1][hi/lo][substep 0/1]
#define FTH_BF16_FETCH(J)                                                          \
    {                                                                              \
        const int64_t kf = kbeg + int64_t(J) * KS;                                 \
        gather_chunk<u32x4, CHUNK, PER_THREAD>(rq, qsrc + (kf / 8) * R * 2);       \
        const u32x4* src = mt + int64_t(J) * TILE;                                 \
        _Pragma("unroll") for (int u = 0; u < 8; ++u) ra[u] = __builtin_nontemporal_load(src + u * 64); \
    }
    FTH_BF16_FETCH(0)
    for (int j = 0; j < nsteps; ++j) {
        u32x4* buf = qs[j & 1];
        // staged planar, [hi|lo][k/8][R], so the B reads below are 16 contiguous
        // bytes per lane (no bank conflicts)
#pragma unroll
        for (int u = 0; u < PER_THREAD; ++u) {
            const int idx = int(threadIdx.x) + 256 * u;
            if (CHUNK % 256 == 0 || idx < CHUNK) buf[(idx & 1) * (CHUNK / 2) + (idx >> 1)] = rq[u];
        }
        bf16x8 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = __builtin_bit_cast(bf16x8, ra[u]);
        if (j + 1 < nsteps) FTH_BF16_FETCH(j + 1)
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int c = 0; c < RT; ++c) {
                const u32x4* bsrc = buf + (2 * lg + t) * R + 16 * c + lr;
                const bf16x8 bhi = __builtin_bit_cast(bf16x8, bsrc[0]);
                const bf16x8 blo = __builtin_bit_cast(bf16x8, bsrc[CHUNK / 2]);
                // row tile 0: a[0 + t] (hi), a[2 + t] (lo); row tile 1: a[4 + t], a[6 + t]
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0 + t], bhi, acc[0][c], 0, 0, 0);
                acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[4 + t], bhi, acc[1][c], 0, 0, 0);
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0 + t], blo, acc[0][c], 0, 0, 0);
                acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[4 + t], blo, acc[1][c], 0, 0, 0);
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2 + t], bhi, acc[0][c], 0, 0, 0);
                acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[6 + t], bhi, acc[1][c], 0, 0, 0);
            }
    }
#undef FTH_BF16_FETCH
    float* part = static_cast<float*>(g.part) + int64_t(ks) * P * R;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < RT; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                part[(m0 + 32 * w + 16 * t + 4 * lg + e) * R + 16 * c + lr] = acc[t][c][e];
}

// ----------------------------------------------------------------- FP64 GEMM
template <int RT>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(const DenseGemmArgs g) {
    constexpr int R = 16 * RT;
    constexpr int BM = 64;  // rows per workgroup: 4 waves x 16
    constexpr int KS = 16;  // k per step (4 substeps of 4)
    constexpr int CHUNK = KS * R;  // doubles per staged k-step
    __shared__ double qs[2][CHUNK];

    const int ks = blockIdx.x % g.ksplit;
    const int64_t rb = blockIdx.x / g.ksplit;
    const int64_t m0 = rb * BM;
    const int64_t kbeg = int64_t(ks) * g.kslice;
    const int nsteps = int(g.kslice / KS);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const int64_t P = g.rows_pad;
    const int64_t n = g.step_base[0] + g.k;
    const double* q = static_cast<const double*>((n & 1) ? g.q1 : g.q0);
    const double* arow = static_cast<const double*>(g.m_hi) + (m0 + 16 * w + lr) * P + 4 * lg;

    f64x4 acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};

    constexpr int PER_THREAD = (CHUNK / 2 + 255) / 256;  // f64x2 per thread
    f64x2 rq[PER_THREAD];
    f64x2 ra0, ra1;
#define FTH_F64_FETCH(J)                                                           \
    {                                                                              \
        const int64_t kf = kbeg + int64_t(J) * KS;                                 \
        gather_chunk<f64x2, CHUNK / 2, PER_THREAD>(                             \
            rq, reinterpret_cast<const f64x2*>(q + kf * R));                     \
        ra0 = *reinterpret_cast<const f64x2*>(arow + kf);                        \
        ra1 = *reinterpret_cast<const f64x2*>(arow + kf + 2);                    \
    }
    FTH_F64_FETCH(0)
    for (int j = 0; j < nsteps; ++j) {
        f64x2* buf = reinterpret_cast<f64x2*>(qs[j & 1]);
        scatter_chunk<f64x2, CHUNK / 2, PER_THREAD>(buf, rq);
        const double a0 = ra0[0], a1 = ra0[1], a2 = ra1[0], a3 = ra1[1];
        if (j + 1 < nsteps) FTH_F64_FETCH(j + 1)
        __syncthreads();
        const double* bq = qs[j & 1];
#pragma unroll
        for (int c = 0; c < RT; ++c) {
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bq[(4 * lg + 0) * R + 16 * c + lr], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bq[(4 * lg + 1) * R + 16 * c + lr], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, bq[(4 * lg + 2) * R + 16 * c + lr], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, bq[(4 * lg + 3) * R + 16 * c + lr], acc[c], 0, 0, 0);
        }
    }
#undef FTH_F64_FETCH
    double* part = static_cast<double*>(g.part) + int64_t(ks) * P * R;
#pragma unroll
    for (int c = 0; c < RT; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) part[(m0 + 16 * w + 4 * e + lg) * R + 16 * c + lr] = acc[c][e];
}

// ------------------------------------------------------------- epilogue
// One row of the dense epilogue: sum the split-K partials in slice order,
// then the shared row update (and, in the split form, the bf16 split of q).
template <typename Real, int NS, int RPT, bool NT>
__device__ __forceinline__ void dense_row(const StepArgs<Real>& a, const StepInfo& si, int64_t i, const Real* qr,
                                          Real* qw, double* trow) {
    using V = Vec<Real, RPT>;
    const int64_t R = a.R;
    Real xi[NS + 1][RPT];
    const bool early = noise_first();
    if (early) row_noise<Real, NS, RPT>(a, si, i, xi);
    const RowState<Real, NS, RPT> st = load_row<Real, NS, RPT, NT>(a, si, qr, i);
    constexpr int KMAX = 8;
    V pv[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        if (s < a.ksplit) pv[s] = load_state<Real, RPT, true>(a.part + (int64_t(s) * a.rows_pad + i) * R + si.r0);
    if (!early) row_noise<Real, NS, RPT>(a, si, i, xi);
    Real acc[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) acc[m] = Real(0);
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        if (s < a.ksplit) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) acc[m] = acc[m] + pv[s].v[m];
        }
    const V qn = finish_row<Real, NS, RPT, NT>(a, si, i, st, acc, xi, qw, trow);
    if constexpr (sizeof(Real) == 4) {
        if (a.qt != nullptr) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) put_qt(a.qt, i, si.r0 + m, a.R, qn.v[m]);
        }
    }
}

template <typename Real, int NS, int RPT, bool NT, bool TR>
__global__ __launch_bounds__(256) void dense_epilogue_kernel(const StepArgs<Real> a, const int k) {
    const StepInfo si = step_info<Real, RPT>(a, k);
    const Real* __restrict__ qr = (si.n & 1) ? a.q1 : a.q0;
    Real* __restrict__ qw = (si.n & 1) ? a.q0 : a.q1;
    const int per_block = blockDim.x >> a.lg_tpr;
    const int64_t b = blockIdx.x;
    if (b >= a.row_tiles_padded) {
        const int64_t pk = (b - a.row_tiles_padded) * per_block + si.slot;
        if (pk < a.npairs) pair_update<Real, RPT>(a, si, qr, pk);
        return;
    }
    const int64_t per = a.row_tiles_padded >> 3;
    const int64_t t = (b & 7) * per + (b >> 3);
    if (t >= a.row_tiles) return;  // whole workgroup
    const int64_t i = t * per_block + si.slot;
    extern __shared__ double trl[];  // [rows of the tile][3], only with trace partials
    double* trow = TR ? trl + si.slot * 3 : nullptr;
    if (i < a.N) dense_row<Real, NS, RPT, NT>(a, si, i, qr, qw, trow);
    if constexpr (TR) {
        __syncthreads();
        wave0_sum_rows(trl, min(int64_t(per_block), a.N - t * per_block), a.tpart + (int64_t(k) * a.tpart_w + t) * 3);
    }
}

template <bool TR>
struct DenseEpilogueKernels {
    template <typename Real, int NS, int RPT, bool NT>
    struct K {
        static const void* fn() {
            return reinterpret_cast<const void*>(&dense_epilogue_kernel<Real, NS, RPT, NT, TR>);
        }
    };
};

}  // namespace dev

template <typename Real>
int launch_dense_epilogue_impl(const StepArgs<Real>& a, const StepLaunch& L, int k, void* stream) {
    const void* fn = a.tpart != nullptr ? dev::pick_kernel<dev::DenseEpilogueKernels<true>::template K, Real>(L)
                                        : dev::pick_kernel<dev::DenseEpilogueKernels<false>::template K, Real>(L);
    return dev::launch_step_kernel<Real>(fn, a, L, k, stream);
}

}  // namespace fth
