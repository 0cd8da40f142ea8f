// Persistent single-workgroup step loop for small dense systems (N * R up
// to a few thousand), where one launch per step would be launch-bound.
//
// One workgroup of N * TPR threads (TPR = R / RPT) runs K steps per launch:
//   - M (if it fits) and both q buffers live in LDS; each thread keeps its
//     row slice of p and s in registers for the whole launch;
//   - the block sums of the accumulators live in LDS; s1 / s2 in global
//     memory are touched only when a block closes;
//   - with p-p pair accumulators, p_n is mirrored to two more LDS buffers so
//     the pairs can read it while rows write p_{n+1};
//   - one workgroup barrier per step separates reading q_n from writing
//     q_{n+1}, which go to alternating LDS buffers.
// The arithmetic of a step is the same as in the sparse and dense kernels
// (row_update.hpp), so the trajectory matches them up to the order of the
// force sum.
#pragma once

#include <hip/hip_runtime.h>

#include "csr_step.hpp"

namespace fth {
namespace dev {

// sum_j M_ij q_j over the row, in column order, for the thread's replicas, with M
// column-major (mrow[j * N] = M_ij: consecutive rows read consecutive words, which
// keeps LDS reads free of bank conflicts and global reads coalesced); the operands
// of 8 columns are loaded before their FMAs so that the loads overlap
template <typename Real, int RPT>
__device__ __forceinline__ void row_force(const Real* mrow, const Real* q, int64_t N, int64_t R, Real* acc) {
    constexpr int B = 8;
#pragma unroll
    for (int m = 0; m < RPT; ++m) acc[m] = Real(0);
    int64_t j = 0;
    for (; j + B <= N; j += B) {
        Real mb[B];
        Vec<Real, RPT> qb[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            mb[u] = mrow[(j + u) * N];
            qb[u] = load_vec<Real, RPT>(q + (j + u) * R);
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
#pragma unroll
            for (int m = 0; m < RPT; ++m) acc[m] = fmaR(mb[u], qb[u].v[m], acc[m]);
    }
    for (; j < N; ++j) {
        const Real mij = mrow[j * N];
        const Vec<Real, RPT> qj = load_vec<Real, RPT>(q + j * R);
#pragma unroll
        for (int m = 0; m < RPT; ++m) acc[m] = fmaR(mij, qj.v[m], acc[m]);
    }
}

// sum_r x_r y_r in FP64 over the replicas, in replica order; with R a multiple of 4
// (always, from 4 replicas on) the rows are read 4 replicas per load
template <typename Real>
__device__ __forceinline__ double pair_dot(const Real* x, const Real* y, int64_t R) {
    double acc = 0.0;
    int64_t r = 0;
    if ((R & 3) == 0) {
        for (; r < R; r += 4) {
            const Vec<Real, 4> u = load_vec<Real, 4>(x + r), v = load_vec<Real, 4>(y + r);
#pragma unroll
            for (int m = 0; m < 4; ++m) acc += double(u.v[m]) * double(v.v[m]);
        }
    }
    for (; r < R; ++r) acc += double(x[r]) * double(y[r]);
    return acc;
}

// MAXT is the largest workgroup the instantiation accepts: at 256 or 512 threads a
// thread may hold 512 or 256 registers, so the state of wide thermostats (and the
// FP64 form) stays in registers instead of spilling to scratch memory.
template <typename Real, int NS, int RPT, int MAXT>
__global__ __launch_bounds__(MAXT) void small_dense_kernel(const StepArgs<Real> a, const int K) {
    extern __shared__ double smem_d[];
    constexpr int D = NS + 1;
    const int64_t N = a.N, R = a.R;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int tpr = 1 << a.lg_tpr;
    const int rq = tid & (tpr - 1), r0 = rq * RPT;
    const int64_t i = tid >> a.lg_tpr;
    const bool active = i < N;
    const int64_t nd = a.dblk != nullptr ? N : 0;
    const bool kp = a.pp_blk != nullptr;          // p-p accumulators kept
    const int64_t np = a.npairs, nacc = np + nd;  // per kind (q, then p)
    const bool pp_pairs = kp && np > 0;
    // LDS layout: block sums (FP64) [q pairs | q diag | p pairs | p diag] | q[2][N][R]
    //             | p[2][N][R] (p-p pairs only) | T, S [2][D][D] | M column-major (if in LDS)
    double* bl = smem_d;
    // (state buffers start on a 32-byte boundary, the alignment of a 4-replica FP64 vector)
    Real* qb = reinterpret_cast<Real*>(bl + (((kp ? 2 : 1) * nacc + 3) & ~int64_t(3)));
    Real* pb = qb + 2 * N * R;
    Real* tsl = pb + (pp_pairs ? 2 * N * R : 0);  // T and S, read in every step
    for (int x = tid; x < 2 * D * D; x += nthr) tsl[x] = a.TS[x];
    // M in LDS when it fits; the force loop is written once per address space (a pointer that
    // may be either would compile to flat loads, which wait on both the LDS and vector counters)
    Real* Ml = tsl + 2 * D * D;
    if (a.m_in_lds)
        for (int64_t x = tid; x < N * N; x += nthr) Ml[x] = a.mdense[x];
    const int64_t n0 = a.step_base[0];
    const Real* qg = (n0 & 1) ? a.q1 : a.q0;
    for (int64_t x = tid; x < N * R; x += nthr) qb[(n0 & 1) * N * R + x] = qg[x];
    for (int64_t x = tid; x < np; x += nthr) bl[x] = a.pblk[x];
    for (int64_t x = tid; x < nd; x += nthr) bl[np + x] = a.dblk[x];
    if (kp) {
        for (int64_t x = tid; x < np; x += nthr) bl[nacc + x] = a.pp_blk[x];
        for (int64_t x = tid; x < nd; x += nthr) bl[nacc + np + x] = a.dp_blk[x];
    }

    RowState<Real, NS, RPT> st;
    if (active) {
        st.q = load_vec<Real, RPT>(qg + i * R + r0);
        const Real* psrow = ps_row(ps_at_step(a, n0), i, D, R, a.ps_lg) + r0;
        const int64_t cs = ps_stride(R, a.ps_lg);
        st.p = load_vec<Real, RPT>(psrow);
#pragma unroll
        for (int c = 0; c < NS; ++c) st.s[c] = load_vec<Real, RPT>(psrow + (c + 1) * cs);
        if (pp_pairs) store_vec<Real, RPT>(pb + (n0 & 1) * N * R + i * R + r0, st.p);
    }
    const Real* T = tsl;
    const Real* S = tsl + D * D;
    // a thread's first pair stays in registers (all of its pairs when there are no more
    // pairs than threads)
    int64_t ia0 = 0, ib0 = 0;
    if (tid < np) {
        ia0 = a.pairs[2 * tid];
        ib0 = a.pairs[2 * tid + 1];
    }
    bool ok = true;
    __syncthreads();

    __shared__ double red[16 * 3];
    for (int k = 0; k < K; ++k) {
        const int64_t n = n0 + k;
        double tr[3] = {0.0, 0.0, 0.0};
        const bool acc_on = n >= a.burn_in;
        const bool close = acc_on && ((n - a.burn_in + 1) % a.block_len) == 0;
        const Real* qr = qb + (n & 1) * N * R;
        Real* qw = qb + ((n + 1) & 1) * N * R;
        // one block-sum update of accumulator slot x in LDS
        auto fold = [&](double* blk, double* s1, double* s2, int64_t idx, int64_t slot, double v) {
            const double b = blk[slot] + v;
            if (close) {
                s1[idx] = s1[idx] + b;
                s2[idx] = s2[idx] + b * b;
                blk[slot] = 0.0;
            } else {
                blk[slot] = b;
            }
        };
        if (acc_on) {
            for (int64_t pk = tid; pk < np; pk += nthr) {
                int64_t ia = ia0, ib = ib0;
                if (pk != tid) {
                    ia = a.pairs[2 * pk];
                    ib = a.pairs[2 * pk + 1];
                }
                const double x = pair_dot(qr + ia * R, qr + ib * R, R);
                fold(bl, a.ps1, a.ps2, pk, pk, x);
                if (pp_pairs) {
                    const Real* pr = pb + (n & 1) * N * R;
                    const double y = pair_dot(pr + ia * R, pr + ib * R, R);
                    fold(bl, a.pp_s1, a.pp_s2, pk, nacc + pk, y);
                }
            }
        }
        if (active) {
            Real acc[RPT];
            if (a.m_in_lds)
                row_force<Real, RPT>(Ml + i, qr + r0, N, R, acc);
            else
                row_force<Real, RPT>(a.mdense + i, qr + r0, N, R, acc);
            if (nd) {
                const double x = dot_row<Real, RPT>(st.q, st.q, tpr);
                if (rq == 0 && acc_on) fold(bl, a.ds1, a.ds2, i, np + i, x);
                if (kp) {
                    const double y = dot_row<Real, RPT>(st.p, st.p, tpr);
                    if (rq == 0 && acc_on) fold(bl, a.dp_s1, a.dp_s2, i, nacc + np + i, y);
                }
            }
            Real xi[NS + 1][RPT];
#pragma unroll
            for (int c = 0; c <= NS; ++c)
                normals<Real, RPT>(a.key0, a.key1, a.stream, uint32_t(i), uint32_t(n), uint32_t(c), uint32_t(r0),
                                   xi[c]);
            if (a.tpart != nullptr) row_traces<Real, NS, RPT>(st, acc, tpr, tr);
            RowState<Real, NS, RPT> nx;
            ok = ou_update<Real, NS, RPT>(T, S, a.h, a.hh, st, acc, xi, nx) && ok;
            store_vec<Real, RPT>(qw + i * R + r0, nx.q);
            if (pp_pairs) store_vec<Real, RPT>(pb + ((n + 1) & 1) * N * R + i * R + r0, nx.p);
            st = nx;
        }
        if (a.tpart != nullptr) {  // one partial per step (a single tile)
            if (!active || rq != 0) tr[0] = tr[1] = tr[2] = 0.0;
            workgroup_sum3(tr, red);
            if (tid == 0)
                for (int c = 0; c < 3; ++c) a.tpart[int64_t(k) * a.tpart_w * 3 + c] = tr[c];
        }
        __syncthreads();
    }
    const int64_t nend = n0 + K;
    Real* qgo = (nend & 1) ? a.q1 : a.q0;
    if (active) {
        store_vec<Real, RPT>(qgo + i * R + r0, st.q);
        Real* psrow = ps_row(ps_at_step(a, nend), i, D, R, a.ps_lg) + r0;
        const int64_t cs = ps_stride(R, a.ps_lg);
        store_vec<Real, RPT>(psrow, st.p);
#pragma unroll
        for (int c = 0; c < NS; ++c) store_vec<Real, RPT>(psrow + (c + 1) * cs, st.s[c]);
    }
    for (int64_t x = tid; x < np; x += nthr) a.pblk[x] = bl[x];
    for (int64_t x = tid; x < nd; x += nthr) a.dblk[x] = bl[np + x];
    if (kp) {
        for (int64_t x = tid; x < np; x += nthr) a.pp_blk[x] = bl[nacc + x];
        for (int64_t x = tid; x < nd; x += nthr) a.dp_blk[x] = bl[nacc + np + x];
    }
    if (!ok) atomicOr(a.flag, 1);
    __syncthreads();
    if (tid == 0) const_cast<int64_t*>(a.step_base)[0] = nend;
}

template <typename Real, int NS, int MAXT>
const void* pick_small_rpt(int rpt) {
    switch (rpt) {
        case 1: return reinterpret_cast<const void*>(&small_dense_kernel<Real, NS, 1, MAXT>);
        case 2: return reinterpret_cast<const void*>(&small_dense_kernel<Real, NS, 2, MAXT>);
        case 4: return reinterpret_cast<const void*>(&small_dense_kernel<Real, NS, 4, MAXT>);
        default: return nullptr;
    }
}

template <typename Real, int MAXT>
const void* pick_small_ns(int ns, int rpt) {
    switch (ns) {
        case 0: return pick_small_rpt<Real, 0, MAXT>(rpt);
        case 1: return pick_small_rpt<Real, 1, MAXT>(rpt);
        case 2: return pick_small_rpt<Real, 2, MAXT>(rpt);
        case 3: return pick_small_rpt<Real, 3, MAXT>(rpt);
        case 4: return pick_small_rpt<Real, 4, MAXT>(rpt);
        case 5: return pick_small_rpt<Real, 5, MAXT>(rpt);
        case 6: return pick_small_rpt<Real, 6, MAXT>(rpt);
        case 7: return pick_small_rpt<Real, 7, MAXT>(rpt);
        case 8: return pick_small_rpt<Real, 8, MAXT>(rpt);
        case 9: return pick_small_rpt<Real, 9, MAXT>(rpt);
        case 10: return pick_small_rpt<Real, 10, MAXT>(rpt);
        default: return nullptr;
    }
}

// the instantiation with the smallest workgroup bound that admits `block` threads
template <typename Real>
const void* pick_small(int ns, int rpt, int block) {
    if (block <= 256) return pick_small_ns<Real, 256>(ns, rpt);
    if (block <= 512) return pick_small_ns<Real, 512>(ns, rpt);
    return pick_small_ns<Real, 1024>(ns, rpt);
}

}  // namespace dev

template <typename Real>
int launch_small_dense_impl(const StepArgs<Real>& a, const StepLaunch& L, int K, size_t lds_bytes, void* stream) {
    const int64_t threads = a.N << a.lg_tpr;
    const int block = int((threads + 63) / 64 * 64);
    if (block > 1024) return -3;
    const void* fn = dev::pick_small<Real>(L.ns, L.rpt, block);
    if (fn == nullptr) return -2;
    StepArgs<Real> copy = a;
    int k = K;
    void* args[] = {&copy, &k};
    hipError_t e = hipLaunchKernel(fn, dim3(1), dim3(unsigned(block)), args, lds_bytes, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

}  // namespace fth
