// Per-row GLE update shared by the sparse step kernel and the dense
// epilogue: given acc = (M q_n)_i for the thread's replicas, apply
//   diagonal accumulator (FP64, block averaged) from q_n,
//   p += (h/2) F;  (p, s) <- T (p, s) + S xi;  p += (h/2) F;  q' = q + h p
// with F = -acc, and store p, s and q_{n+1}.
//
// Thread mapping: row i is served by TPR = R / RPT consecutive lanes; lane rq
// owns replicas [rq*RPT, rq*RPT + RPT).  q is [rows][R]; the thermostat part
// is interleaved per row as ps[rows][ns+1][R] (p first), so one row's
// momenta are a single contiguous (ns+1)*R block.
#pragma once

#include <hip/hip_runtime.h>

#include "fth_internal.h"
#include "noise.hpp"

namespace fth {
namespace dev {

template <typename Real, int RPT>
struct alignas(sizeof(Real) * RPT) Vec {
    Real v[RPT];
};

template <typename Real, int RPT>
__device__ __forceinline__ Vec<Real, RPT> load_vec(const Real* p) {
    return *reinterpret_cast<const Vec<Real, RPT>*>(p);
}

template <typename Real, int RPT>
__device__ __forceinline__ void store_vec(Real* p, const Vec<Real, RPT>& v) {
    *reinterpret_cast<Vec<Real, RPT>*>(p) = v;
}

// Streaming (non-temporal) forms for state that is touched once per step:
// when the state does not fit the 256 MB Infinity Cache, keeping it out of
// L2/MALL leaves those caches to the data that is reused.
template <typename Real, int RPT, bool NT>
__device__ __forceinline__ Vec<Real, RPT> load_state(const Real* p) {
    if constexpr (NT) {
        Vec<Real, RPT> v;
#pragma unroll
        for (int m = 0; m < RPT; ++m) v.v[m] = __builtin_nontemporal_load(p + m);
        return v;
    } else {
        return load_vec<Real, RPT>(p);
    }
}

template <typename Real, int RPT, bool NT>
__device__ __forceinline__ void store_state(Real* p, const Vec<Real, RPT>& v) {
    if constexpr (NT) {
#pragma unroll
        for (int m = 0; m < RPT; ++m) __builtin_nontemporal_store(v.v[m], p + m);
    } else {
        store_vec<Real, RPT>(p, v);
    }
}

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Block-averaging accumulator update (one element, one step).
__device__ __forceinline__ void acc_update(double* blk, double* s1, double* s2, int64_t idx, double x,
                                           bool close) {
    const double b = blk[idx] + x;
    if (close) {
        s1[idx] = s1[idx] + b;
        s2[idx] = s2[idx] + b * b;
        blk[idx] = 0.0;
    } else {
        blk[idx] = b;
    }
}

__device__ __forceinline__ double group_sum(double x, int tpr) {
    for (int off = tpr >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Per-step constants every launch derives from the device step counter.
struct StepInfo {
    int64_t n;     // global step index
    bool acc_on;   // n >= burn_in
    bool close;    // this step closes a block
    int rq, r0, slot, tpr;
};

template <typename Real, int RPT>
__device__ __forceinline__ StepInfo step_info(const StepArgs<Real>& a, int k) {
    StepInfo s;
    s.n = a.step_base[0] + k;
    s.acc_on = s.n >= a.burn_in;
    s.close = s.acc_on && ((s.n - a.burn_in + 1) % a.block_len) == 0;
    s.tpr = 1 << a.lg_tpr;
    s.rq = threadIdx.x & (s.tpr - 1);
    s.r0 = s.rq * RPT;
    s.slot = threadIdx.x >> a.lg_tpr;
    return s;
}

// (p, s) of row i: rows are grouped by 2^lg, and inside a group each component
// is a contiguous [2^lg][R] block, so one component of a group spans at least
// a 128-byte line whatever R is.  Returns the row's component-0 slice;
// component c is at + c * ps_stride(R, lg).
template <typename Real>
__device__ __forceinline__ Real* ps_row(Real* ps, int64_t i, int D, int64_t R, int lg) {
    return ps + ((((i >> lg) * D) << lg) + (i & ((int64_t(1) << lg) - 1))) * R;
}
__device__ __forceinline__ int64_t ps_stride(int64_t R, int lg) { return R << lg; }

// (p, s) at step n is in buffer n & 1; step n writes step n+1's into the other.
template <typename Real>
__device__ __forceinline__ Real* ps_at_step(const StepArgs<Real>& a, int64_t n) {
    return (n & 1) ? a.ps_b : a.ps;
}

// FP64 sum over the thread's replicas of x_m y_m, then over the row's lanes.
template <typename Real, int RPT>
__device__ __forceinline__ double dot_row(const Vec<Real, RPT>& x, const Vec<Real, RPT>& y, int tpr) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) s += double(x.v[m]) * double(y.v[m]);
    return group_sum(s, tpr);
}

// Selected pairs: sum_r q_i^r q_j^r from q_n (and sum_r p_i^r p_j^r from p_n
// when p-p accumulators are kept) into the pair accumulators.
template <typename Real, int RPT>
__device__ __forceinline__ void pair_update(const StepArgs<Real>& a, const StepInfo& si, const Real* qr, int64_t pk) {
    using V = Vec<Real, RPT>;
    const int64_t R = a.R;
    const int64_t pi = a.pairs[2 * pk], pj = a.pairs[2 * pk + 1];
    const V qi = load_vec<Real, RPT>(qr + pi * R + si.r0);
    const V qj = load_vec<Real, RPT>(qr + pj * R + si.r0);
    const double x = dot_row<Real, RPT>(qi, qj, si.tpr);
    if (si.rq == 0 && si.acc_on) acc_update(a.pblk, a.ps1, a.ps2, pk, x, si.close);
    if (a.pp_blk != nullptr) {
        const Real* psr = ps_at_step(a, si.n);
        const V p_i = load_vec<Real, RPT>(ps_row(psr, pi, a.D(), R, a.ps_lg) + si.r0);
        const V p_j = load_vec<Real, RPT>(ps_row(psr, pj, a.D(), R, a.ps_lg) + si.r0);
        const double y = dot_row<Real, RPT>(p_i, p_j, si.tpr);
        if (si.rq == 0 && si.acc_on) acc_update(a.pp_blk, a.pp_s1, a.pp_s2, pk, y, si.close);
    }
}

// The thread's slice of one row's state.
template <typename Real, int NS, int RPT>
struct RowState {
    Vec<Real, RPT> q, p;
    Vec<Real, RPT> s[NS > 0 ? NS : 1];
};

template <typename Real, int NS, int RPT, bool NT>
__device__ __forceinline__ RowState<Real, NS, RPT> load_row(const StepArgs<Real>& a, const StepInfo& si,
                                                            const Real* qr, int64_t i) {
    RowState<Real, NS, RPT> st;
    const int64_t R = a.R;
    const int r0 = si.r0;
    constexpr int D = NS + 1;
    st.q = load_vec<Real, RPT>(qr + i * R + r0);
    const Real* psrow = ps_row(ps_at_step(a, si.n), i, D, R, a.ps_lg) + r0;
    const int64_t cs = ps_stride(R, a.ps_lg);
    st.p = load_state<Real, RPT, NT>(psrow);
#pragma unroll
    for (int c = 0; c < NS; ++c) st.s[c] = load_state<Real, RPT, NT>(psrow + (c + 1) * cs);
    return st;
}

template <typename Real, int NS, int RPT>
__device__ __forceinline__ void row_noise(const StepArgs<Real>& a, const StepInfo& si, int64_t i,
                                          Real (&xi)[NS + 1][RPT]) {
#pragma unroll
    for (int c = 0; c <= NS; ++c)
        normals<Real, RPT>(a.key0, a.key1, a.stream, uint32_t(i), uint32_t(si.n), uint32_t(c), uint32_t(si.r0),
                           xi[c]);
}

// Kicks, exact OU step and drift on registers: from (q, p, s) and
// acc = (M q)_i produce (q', p', s').  Returns false if a value is not finite.
template <typename Real, int NS, int RPT>
__device__ __forceinline__ bool ou_update(const Real* T, const Real* S, Real h, Real hh,
                                          const RowState<Real, NS, RPT>& st, const Real (&acc)[RPT],
                                          const Real (&xi)[NS + 1][RPT], RowState<Real, NS, RPT>& out) {
    constexpr int D = NS + 1;
    bool ok = true;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const Real f = -acc[m];
        Real x[D];
        x[0] = fmaR(hh, f, st.p.v[m]);
#pragma unroll
        for (int c = 0; c < NS; ++c) x[c + 1] = st.s[c].v[m];
        Real y[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            Real v = Real(0);
#pragma unroll
            for (int c = 0; c < D; ++c) v = fmaR(T[r * D + c], x[c], v);
#pragma unroll
            for (int c = 0; c <= r; ++c) v = fmaR(S[r * D + c], xi[c][m], v);
            y[r] = v;
        }
        const Real pnew = fmaR(hh, f, y[0]);
        out.p.v[m] = pnew;
#pragma unroll
        for (int c = 0; c < NS; ++c) out.s[c].v[m] = y[c + 1];
        out.q.v[m] = fmaR(h, pnew, st.q.v[m]);
        ok = ok && __builtin_isfinite(out.q.v[m]) && __builtin_isfinite(pnew);
    }
    return ok;
}

// Row sums behind the trace estimators: q^2, q (M q) and p^2 over the row's
// replicas (identical in every lane of the row); acc holds (M q)_i.
template <typename Real, int NS, int RPT>
__device__ __forceinline__ void row_traces(const RowState<Real, NS, RPT>& st, const Real (&acc)[RPT], int tpr,
                                           double (&tr)[3]) {
    double qm = 0.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) qm += double(st.q.v[m]) * double(acc[m]);
    tr[0] = dot_row<Real, RPT>(st.q, st.q, tpr);
    tr[1] = group_sum(qm, tpr);
    tr[2] = dot_row<Real, RPT>(st.p, st.p, tpr);
}

// Sum of the rows' trace slots trl[0..nrows)[3] by wave 0, in a fixed order
// (strided per lane, then an xor butterfly); call after a barrier.  Lane 0
// writes the three sums to out.
__device__ __forceinline__ void wave0_sum_rows(const double* trl, int64_t nrows, double* out) {
    if (threadIdx.x >= 64) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t r = threadIdx.x; r < nrows; r += 64)
        for (int c = 0; c < 3; ++c) v[c] += trl[r * 3 + c];
    for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) out[c] = v[c];
}

// Workgroup sum of three values held by the first lane of every row (other
// lanes pass 0), in a fixed order: lanes of a wave by xor butterfly, then the
// waves in index order.  Every thread of the workgroup must call it.
__device__ __forceinline__ void workgroup_sum3(double (&v)[3], double* red /* [16][3] LDS */) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
    const int wave = int(threadIdx.x) >> 6, lane = int(threadIdx.x) & 63;
    if (lane == 0)
        for (int c = 0; c < 3; ++c) red[wave * 3 + c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = int(blockDim.x + 63) >> 6;
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[w * 3 + c];
            v[c] = s;
        }
    }
}

// Diagonal accumulation, kicks, exact OU step, drift and stores.  Returns
// q_{n+1} for the thread's replicas.  With trace partials kept, the row's
// trace sums go to trow[0..2] (an LDS slot of the row) before the update, so
// nothing extra stays live through it.
template <typename Real, int NS, int RPT, bool NT>
__device__ __forceinline__ Vec<Real, RPT> finish_row(const StepArgs<Real>& a, const StepInfo& si, int64_t i,
                                                     const RowState<Real, NS, RPT>& st, const Real (&acc)[RPT],
                                                     const Real (&xi)[NS + 1][RPT], Real* qw, double* trow) {
    constexpr int D = NS + 1;
    const int64_t R = a.R;
    if (a.dblk != nullptr) {
        const double x = dot_row<Real, RPT>(st.q, st.q, si.tpr);
        if (si.rq == 0 && si.acc_on) acc_update(a.dblk, a.ds1, a.ds2, i, x, si.close);
    }
    if (a.dp_blk != nullptr) {
        const double y = dot_row<Real, RPT>(st.p, st.p, si.tpr);
        if (si.rq == 0 && si.acc_on) acc_update(a.dp_blk, a.dp_s1, a.dp_s2, i, y, si.close);
    }
    if (trow != nullptr) {
        double tr[3];
        row_traces<Real, NS, RPT>(st, acc, si.tpr, tr);
        if (si.rq == 0)
            for (int c = 0; c < 3; ++c) trow[c] = tr[c];
    }
    RowState<Real, NS, RPT> nx;
    const bool ok = ou_update<Real, NS, RPT>(a.TS, a.TS + D * D, a.h, a.hh, st, acc, xi, nx);
    Real* psrow = ps_row(ps_at_step(a, si.n + 1), i, D, R, a.ps_lg) + si.r0;
    const int64_t cs = ps_stride(R, a.ps_lg);
    store_state<Real, RPT, NT>(psrow, nx.p);
#pragma unroll
    for (int c = 0; c < NS; ++c) store_state<Real, RPT, NT>(psrow + (c + 1) * cs, nx.s[c]);
    store_state<Real, RPT, NT>(qw + i * R + si.r0, nx.q);
    if (!ok) atomicOr(a.flag, 1);
    return nx.q;
}

}  // namespace dev
}  // namespace fth
