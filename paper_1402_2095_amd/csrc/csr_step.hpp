// Fused sparse time step of the GLE-thermostatted harmonic system (one
// launch per step), templated on the state precision, the number of extra
// GLE momenta NS and the replicas handled per thread RPT.
//
// Thread mapping: a row i of M is served by TPR = R / RPT consecutive lanes;
// lane rq owns replicas [rq*RPT, rq*RPT + RPT).  State is replica-innermost:
// q is [N][R] (ping-pong pair), the thermostat part (p, s_1..s_ns) is
// interleaved per row as ps[N][ns+1][R], so one row's momenta form a single
// contiguous (ns+1)*R block: the lanes of a wave stream one region for
// (p, s) instead of ns+1 separate arrays, and every matrix entry is reused R
// times.  Per thread and step:
//   1. gather the CSR row: acc = sum_k val[k] q_n[col[k]]   (stored order)
//   2. diagonal accumulator: sum over the row's replicas of q_i^2 in FP64,
//      butterfly-reduced across the TPR lanes, one lane updates the block sum
//   3. normals for components 0..NS (one Philox block per 4 replicas)
//   4. p += (h/2) F;  (p, s) <- T (p, s) + S xi;  p += (h/2) F;  q' = q + h p
// Off-diagonal pairs are extra blocks of the same launch: they read q_n only,
// which no block of this launch writes (q_{n+1} goes to the other buffer).
//
// Row tiles are mapped XCD-contiguously: the hardware deals consecutive
// workgroups round-robin to the 8 XCDs, so workgroup b takes tile
// (b mod 8) * (tiles / 8) + b / 8 and each XCD sweeps one contiguous slab of
// rows, keeping the neighbour rows its gathers touch in its own L2.
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
// L2/MALL leaves those caches to the gathered neighbour rows.
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

template <typename Real, int NS, int RPT, bool NT>
__global__ __launch_bounds__(256) void csr_step_kernel(const CsrStepArgs<Real> a, const int k) {
    constexpr int D = NS + 1;
    using V = Vec<Real, RPT>;
    const int64_t n = a.step_base[0] + k;
    const Real* __restrict__ qr = (n & 1) ? a.q1 : a.q0;
    Real* __restrict__ qw = (n & 1) ? a.q0 : a.q1;
    const int lg = a.lg_tpr;
    const int tpr = 1 << lg;
    const int rq = threadIdx.x & (tpr - 1);
    const int r0 = rq * RPT;
    const int slot = threadIdx.x >> lg;
    const int per_block = blockDim.x >> lg;
    const bool acc_on = n >= a.burn_in;
    const bool close = acc_on && ((n - a.burn_in + 1) % a.block_len) == 0;
    const int64_t b = blockIdx.x;
    const int64_t R = a.R;

    if (b >= a.row_tiles_padded) {
        // ---- off-diagonal (or any) selected pairs: sum_r q_i^r q_j^r ----
        const int64_t pk = (b - a.row_tiles_padded) * per_block + slot;
        if (pk >= a.npairs) return;
        const int64_t pi = a.pairs[2 * pk], pj = a.pairs[2 * pk + 1];
        const V qi = load_vec<Real, RPT>(qr + pi * R + r0);
        const V qj = load_vec<Real, RPT>(qr + pj * R + r0);
        double x = 0.0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) x += double(qi.v[m]) * double(qj.v[m]);
        x = group_sum(x, tpr);
        if (rq == 0 && acc_on) acc_update(a.pblk, a.ps1, a.ps2, pk, x, close);
        return;
    }

    const int64_t per = a.row_tiles_padded >> 3;
    const int64_t t = (b & 7) * per + (b >> 3);
    if (t >= a.row_tiles) return;
    const int64_t i = t * per_block + slot;
    if (i >= a.N) return;

    // Loads first (own state and the first chunk of the CSR row), then the
    // noise, which needs no memory and covers the load latency, then the
    // gather FMAs in stored order.
    constexpr int G = 8;  // CSR entries gathered per batch
    const int64_t kb = a.row_ptr[i], ke = a.row_ptr[i + 1];
    const V qi = load_vec<Real, RPT>(qr + i * R + r0);
    Real* __restrict__ psrow = a.ps + i * (D * R) + r0;  // p, s_1..s_NS of row i
    const V pv = load_state<Real, RPT, NT>(psrow);
    V sv[NS > 0 ? NS : 1];
#pragma unroll
    for (int c = 0; c < NS; ++c) sv[c] = load_state<Real, RPT, NT>(psrow + (c + 1) * R);

    int64_t cj[G];
    Real vj[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const bool in = kb + u < ke;
        cj[u] = in ? int64_t(a.col[kb + u]) : i;
        vj[u] = in ? a.val[kb + u] : Real(0);
    }
    V qj[G];
#pragma unroll
    for (int u = 0; u < G; ++u) qj[u] = load_vec<Real, RPT>(qr + cj[u] * R + r0);

    // normals (components 0..NS) while the loads are in flight
    Real xi[D][RPT];
#pragma unroll
    for (int c = 0; c < D; ++c)
        normals<Real, RPT>(a.key0, a.key1, a.stream, uint32_t(i), uint32_t(n), uint32_t(c), uint32_t(r0), xi[c]);

    // force: acc = sum_k val[k] q_n[col[k]] (F = -acc), stored order
    Real acc[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) acc[m] = Real(0);
#pragma unroll
    for (int u = 0; u < G; ++u)
        if (kb + u < ke) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) acc[m] = fmaR(vj[u], qj[u].v[m], acc[m]);
        }
    for (int64_t kk = kb + G; kk < ke; ++kk) {  // rows longer than one batch
        const int64_t j = a.col[kk];
        const Real v = a.val[kk];
        const V q = load_vec<Real, RPT>(qr + j * R + r0);
#pragma unroll
        for (int m = 0; m < RPT; ++m) acc[m] = fmaR(v, q.v[m], acc[m]);
    }

    // diagonal accumulator from q_n
    if (a.dblk != nullptr) {
        double x = 0.0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) x += double(qi.v[m]) * double(qi.v[m]);
        x = group_sum(x, tpr);
        if (rq == 0 && acc_on) acc_update(a.dblk, a.ds1, a.ds2, i, x, close);
    }

    // 4. kick, exact OU step, kick, drift
    const Real* T = a.TS;
    const Real* S = a.TS + D * D;
    V pn, qn;
    V sn[NS > 0 ? NS : 1];
    bool ok = true;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const Real f = -acc[m];
        Real x[D];
        x[0] = fmaR(a.hh, f, pv.v[m]);
#pragma unroll
        for (int c = 0; c < NS; ++c) x[c + 1] = sv[c].v[m];
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
        const Real pnew = fmaR(a.hh, f, y[0]);
        pn.v[m] = pnew;
#pragma unroll
        for (int c = 0; c < NS; ++c) sn[c].v[m] = y[c + 1];
        qn.v[m] = fmaR(a.h, pnew, qi.v[m]);
        ok = ok && __builtin_isfinite(qn.v[m]) && __builtin_isfinite(pnew);
    }
    store_state<Real, RPT, NT>(psrow, pn);
#pragma unroll
    for (int c = 0; c < NS; ++c) store_state<Real, RPT, NT>(psrow + (c + 1) * R, sn[c]);
    store_state<Real, RPT, NT>(qw + i * R + r0, qn);
    if (!ok) atomicOr(a.flag, 1);
}

template <typename Real, int NS, bool NT>
const void* pick_rpt(int rpt) {
    switch (rpt) {
        case 1: return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, 1, NT>);
        case 2: return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, 2, NT>);
        case 4: return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, 4, NT>);
        case 8: return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, 8, NT>);
        default: return nullptr;
    }
}

template <typename Real, bool NT>
const void* pick_ns(int ns, int rpt) {
    switch (ns) {
        case 0: return pick_rpt<Real, 0, NT>(rpt);
        case 1: return pick_rpt<Real, 1, NT>(rpt);
        case 2: return pick_rpt<Real, 2, NT>(rpt);
        case 3: return pick_rpt<Real, 3, NT>(rpt);
        case 4: return pick_rpt<Real, 4, NT>(rpt);
        case 5: return pick_rpt<Real, 5, NT>(rpt);
        case 6: return pick_rpt<Real, 6, NT>(rpt);
        case 7: return pick_rpt<Real, 7, NT>(rpt);
        case 8: return pick_rpt<Real, 8, NT>(rpt);
        case 9: return pick_rpt<Real, 9, NT>(rpt);
        case 10: return pick_rpt<Real, 10, NT>(rpt);
        default: return nullptr;
    }
}

template <typename Real>
const void* pick_csr_kernel(int ns, int rpt, bool nt) {
    return nt ? pick_ns<Real, true>(ns, rpt) : pick_ns<Real, false>(ns, rpt);
}

}  // namespace dev

template <typename Real>
int launch_csr_step_impl(const CsrStepArgs<Real>& a, const CsrLaunch& L, int k, void* stream) {
    const void* fn = dev::pick_csr_kernel<Real>(L.ns, L.rpt, L.nt);
    if (fn == nullptr) return -2;
    const int64_t grid = a.row_tiles_padded + L.pair_tiles;
    if (grid <= 0) return 0;
    if (grid > 0x7FFFFFFF) return -3;
    void* args[] = {const_cast<CsrStepArgs<Real>*>(&a), &k};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(unsigned(L.block)), args, 0,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

}  // namespace fth
