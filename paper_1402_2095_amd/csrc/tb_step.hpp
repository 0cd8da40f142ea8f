// Temporally blocked sparse step for matrices of small half-bandwidth w:
// one launch advances the system by KT steps.
//
// Workgroup t owns output rows [t T, t T + T) and loads an extended range of
// E = T + 2 H rows with H = KT w.  After step s (0-based) a row's value is
// exact if its neighbours were exact before it, so the exact region shrinks
// by w rows on each side per step; after KT steps it is exactly the output
// range.  Rows are computed only while they can still reach the output.
//   - q of the extended range lives in LDS (two buffers, q_n and q_{n+1}),
//     followed, with trace estimators, by two [T][3] buffers of row sums;
//   - p, s and the CSR row live in registers for the whole launch;
//   - the diagonal block sum of an output row lives in a register; s1 / s2
//     are updated in global memory only when a block closes;
//   - q (and p, with p-p accumulators) of output rows that appear in a
//     selected pair is copied each step to a snapshot buffer; a second small
//     kernel then forms the pair products step by step, in the same order as
//     the one-step kernel.
// Global state is double-buffered, so no workgroup can read a halo row that
// another workgroup of the same launch has already written back: q and
// (p, s) are read from buffer n0 & 1 and written to (n0 + KT) & 1 (KT odd).
// The arithmetic of each row and step is exactly the one-step kernel's
// (same gather order, noise, update), so trajectories are bit-identical.
#pragma once

#include <hip/hip_runtime.h>

#include "row_update.hpp"

namespace fth {
namespace dev {

// XTRA: momentum-form or trace accumulators are kept (compiled out otherwise,
// which keeps the common form within the register budget of 1024 threads).
template <typename Real, int NS, int RPT, int KT, bool XTRA>
__global__ __launch_bounds__(tb_max_block(sizeof(Real) == 8, NS, XTRA)) void tb_step_kernel(const StepArgs<Real> a, const TbArgs<Real> tb, const int k) {
    extern __shared__ double tb_smem[];
    Real* qlds = reinterpret_cast<Real*>(tb_smem);  // [2][E][R]
    constexpr int G = 8;                             // CSR entries per row (at most)
    constexpr int D = NS + 1;
    using V = Vec<Real, RPT>;
    const int64_t R = a.R;
    const int E = tb.E, T = tb.T, w = tb.w, H = KT * tb.w;
    const int lg = a.lg_tpr, tpr = 1 << lg;
    const int rq = int(threadIdx.x) & (tpr - 1), r0 = rq * RPT;
    const int e = int(threadIdx.x) >> lg;  // row within the extended range
    const int64_t per = a.row_tiles_padded >> 3;
    const int64_t b = blockIdx.x;
    const int64_t t = (b & 7) * per + (b >> 3);
    if (t >= a.row_tiles) return;  // whole workgroup: no barrier is skipped by part of it
    const int64_t i = t * T - H + e;
    const bool row_ok = e < E && i >= 0 && i < a.N;
    const bool output = row_ok && e >= H && e < H + T;
    const int64_t n0 = a.step_base[0] + k;
    const Real* __restrict__ qg = (n0 & 1) ? a.q1 : a.q0;
    Real* __restrict__ qgo = ((n0 + KT) & 1) ? a.q1 : a.q0;

    RowState<Real, NS, RPT> st;
    int dcol[G];
    Real dval[G];
    // with the extra accumulators the row's values live in LDS ([E][8], after q
    // and the trace rows) and its column offsets in one packed register pair,
    // which keeps the thread within the register budget without spills
    Real* vlds = reinterpret_cast<Real*>(reinterpret_cast<char*>(qlds) + size_t(2) * E * R * sizeof(Real) +
                                         (a.tpart != nullptr ? size_t(2) * T * 3 * sizeof(double) : 0));
    uint64_t offs = 0;
    int nz = 0;
    double blk = 0.0, blkp = 0.0;
    int32_t pslot = -1;
    if (row_ok) {
        st.q = load_vec<Real, RPT>(qg + i * R + r0);
        const Real* psrow = ps_row(ps_at_step(a, n0), i, D, R, a.ps_lg) + r0;
        const int64_t cs = ps_stride(R, a.ps_lg);
        st.p = load_vec<Real, RPT>(psrow);
#pragma unroll
        for (int c = 0; c < NS; ++c) st.s[c] = load_vec<Real, RPT>(psrow + (c + 1) * cs);
        const int64_t kb = a.row_ptr[i], ke = a.row_ptr[i + 1];
        nz = int(ke - kb);
        if constexpr (XTRA) {
            for (int u = rq; u < G; u += tpr) vlds[e * G + u] = u < nz ? a.val[kb + u] : Real(0);
#pragma unroll
            for (int u = 0; u < G; ++u)
                offs |= uint64_t(uint8_t(int8_t(u < nz ? int(a.col[kb + u] - i) : 0))) << (8 * u);
        } else {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                dcol[u] = u < nz ? int(a.col[kb + u] - i) : 0;
                dval[u] = u < nz ? a.val[kb + u] : Real(0);
            }
        }
        store_vec<Real, RPT>(qlds + int64_t(e) * R + r0, st.q);
        if (output && a.dblk != nullptr && rq == 0) blk = a.dblk[i];
        if (XTRA && output && a.dp_blk != nullptr && rq == 0) blkp = a.dp_blk[i];
        if (output && tb.pair_slot != nullptr) pslot = tb.pair_slot[i];
    }
    const Real* T_ = a.TS;
    const Real* S_ = a.TS + D * D;
    bool ok = true;
    __syncthreads();

    // trace sums of the output rows, [step parity][T][3] after q in LDS: written
    // by the first lane of each row, summed by wave 0 after the step's barrier
    // while the other waves go on (the next step writes the other half)
    double* trl = reinterpret_cast<double*>(qlds + int64_t(2) * E * R);
#pragma unroll 1
    for (int s = 0; s < KT; ++s) {
        const int64_t n = n0 + s;
        const bool acc_on = n >= a.burn_in;
        const bool close = acc_on && ((n - a.burn_in + 1) % a.block_len) == 0;
        const Real* cur = qlds + int64_t(s & 1) * E * R;
        Real* nxt = qlds + int64_t((s + 1) & 1) * E * R;
        if (output) {
            if (a.dblk != nullptr) {
                const double x = dot_row<Real, RPT>(st.q, st.q, tpr);
                if (rq == 0 && acc_on) {
                    blk = blk + x;
                    if (close) {
                        a.ds1[i] = a.ds1[i] + blk;
                        a.ds2[i] = a.ds2[i] + blk * blk;
                        blk = 0.0;
                    }
                }
            }
            if (XTRA && a.dp_blk != nullptr) {
                const double y = dot_row<Real, RPT>(st.p, st.p, tpr);
                if (rq == 0 && acc_on) {
                    blkp = blkp + y;
                    if (close) {
                        a.dp_s1[i] = a.dp_s1[i] + blkp;
                        a.dp_s2[i] = a.dp_s2[i] + blkp * blkp;
                        blkp = 0.0;
                    }
                }
            }
            if (pslot >= 0) {
                store_vec<Real, RPT>(tb.snap + (int64_t(2 * s) * tb.nslots + pslot) * R + r0, st.q);
                if (XTRA && a.pp_blk != nullptr)
                    store_vec<Real, RPT>(tb.snap + (int64_t(2 * s + 1) * tb.nslots + pslot) * R + r0, st.p);
            }
        }
        // rows still needed after this step: e in [(s+1) w, E - (s+1) w)
        if (row_ok && e >= (s + 1) * w && e < E - (s + 1) * w) {
            Real acc[RPT];
#pragma unroll
            for (int m = 0; m < RPT; ++m) acc[m] = Real(0);
            uint64_t offs_s = offs;
            if constexpr (XTRA) asm volatile("" : "+v"(offs_s));   // unpacked in each step
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (u < nz) {
                    const int dc = XTRA ? int(int8_t(uint8_t(offs_s >> (8 * u)))) : dcol[u];
                    const V qj = load_vec<Real, RPT>(cur + int64_t(e + dc) * R + r0);
                    const Real mv = XTRA ? vlds[e * G + u] : dval[u];
#pragma unroll
                    for (int m = 0; m < RPT; ++m) acc[m] = fmaR(mv, qj.v[m], acc[m]);
                }
            Real xi[NS + 1][RPT];
#pragma unroll
            for (int c = 0; c <= NS; ++c)
                normals<Real, RPT>(a.key0, a.key1, a.stream, uint32_t(i), uint32_t(n), uint32_t(c), uint32_t(r0),
                                   xi[c]);
            if (XTRA && output && a.tpart != nullptr) {
                double tr[3];
                row_traces<Real, NS, RPT>(st, acc, tpr, tr);
                if (rq == 0)
                    for (int c = 0; c < 3; ++c) trl[((s & 1) * T + (e - H)) * 3 + c] = tr[c];
            }
            RowState<Real, NS, RPT> nx;
            ok = ou_update<Real, NS, RPT>(T_, S_, a.h, a.hh, st, acc, xi, nx) && ok;
            store_vec<Real, RPT>(nxt + int64_t(e) * R + r0, nx.q);
            st = nx;
        }
        __syncthreads();
        if (XTRA && a.tpart != nullptr && threadIdx.x < 64) {  // wave 0: the T output rows in a fixed order
            const int64_t nout = min(int64_t(T), a.N - t * T);
            double v[3] = {0.0, 0.0, 0.0};
            for (int64_t r = threadIdx.x; r < nout; r += 64)
                for (int c = 0; c < 3; ++c) v[c] += trl[((s & 1) * T + r) * 3 + c];
            for (int c = 0; c < 3; ++c)
                for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
            if (threadIdx.x == 0)
                for (int c = 0; c < 3; ++c) a.tpart[(int64_t(k + s) * a.tpart_w + t) * 3 + c] = v[c];
        }
    }
    if (output) {
        store_state<Real, RPT, true>(qgo + i * R + r0, st.q);
        Real* psrow = ps_row(ps_at_step(a, n0 + KT), i, D, R, a.ps_lg) + r0;
        const int64_t cs = ps_stride(R, a.ps_lg);
        store_state<Real, RPT, true>(psrow, st.p);
#pragma unroll
        for (int c = 0; c < NS; ++c) store_state<Real, RPT, true>(psrow + (c + 1) * cs, st.s[c]);
        if (a.dblk != nullptr && rq == 0) a.dblk[i] = blk;
        if (XTRA && a.dp_blk != nullptr && rq == 0) a.dp_blk[i] = blkp;
        if (!ok) atomicOr(a.flag, 1);
    }
}

// Pair products from the step snapshots, KT steps in order.
template <typename Real, int RPT, int KT>
__global__ __launch_bounds__(256) void tb_pairs_kernel(const StepArgs<Real> a, const TbArgs<Real> tb, const int k) {
    const int lg = a.lg_tpr, tpr = 1 << lg;
    const int rq = int(threadIdx.x) & (tpr - 1), r0 = rq * RPT;
    const int64_t pk = int64_t(blockIdx.x) * (int(blockDim.x) >> lg) + (int(threadIdx.x) >> lg);
    if (pk >= a.npairs) return;
    const int64_t R = a.R;
    const int32_t si = tb.pair_slots[2 * pk], sj = tb.pair_slots[2 * pk + 1];
    const int64_t n0 = a.step_base[0] + k;
    for (int s = 0; s < KT; ++s) {
        const int64_t n = n0 + s;
        const bool acc_on = n >= a.burn_in;
        const bool close = acc_on && ((n - a.burn_in + 1) % a.block_len) == 0;
        const Real* sq = tb.snap + int64_t(2 * s) * tb.nslots * R + r0;
        const double x = dot_row<Real, RPT>(load_vec<Real, RPT>(sq + si * R), load_vec<Real, RPT>(sq + sj * R), tpr);
        if (rq == 0 && acc_on) acc_update(a.pblk, a.ps1, a.ps2, pk, x, close);
        if (a.pp_blk != nullptr) {
            const Real* sp = tb.snap + int64_t(2 * s + 1) * tb.nslots * R + r0;
            const double y =
                dot_row<Real, RPT>(load_vec<Real, RPT>(sp + si * R), load_vec<Real, RPT>(sp + sj * R), tpr);
            if (rq == 0 && acc_on) acc_update(a.pp_blk, a.pp_s1, a.pp_s2, pk, y, close);
        }
    }
}

template <typename Real, int KT, bool X>
const void* pick_tb_ns(int ns) {
    switch (ns) {
        case 0: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 0, 4, KT, X>);
        case 1: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 1, 4, KT, X>);
        case 2: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 2, 4, KT, X>);
        case 3: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 3, 4, KT, X>);
        case 4: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 4, 4, KT, X>);
        case 5: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 5, 4, KT, X>);
        case 6: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 6, 4, KT, X>);
        case 7: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 7, 4, KT, X>);
        case 8: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 8, 4, KT, X>);
        case 9: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 9, 4, KT, X>);
        case 10: return reinterpret_cast<const void*>(&tb_step_kernel<Real, 10, 4, KT, X>);
        default: return nullptr;
    }
}

}  // namespace dev

// Supported: replicas per thread 4, KT in {3, 5}.
template <typename Real>
int launch_tb_step_impl(const StepArgs<Real>& a, const TbArgs<Real>& tb, const StepLaunch& L, int KT, int k,
                        void* stream) {
    if (L.rpt != 4) return -2;
    const bool x = a.pp_blk != nullptr || a.dp_blk != nullptr || a.tpart != nullptr;
    const void* fn = KT == 3 ? (x ? dev::pick_tb_ns<Real, 3, true>(L.ns) : dev::pick_tb_ns<Real, 3, false>(L.ns))
                     : KT == 5 ? (x ? dev::pick_tb_ns<Real, 5, true>(L.ns) : dev::pick_tb_ns<Real, 5, false>(L.ns))
                               : nullptr;
    if (fn == nullptr) return -2;
    const int block = tb.E << a.lg_tpr;
    if (block > tb_max_block(sizeof(Real) == 8, L.ns, x) || block % 64 != 0) return -3;
    const size_t lds = size_t(2) * size_t(tb.E) * size_t(a.R) * sizeof(Real) +
                       (a.tpart != nullptr ? size_t(2) * size_t(tb.T) * 3 * sizeof(double) : 0) +
                       (x ? size_t(tb.E) * 8 * sizeof(Real) : 0);
    StepArgs<Real> aa = a;
    TbArgs<Real> tt = tb;
    int kk = k;
    void* args[] = {&aa, &tt, &kk};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(a.row_tiles_padded)), dim3(unsigned(block)), args, lds,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

template <typename Real>
int launch_tb_pairs_impl(const StepArgs<Real>& a, const TbArgs<Real>& tb, const StepLaunch& L, int KT, int k,
                         void* stream) {
    if (a.npairs == 0) return 0;
    if (L.rpt != 4) return -2;
    const void* fn = KT == 3   ? reinterpret_cast<const void*>(&dev::tb_pairs_kernel<Real, 4, 3>)
                     : KT == 5 ? reinterpret_cast<const void*>(&dev::tb_pairs_kernel<Real, 4, 5>)
                               : nullptr;
    if (fn == nullptr) return -2;
    const int per_block = 256 >> a.lg_tpr;
    const int64_t grid = (a.npairs + per_block - 1) / per_block;
    StepArgs<Real> aa = a;
    TbArgs<Real> tt = tb;
    int kk = k;
    void* args[] = {&aa, &tt, &kk};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(256), args, 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

}  // namespace fth
