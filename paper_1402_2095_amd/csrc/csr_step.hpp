// Fused sparse time step of the GLE-thermostatted harmonic system (one
// launch per step), templated on the state precision, the number of extra
// GLE momenta NS, the replicas handled per thread RPT and streaming state
// access NT.
//
// Per thread (row i, replicas [r0, r0+RPT)) and step:
//   1. issue the loads: own q, p, s and the first batch of the CSR row with
//      its gathered neighbour q rows;
//   2. generate the normals for components 0..NS (no memory; covers the load
//      latency; half of the waves do this before step 1, see noise_first);
//   3. acc = sum_k val[k] q_n[col[k]] in stored order;
//   4. the shared row update: diagonal accumulator, kicks, exact OU step,
//      drift (row_update.hpp).
// Off-diagonal pairs are extra workgroups of the same launch: they read q_n
// only, which no workgroup of this launch writes (q_{n+1} goes to the other
// buffer).
//
// Row tiles are mapped XCD-contiguously: the hardware deals consecutive
// workgroups round-robin to the 8 XCDs, so workgroup b takes tile
// (b mod 8) * (tiles / 8) + b / 8 and each XCD sweeps one contiguous slab of
// rows, keeping the neighbour rows its gathers touch in its own L2.
#pragma once

#include <hip/hip_runtime.h>

#include "row_update.hpp"

namespace fth {
namespace dev {

// Half of the waves draw their normals before issuing their loads, the
// other half while the loads are in flight.  A step is about one round of
// waves per SIMD, so with a single order every wave would load, compute and
// store in the same phase; the split keeps memory and the ALUs busy
// together (the values drawn are the same either way).  Measured on the 64^3
// Laplacian: 21.0 us per step against 21.6 us with one order (and 24.6 us
// with the two orders as separate instantiations, which the compiler lays
// out worse).
__device__ __forceinline__ bool noise_first() { return ((blockIdx.x + (threadIdx.x >> 6)) & 1) != 0; }

// One row of one request: gather, noise, force, shared row update.
// LONG: rows of more than 16 entries (the M1 lattice has 81).  Past the first
// batch, such rows gather GL entries per batch instead of four: each batch is
// a chain of two dependent loads (column indices, then the rows they name),
// so a long row costs (nnz - 4) / GL chains instead of (nnz - 4) / 4.  The
// products are still added in stored order, so the result is the same.
template <typename Real, int NS, int RPT, bool NT, bool LONG = false>
__device__ __forceinline__ void csr_row(const StepArgs<Real>& a, const StepInfo& si, int64_t i, const Real* qr,
                                        Real* qw, double* trow) {
    using V = Vec<Real, RPT>;
    const int64_t R = a.R;
    // CSR entries gathered per batch: four keeps the kernel near 80 VGPRs (six waves
    // per SIMD), which measured faster than eight entries at 92-114 VGPRs
    constexpr int G = 4;
    constexpr int GL = LONG ? (RPT >= 8 ? 8 : 16) : G;
    Real xi[NS + 1][RPT];
    const bool early = noise_first();
    if (early) row_noise<Real, NS, RPT>(a, si, i, xi);
    const int64_t kb = a.row_ptr[i], ke = a.row_ptr[i + 1];
    const RowState<Real, NS, RPT> st = load_row<Real, NS, RPT, NT>(a, si, qr, i);
    V qj[G];
    Real vj[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        vj[u] = Real(0);
        if (kb + u < ke) {
            vj[u] = a.val[kb + u];
            qj[u] = load_vec<Real, RPT>(qr + int64_t(a.col[kb + u]) * R + si.r0);
        }
    }

    if (!early) row_noise<Real, NS, RPT>(a, si, i, xi);

    Real acc[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) acc[m] = Real(0);
#pragma unroll
    for (int u = 0; u < G; ++u)
        if (kb + u < ke) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) acc[m] = fmaR(vj[u], qj[u].v[m], acc[m]);
        }
    for (int64_t base = kb + G; base < ke; base += GL) {  // rows longer than one batch
        V ql[GL];
        Real vl[GL];
        int32_t cl[GL];
#pragma unroll
        for (int u = 0; u < GL; ++u) {
            vl[u] = Real(0);
            cl[u] = 0;
            if (base + u < ke) {
                vl[u] = a.val[base + u];
                cl[u] = a.col[base + u];
            }
        }
#pragma unroll
        for (int u = 0; u < GL; ++u)
            if (base + u < ke) ql[u] = load_vec<Real, RPT>(qr + int64_t(cl[u]) * R + si.r0);
#pragma unroll
        for (int u = 0; u < GL; ++u)
            if (base + u < ke) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) acc[m] = fmaR(vl[u], ql[u].v[m], acc[m]);
            }
    }
    (void)finish_row<Real, NS, RPT, NT>(a, si, i, st, acc, xi, qw, trow);
}

// One row in the coded form: the row's 8 column codes and 8 value codes are
// two 8-byte loads; codes index the offset and value tables staged in LDS.
// Slots keep the CSR order, so the sum is the plain form's, bit for bit.
template <typename Real, int NS, int RPT, bool NT>
__device__ __forceinline__ void coded_row(const StepArgs<Real>& a, const StepInfo& si, int64_t i, const Real* qr,
                                          Real* qw, const int32_t* s_off, const Real* s_val, double* trow) {
    using V = Vec<Real, RPT>;
    const int64_t R = a.R;
    constexpr int G = 4;  // slots gathered per batch (two batches)
    Real xi[NS + 1][RPT];
    const bool early = noise_first();
    if (early) row_noise<Real, NS, RPT>(a, si, i, xi);
    const uint64_t cc = a.ell_col[i];
    const uint64_t vc = a.ell_vcode != nullptr ? a.ell_vcode[i] : 0;
    const RowState<Real, NS, RPT> st = load_row<Real, NS, RPT, NT>(a, si, qr, i);
    auto value = [&](int u) -> Real {
        return a.ell_vcode != nullptr ? s_val[(vc >> (8 * u)) & 255u] : a.ell_vraw[i * kCodedSlots + u];
    };
    V qj[G];
    Real vj[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const uint32_t code = uint32_t(cc >> (8 * u)) & 255u;
        vj[u] = Real(0);
        if (code != 255u) {
            vj[u] = value(u);
            qj[u] = load_vec<Real, RPT>(qr + (i + s_off[code]) * R + si.r0);
        }
    }
    if (!early) row_noise<Real, NS, RPT>(a, si, i, xi);
    Real acc[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) acc[m] = Real(0);
#pragma unroll
    for (int u = 0; u < G; ++u)
        if (((cc >> (8 * u)) & 255u) != 255u) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) acc[m] = fmaR(vj[u], qj[u].v[m], acc[m]);
        }
    if ((cc >> (8 * G)) != ~uint64_t(0) >> (8 * G)) {  // second batch not empty
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const uint32_t code = uint32_t(cc >> (8 * (G + u))) & 255u;
            vj[u] = Real(0);
            if (code != 255u) {
                vj[u] = value(G + u);
                qj[u] = load_vec<Real, RPT>(qr + (i + s_off[code]) * R + si.r0);
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u)
            if (((cc >> (8 * (G + u))) & 255u) != 255u) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) acc[m] = fmaR(vj[u], qj[u].v[m], acc[m]);
            }
    }
    (void)finish_row<Real, NS, RPT, NT>(a, si, i, st, acc, xi, qw, trow);
}

// TR: trace partials are kept (a separate instantiation, so the common form
// carries none of their code or registers).
// LONG: the plain form with long-row gather batches (see csr_row).
template <typename Real, int NS, int RPT, bool NT, bool CODED, bool TR, bool LONG = false>
__global__ __launch_bounds__(256) void csr_step_kernel(const StepArgs<Real> a, const int k) {
    const StepInfo si = step_info<Real, RPT>(a, k);
    const Real* __restrict__ qr = (si.n & 1) ? a.q1 : a.q0;
    Real* __restrict__ qw = (si.n & 1) ? a.q0 : a.q1;
    const int per_block = blockDim.x >> a.lg_tpr;
    const int64_t b = blockIdx.x;
    __shared__ int32_t s_off[CODED ? kCodedMaxOffsets : 1];
    __shared__ Real s_val[CODED ? kCodedMaxValues : 1];
    if constexpr (CODED) {  // every thread reaches the barrier
        for (int t = int(threadIdx.x); t < a.n_off; t += int(blockDim.x)) s_off[t] = a.dict_off[t];
        for (int t = int(threadIdx.x); t < a.n_val; t += int(blockDim.x)) s_val[t] = a.dict_val[t];
        __syncthreads();
    }

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
    if (i < a.N) {
        if constexpr (CODED)
            coded_row<Real, NS, RPT, NT>(a, si, i, qr, qw, s_off, s_val, trow);
        else
            csr_row<Real, NS, RPT, NT, LONG>(a, si, i, qr, qw, trow);
    }
    if constexpr (TR) {
        __syncthreads();
        wave0_sum_rows(trl, min(int64_t(per_block), a.N - t * per_block), a.tpart + (int64_t(k) * a.tpart_w + t) * 3);
    }
}

// ---------------------------------------------------------------- dispatch
template <template <typename, int, int, bool> class K, typename Real, int NS, bool NT>
struct PickRpt {
    static const void* get(int rpt) {
        switch (rpt) {
            case 1: return K<Real, NS, 1, NT>::fn();
            case 2: return K<Real, NS, 2, NT>::fn();
            case 4: return K<Real, NS, 4, NT>::fn();
            case 8: return K<Real, NS, 8, NT>::fn();
            default: return nullptr;
        }
    }
};

template <template <typename, int, int, bool> class K, typename Real, bool NT>
const void* pick_ns(int ns, int rpt) {
    switch (ns) {
        case 0: return PickRpt<K, Real, 0, NT>::get(rpt);
        case 1: return PickRpt<K, Real, 1, NT>::get(rpt);
        case 2: return PickRpt<K, Real, 2, NT>::get(rpt);
        case 3: return PickRpt<K, Real, 3, NT>::get(rpt);
        case 4: return PickRpt<K, Real, 4, NT>::get(rpt);
        case 5: return PickRpt<K, Real, 5, NT>::get(rpt);
        case 6: return PickRpt<K, Real, 6, NT>::get(rpt);
        case 7: return PickRpt<K, Real, 7, NT>::get(rpt);
        case 8: return PickRpt<K, Real, 8, NT>::get(rpt);
        case 9: return PickRpt<K, Real, 9, NT>::get(rpt);
        case 10: return PickRpt<K, Real, 10, NT>::get(rpt);
        default: return nullptr;
    }
}

template <template <typename, int, int, bool> class K, typename Real>
const void* pick_kernel(const StepLaunch& L) {
    return L.nt ? pick_ns<K, Real, true>(L.ns, L.rpt) : pick_ns<K, Real, false>(L.ns, L.rpt);
}

template <bool TR>
struct CsrKernels {
    template <typename Real, int NS, int RPT, bool NT>
    struct Plain {
        static const void* fn() {
            return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, RPT, NT, false, TR>);
        }
    };
    // The coded and long-row forms are instantiated for 4 and 8 replicas per thread only.
    template <typename Real, int NS, int RPT, bool NT>
    struct Coded {
        static const void* fn() {
            if constexpr (RPT >= 4)
                return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, RPT, NT, true, TR>);
            else
                return nullptr;
        }
    };
    template <typename Real, int NS, int RPT, bool NT>
    struct Long {
        static const void* fn() {
            if constexpr (RPT >= 4)
                return reinterpret_cast<const void*>(&csr_step_kernel<Real, NS, RPT, NT, false, TR, true>);
            else
                return nullptr;
        }
    };
};

template <typename Real>
int launch_step_kernel(const void* fn, const StepArgs<Real>& a, const StepLaunch& L, int k, void* stream) {
    if (fn == nullptr) return -2;
    const int64_t grid = a.row_tiles_padded + L.pair_tiles;
    if (grid <= 0) return 0;
    if (grid > 0x7FFFFFFF) return -3;
    void* args[] = {const_cast<StepArgs<Real>*>(&a), &k};
    const size_t lds = a.tpart != nullptr ? size_t(L.block >> a.lg_tpr) * 3 * sizeof(double) : 0;
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(unsigned(L.block)), args, lds,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

}  // namespace dev

// TR: the instantiations with trace partials (kept in a file of their own so
// the two halves compile in parallel).
template <typename Real, bool TR>
int launch_csr_step_impl(const StepArgs<Real>& a, const StepLaunch& L, int k, void* stream) {
    if (TR != (a.tpart != nullptr)) return -4;
    using KS = dev::CsrKernels<TR>;
    const void* fn = L.coded       ? dev::pick_kernel<KS::template Coded, Real>(L)
                     : L.long_rows ? dev::pick_kernel<KS::template Long, Real>(L)
                                   : dev::pick_kernel<KS::template Plain, Real>(L);
    return dev::launch_step_kernel<Real>(fn, a, L, k, stream);
}

}  // namespace fth
