// Persistent form of the temporally blocked sparse step.
//
// The arithmetic is the one-launch-per-tile blocked step's (tb_step.hpp):
// workgroup-sized row tiles, an extended range of E = T + 2 KT w rows per
// tile, q of the extended range in LDS, (p, s) and the row's entries in
// registers, KT steps per launch, every row computed exactly as the one-step
// kernel computes it.  What changes is the schedule:
//   - the grid holds as many workgroups as fit on the device at once, and
//     each walks a contiguous range of tiles (the ranges of the workgroups
//     that share an XCD are adjacent, so halo rows meet in that XCD's L2);
//   - while a workgroup computes the KT steps of tile t, the state and the
//     matrix rows of tile t+1 stream into a per-wave staging area of LDS
//     with 16-byte direct-to-LDS loads, which hold no registers;
//   - the matrix rows come from a slot form (TbSlotRow: values, one-byte
//     column offsets, count), so a row needs no row-pointer indirection and a
//     wave's rows are one contiguous byte range.
// A tile's loads are therefore in flight during the previous tile's
// compute, and the load phase that a one-tile workgroup spends waiting is
// gone.  Staging is wave-private: a wave reads back only what its own loads
// wrote, after waiting for them, so no barrier guards it.
#pragma once

#include <hip/hip_runtime.h>

#include "row_update.hpp"

namespace fth {
namespace dev {

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void global_void_t;

// 16 bytes from global memory into LDS: lane l of the wave writes
// dst + 16 l (dst is the wave's uniform base).
__device__ __forceinline__ void stage16(const void* src, char* dst_wave_base) {
    // C casts: the builtin takes address-space qualified pointers
    __builtin_amdgcn_global_load_lds((global_void_t*)(src), (lds_void_t*)(dst_wave_base), 16, 0, 0);
}

// 4 bytes from global memory into LDS: lane l of the wave writes dst + 4 l.
__device__ __forceinline__ void stage4(const void* src, char* dst_wave_base) {
    // C casts: the builtin takes address-space qualified pointers
    __builtin_amdgcn_global_load_lds((global_void_t*)(src), (lds_void_t*)(dst_wave_base), 4, 0, 0);
}

__device__ __forceinline__ double stage_f64(const char* aux, int word, int lane) {
    const uint32_t lo = *reinterpret_cast<const uint32_t*>(aux + word * 256 + lane * 4);
    const uint32_t hi = *reinterpret_cast<const uint32_t*>(aux + (word + 1) * 256 + lane * 4);
    return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// s_waitcnt encodings (gfx9 family): vmcnt(0) with the other counters open,
// and lgkmcnt(0) with the other counters open.
constexpr int kWaitVm0 = 0x0F70;
constexpr int kWaitLgkm0 = 0xC07F;

template <typename Real, int RPT>
__device__ __forceinline__ Vec<Real, RPT> stage_vec(const char* wbase, int instr, int lane) {
    // a thread's RPT replicas are VI consecutive 16-byte pieces, piece v in
    // load slot instr + v
    constexpr int VI = int(sizeof(Real)) * RPT / 16;
    Vec<Real, RPT> v;
#pragma unroll
    for (int p = 0; p < VI; ++p) {
        const float4 x = *reinterpret_cast<const float4*>(wbase + (instr + p) * 1024 + lane * 16);
        *reinterpret_cast<float4*>(reinterpret_cast<char*>(v.v) + 16 * p) = x;
    }
    return v;
}

template <typename Real, int NS, int KT, bool XTRA>
__global__ __launch_bounds__(tb_max_block(sizeof(Real) == 8, NS, XTRA)) void tbp_step_kernel(const StepArgs<Real> a,
                                                                                             const TbArgs<Real> tb,
                                                                                             const int k) {
    extern __shared__ double tb_smem[];
    constexpr int RPT = 4;
    constexpr int D = NS + 1;
    constexpr int VI = int(sizeof(Real)) * RPT / 16;  // 16-byte loads per 4-replica vector
    constexpr int NSI = (NS + 2) * VI;                // state loads per thread: q, p, s_1..s_ns
    constexpr int SB = int(sizeof(TbSlotRow<Real>));
    using V = Vec<Real, RPT>;
    const int64_t R = a.R;
    const int E = tb.E, T = tb.T, w = tb.w, H = KT * tb.w;
    const int lg = a.lg_tpr, tpr = 1 << lg;
    const int rq = int(threadIdx.x) & (tpr - 1), r0 = rq * RPT;
    const int e = int(threadIdx.x) >> lg;  // row within the extended range
    const int lane = int(threadIdx.x) & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);  // uniform in the wave: scalar
    const int rows_per_wave = 64 >> lg;
    const int CI = (rows_per_wave * SB + 1023) / 1024;
    constexpr int AUX = kTbpAuxWords;

    Real* qlds = reinterpret_cast<Real*>(tb_smem);  // [2][E][R]
    double* trl = reinterpret_cast<double*>(qlds + int64_t(2) * E * R);
    char* stage_base = reinterpret_cast<char*>(trl + (XTRA && a.tpart != nullptr ? 2 * T * 3 : 0));
    // per wave: NSI state loads, CI slot-row loads (1 KB each), AUX words (256 B each)
    char* wst = stage_base + wave * ((NSI + CI) * 1024 + AUX * 256);
    char* waux = wst + (NSI + CI) * 1024;
    // with the momentum and trace accumulators the row's matrix values live in
    // LDS for the tile ([E][8], shared by the row's lanes) instead of in eight
    // registers per thread, which the extra accumulators need
    Real* vlds = reinterpret_cast<Real*>(stage_base + (int(blockDim.x) >> 6) * ((NSI + CI) * 1024 + AUX * 256));

    // contiguous tile range of this workgroup; workgroups are dealt to the 8
    // XCDs round-robin, so those of one XCD get adjacent ranges
    const int64_t G = gridDim.x;
    const int64_t b = blockIdx.x;
    const int64_t L = (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
    const int64_t t_begin = L * a.row_tiles / G, t_end = (L + 1) * a.row_tiles / G;
    if (t_begin >= t_end) return;  // whole workgroup

    const int64_t n0 = a.step_base[0] + k;
    const Real* __restrict__ qg = (n0 & 1) ? a.q1 : a.q0;
    Real* __restrict__ qgo = ((n0 + KT) & 1) ? a.q1 : a.q0;
    const Real* psg = ps_at_step(a, n0);
    Real* psgo = ps_at_step(a, n0 + KT);
    const int64_t cs = ps_stride(R, a.ps_lg);
    const char* slots = static_cast<const char*>(tb.slots);
    const int64_t Nm1 = a.N - 1;

    // Stage tile t: this thread's state, and the wave's slot rows as one
    // byte range.  Rows outside [0, N) load row 0 or N-1 instead (never used),
    // so every lane issues the same loads and no branch depends on the data.
    auto issue = [&](int64_t t, int e, int r0, int lane) {
        const int64_t i = min(max(t * T - H + e, int64_t(0)), Nm1);
        const char* qsrc = reinterpret_cast<const char*>(qg + i * R + r0);
#pragma unroll
        for (int v = 0; v < VI; ++v) stage16(qsrc + 16 * v, wst + v * 1024);
        const char* psrc = reinterpret_cast<const char*>(ps_row(psg, i, D, R, a.ps_lg) + r0);
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
            for (int v = 0; v < VI; ++v)
                stage16(psrc + c * cs * int64_t(sizeof(Real)) + 16 * v, wst + ((1 + c) * VI + v) * 1024);
        const int64_t wrow0 = t * T - H + int64_t(wave) * rows_per_wave;
        for (int c = 0; c < CI; ++c) {
            const int chunk = c * 64 + lane;
            const int rw = min(chunk * 16 / SB, rows_per_wave - 1);
            const int64_t row = min(max(wrow0 + rw, int64_t(0)), Nm1);
            const int in_row = chunk * 16 - rw * SB;  // offset inside the row (clamped chunks repeat the last)
            stage16(slots + row * SB + min(in_row, SB - 16), wst + (NSI + c) * 1024);
        }
        if (a.dblk != nullptr) {
            stage4(reinterpret_cast<const char*>(a.dblk + i), waux);
            stage4(reinterpret_cast<const char*>(a.dblk + i) + 4, waux + 256);
        }
        if (tb.pair_slot != nullptr) stage4(tb.pair_slot + i, waux + 512);
    };
    // The momentum-form block sum of a row is prefetched into a register
    // instead (LDS holds no room for it at 1024 threads); the tile-start wait
    // for the staged loads covers it too.  Only output rows use it, and a row
    // is an output row of one tile only, so no other tile writes it meanwhile.
    auto fetch_blkp = [&](int64_t t, int e) -> double {
        if (!(XTRA && a.dp_blk != nullptr)) return 0.0;
        return a.dp_blk[min(max(t * T - H + e, int64_t(0)), Nm1)];
    };

    const Real* T_ = a.TS;
    const Real* S_ = a.TS + D * D;
    bool ok = true;
    issue(t_begin, e, r0, lane);
    double blkp_next = fetch_blkp(t_begin, e);
#pragma unroll 1
    for (int64_t t = t_begin; t < t_end; ++t) {
        // Per-tile copies of the thread's coordinates that the compiler must
        // treat as changing every tile: address arithmetic derived from them
        // is redone per tile instead of being hoisted and kept live (which
        // spills at the register budget of 1024 threads).
        int e_t = e, r0_t = r0, lane_t = lane;
        asm volatile("" : "+v"(e_t), "+v"(r0_t), "+v"(lane_t));
        const int64_t i = t * T - H + e_t;
        const bool row_ok = i >= 0 && i < a.N;
        const bool output = row_ok && e >= H && e < H + T;
        __builtin_amdgcn_s_waitcnt(kWaitVm0);  // this wave's staging of tile t has landed
        double blk = 0.0, blkp = 0.0;
        int32_t pslot = -1;
        if (output && rq == 0) {
            if (a.dblk != nullptr) blk = stage_f64(waux, 0, lane_t);
            if (XTRA && a.dp_blk != nullptr) blkp = blkp_next;
        }
        if (output && tb.pair_slot != nullptr) pslot = *reinterpret_cast<const int32_t*>(waux + 512 + lane_t * 4);
        RowState<Real, NS, RPT> st;
        st.q = stage_vec<Real, RPT>(wst, 0, lane_t);
        st.p = stage_vec<Real, RPT>(wst, VI, lane_t);
#pragma unroll
        for (int c = 0; c < NS; ++c) st.s[c] = stage_vec<Real, RPT>(wst, (2 + c) * VI, lane_t);
        const TbSlotRow<Real>* srow = reinterpret_cast<const TbSlotRow<Real>*>(wst + NSI * 1024 + (lane_t >> lg) * SB);
        Real dval[8];
        if constexpr (XTRA) {
            for (int u = rq; u < 8; u += tpr) vlds[e_t * 8 + u] = srow->val[u];
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) dval[u] = srow->val[u];
        }
        // column offsets stay packed (two registers) and are unpacked at use
        const uint64_t offs = *reinterpret_cast<const uint64_t*>(srow->off);
        const int nz = srow->nz;
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);  // staging read into registers before it is refilled
        if (t + 1 < t_end) {
            issue(t + 1, e_t, r0_t, lane_t);
            blkp_next = fetch_blkp(t + 1, e_t);
        }
        store_vec<Real, RPT>(qlds + int64_t(e_t) * R + r0_t, st.q);
        __syncthreads();

#pragma unroll 1
        for (int s = 0; s < KT; ++s) {
            const int64_t n = n0 + s;
            const bool acc_on = n >= a.burn_in;
            const bool close = acc_on && ((n - a.burn_in + 1) % a.block_len) == 0;
            const Real* cur = qlds + int64_t(s & 1) * E * R;
            Real* nxt = qlds + int64_t((s + 1) & 1) * E * R;
            // the row index as the compiler must treat it in each step: the block
            // sums' addresses are then formed where a block closes (rarely) instead
            // of being kept live across the step loop
            int64_t i_s = i;
            asm volatile("" : "+v"(i_s));
            // with the extra accumulators, the neighbour offsets are unpacked in each
            // step (not once per tile into eight registers)
            uint64_t offs_s = offs;
            if constexpr (XTRA) asm volatile("" : "+v"(offs_s));
            if (output) {
                if (a.dblk != nullptr) {
                    const double x = dot_row<Real, RPT>(st.q, st.q, tpr);
                    if (rq == 0 && acc_on) {
                        blk = blk + x;
                        if (close) {
                            a.ds1[i_s] = a.ds1[i_s] + blk;
                            a.ds2[i_s] = a.ds2[i_s] + blk * blk;
                            blk = 0.0;
                        }
                    }
                }
                if (XTRA && a.dp_blk != nullptr) {
                    const double y = dot_row<Real, RPT>(st.p, st.p, tpr);
                    if (rq == 0 && acc_on) {
                        blkp = blkp + y;
                        if (close) {
                            a.dp_s1[i_s] = a.dp_s1[i_s] + blkp;
                            a.dp_s2[i_s] = a.dp_s2[i_s] + blkp * blkp;
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
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nz) {
                        const int dc = int(int8_t(uint8_t(offs_s >> (8 * u))));
                        const V qj = load_vec<Real, RPT>(cur + int64_t(e + dc) * R + r0);
                        const Real mv = XTRA ? vlds[e * 8 + u] : dval[u];
#pragma unroll
                        for (int m = 0; m < RPT; ++m) acc[m] = fmaR(mv, qj.v[m], acc[m]);
                    }
                Real xi[NS + 1][RPT];
#pragma unroll
                for (int c = 0; c <= NS; ++c)
                    normals<Real, RPT>(a.key0, a.key1, a.stream, uint32_t(i), uint32_t(n), uint32_t(c),
                                       uint32_t(r0), xi[c]);
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
            store_state<Real, RPT, true>(qgo + i * R + r0_t, st.q);
            Real* psrow = ps_row(psgo, i, D, R, a.ps_lg) + r0_t;
            store_state<Real, RPT, true>(psrow, st.p);
#pragma unroll
            for (int c = 0; c < NS; ++c) store_state<Real, RPT, true>(psrow + (c + 1) * cs, st.s[c]);
            if (a.dblk != nullptr && rq == 0) a.dblk[i] = blk;
            if (XTRA && a.dp_blk != nullptr && rq == 0) a.dp_blk[i] = blkp;
        }
    }
    if (!ok) atomicOr(a.flag, 1);
}

// Slot form of CSR rows of at most 8 entries (one thread per row).
template <typename Real>
__global__ void tb_slots_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                const Real* __restrict__ val, int64_t N, TbSlotRow<Real>* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t kb = row_ptr[i];
    const int nz = int(min(row_ptr[i + 1] - kb, int64_t(8)));
    TbSlotRow<Real> r;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        r.val[u] = u < nz ? val[kb + u] : Real(0);
        r.off[u] = u < nz ? int8_t(int64_t(col[kb + u]) - i) : int8_t(0);
    }
    r.nz = nz;
    r.pad = 0;
    out[i] = r;
}

template <typename Real, int KT, bool X>
const void* pick_tbp_ns(int ns) {
    switch (ns) {
        case 0: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 0, KT, X>);
        case 1: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 1, KT, X>);
        case 2: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 2, KT, X>);
        case 3: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 3, KT, X>);
        case 4: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 4, KT, X>);
        case 5: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 5, KT, X>);
        case 6: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 6, KT, X>);
        case 7: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 7, KT, X>);
        case 8: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 8, KT, X>);
        case 9: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 9, KT, X>);
        case 10: return reinterpret_cast<const void*>(&tbp_step_kernel<Real, 10, KT, X>);
        default: return nullptr;
    }
}

template <typename Real>
const void* pick_tbp(int ns, int KT, bool x) {
    if (KT == 3) return x ? pick_tbp_ns<Real, 3, true>(ns) : pick_tbp_ns<Real, 3, false>(ns);
    if (KT == 5) return x ? pick_tbp_ns<Real, 5, true>(ns) : pick_tbp_ns<Real, 5, false>(ns);
    return nullptr;
}

}  // namespace dev

template <typename Real>
int launch_tbp_step_impl(const StepArgs<Real>& a, const TbArgs<Real>& tb, const StepLaunch& L, int KT, int k,
                         void* stream) {
    if (L.rpt != 4 || tb.slots == nullptr || tb.grid <= 0) return -2;
    const bool x = a.pp_blk != nullptr || a.dp_blk != nullptr || a.tpart != nullptr;
    const void* fn = dev::pick_tbp<Real>(L.ns, KT, x);
    if (fn == nullptr) return -2;
    const int block = tb.E << a.lg_tpr;
    if (block > tb_max_block(sizeof(Real) == 8, L.ns, x) || block % 64 != 0) return -3;
    const size_t lds = tbp_lds_bytes(sizeof(Real) == 8, L.ns, block, a.R, tb.T, a.tpart != nullptr, x);
    StepArgs<Real> aa = a;
    TbArgs<Real> tt = tb;
    int kk = k;
    void* args[] = {&aa, &tt, &kk};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(tb.grid)), dim3(unsigned(block)), args, lds,
                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

template <typename Real>
int tbp_resident_grid_impl(int ns, int KT, bool xtra, int block, size_t lds) {
    const void* fn = dev::pick_tbp<Real>(ns, KT, xtra);
    if (fn == nullptr) return 0;
    int dev_id = 0, cus = 0, max_lds = 0;
    if (hipGetDevice(&dev_id) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id) != hipSuccess) return 0;
    if (lds > size_t(max_lds)) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess) return 0;
    return per_cu * cus;
}

template <typename Real>
int launch_tb_slots_impl(const int64_t* row_ptr, const int32_t* col, const Real* val, int64_t N, void* out,
                         void* stream) {
    const int64_t grid = (N + 255) / 256;
    hipLaunchKernelGGL(dev::tb_slots_kernel<Real>, dim3(unsigned(grid)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), row_ptr, col, val, N, static_cast<TbSlotRow<Real>*>(out));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fth
