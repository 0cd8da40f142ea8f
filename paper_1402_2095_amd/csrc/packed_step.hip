// Packed multi-request sparse step: one persistent launch advances every
// active request of a group (same ns, replicas per thread 4, FP32 state) by
// one step.  Work is a device list of tiles (request slot, row tile or pair
// tile); the request table holds each request's step arguments, including
// its own step counter, noise stream and block schedule, so a request's
// arithmetic does not depend on what else is packed with it.
//
// The grid is fixed (it does not depend on the tile count, which is read
// from device memory), so a captured graph of K steps stays valid while
// requests come and go.  The tile list is cut into 8 contiguous pieces, one
// per XCD (workgroups are dealt round-robin over the XCDs), so each XCD
// sweeps contiguous rows of a request.
#include "csr_step.hpp"

namespace fth {
namespace dev {

template <int NS, bool NT>
__global__ __launch_bounds__(256) void packed_csr_kernel(const StepArgs<float>* __restrict__ table,
                                                         const PackedTile* __restrict__ tiles,
                                                         const int32_t* __restrict__ ntiles_p, const int k) {
    constexpr int RPT = 4;
    const int ntiles = ntiles_p[0];
    const int per_xcd = int(gridDim.x >> 3);
    const int xcd = int(blockIdx.x & 7), local = int(blockIdx.x >> 3);
    const int chunk = (ntiles + 7) >> 3;
    const int end = min(ntiles, (xcd + 1) * chunk);
    for (int t = xcd * chunk + local; t < end; t += per_xcd) {
        const PackedTile tl = tiles[t];
        const StepArgs<float>& a = table[tl.slot];
        const StepInfo si = step_info<float, RPT>(a, k);
        const float* __restrict__ qr = (si.n & 1) ? a.q1 : a.q0;
        float* __restrict__ qw = (si.n & 1) ? a.q0 : a.q1;
        const int per_block = int(blockDim.x) >> a.lg_tpr;
        if (tl.pairs) {
            const int64_t pk = tl.index * per_block + si.slot;
            if (pk < a.npairs) pair_update<float, RPT>(a, si, qr, pk);
            continue;
        }
        const int64_t i = tl.index * per_block + si.slot;
        if (i < a.N) csr_row<float, NS, RPT, NT>(a, si, i, qr, qw, nullptr);  // no traces for packed requests
    }
}

// Advances the step counter of every live slot (the count is read on the
// device, so a captured graph follows the group's membership).
__global__ void advance_all_kernel(const StepArgs<float>* __restrict__ table, const int32_t* __restrict__ nslots_p,
                                   int64_t K) {
    const int nslots = nslots_p[0];
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) const_cast<int64_t*>(table[s].step_base)[0] += K;
}

template <bool NT>
const void* pick_packed(int ns) {
    switch (ns) {
        case 0: return reinterpret_cast<const void*>(&packed_csr_kernel<0, NT>);
        case 1: return reinterpret_cast<const void*>(&packed_csr_kernel<1, NT>);
        case 2: return reinterpret_cast<const void*>(&packed_csr_kernel<2, NT>);
        case 3: return reinterpret_cast<const void*>(&packed_csr_kernel<3, NT>);
        case 4: return reinterpret_cast<const void*>(&packed_csr_kernel<4, NT>);
        case 5: return reinterpret_cast<const void*>(&packed_csr_kernel<5, NT>);
        case 6: return reinterpret_cast<const void*>(&packed_csr_kernel<6, NT>);
        case 7: return reinterpret_cast<const void*>(&packed_csr_kernel<7, NT>);
        case 8: return reinterpret_cast<const void*>(&packed_csr_kernel<8, NT>);
        case 9: return reinterpret_cast<const void*>(&packed_csr_kernel<9, NT>);
        case 10: return reinterpret_cast<const void*>(&packed_csr_kernel<10, NT>);
        default: return nullptr;
    }
}

}  // namespace dev

int launch_packed_csr(const StepArgs<float>* table, const PackedTile* tiles, const int32_t* ntiles, int ns, bool nt,
                      int grid, int k, void* stream) {
    const void* fn = nt ? dev::pick_packed<true>(ns) : dev::pick_packed<false>(ns);
    if (fn == nullptr) return -2;
    if (grid <= 0 || grid % 8 != 0) return -3;
    void* args[] = {const_cast<StepArgs<float>**>(&table), const_cast<PackedTile**>(&tiles),
                    const_cast<int32_t**>(&ntiles), &k};
    hipError_t e = hipLaunchKernel(fn, dim3(unsigned(grid)), dim3(256), args, 0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : -1;
}

int launch_advance_all(const StepArgs<float>* table, const int32_t* nslots, int64_t K, void* stream) {
    hipLaunchKernelGGL(dev::advance_all_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), table,
                       nslots, K);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fth
