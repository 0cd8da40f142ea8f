// Counter-based Gaussian noise for the GLE thermostat, device side.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit
// multiplications by fixed odd constants, with a Weyl-sequence key schedule.
//
// Counter layout (one block = four normals, for four consecutive replicas):
//   key     = (seed mod 2^32, seed >> 32)
//   counter = (dof i, step n, (component j << 16) | (replica r >> 2), stream)
// Word w = r & 3 of the block belongs to replica r.  Each word x becomes
// u = (2 (x >> 9) + 1) 2^-24, an odd multiple of 2^-24 in (0, 1), exact in
// FP32 and FP64.  Box-Muller on words (0, 1) and (2, 3): the even word gives
// sqrt(-2 ln u_even) cos(2 pi u_odd), the odd word the same radius times
// sin(2 pi u_odd).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fth {
namespace dev {

struct Block4 {
    uint32_t w[4];
};

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = uint64_t(kMulA) * c0;
        const uint64_t pb = uint64_t(kMulB) * c2;
        // three-way XOR in one v_bitop3_b32 (truth table 0x96)
        const uint32_t x0 = __builtin_amdgcn_bitop3_b32(uint32_t(pb >> 32), c1, k0, 0x96);
        const uint32_t x2 = __builtin_amdgcn_bitop3_b32(uint32_t(pa >> 32), c3, k1, 0x96);
        c1 = uint32_t(pb);
        c3 = uint32_t(pa);
        c0 = x0;
        c2 = x2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Block4{{c0, c1, c2, c3}};
}

// u = (2 (x >> 9) + 1) 2^-24 in FP32 without a conversion: the top 23 bits
// as the mantissa of a float in [1, 2) give 1 + (x >> 9) 2^-23, and
// subtracting 1 - 2^-24 is exact (Sterbenz: both operands lie in [1/2, 2]).
// The bit pattern 0x3f800000 | (x >> 9) is the low word of the 64-bit value
// {0x7f, x} shifted right by 9: one v_alignbit_b32 instead of a shift and an or.
__device__ __forceinline__ float uniform_f32(uint32_t x) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, x, 9u)) - 0x1.fffffep-1f;
}

// Box-Muller in FP32 with the hardware transcendental unit: v_log_f32 is
// log2, v_sin_f32 / v_cos_f32 take their argument in revolutions, so
// sin(2 pi u) needs no multiply.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& zc, float& zs) {
    const float ua = uniform_f32(a);
    const float ub = uniform_f32(b);
    const float l2 = __builtin_amdgcn_logf(ua);                      // log2(ua) < 0
    const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * l2);  // sqrt(-2 ln ua)
    zc = rad * __builtin_amdgcn_cosf(ub);
    zs = rad * __builtin_amdgcn_sinf(ub);
}

// Box-Muller in FP64 with the device math library.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& zc, double& zs) {
    const double ua = __builtin_fma(double(a >> 9), 0x1p-23, 0x1p-24);
    const double ub = __builtin_fma(double(b >> 9), 0x1p-23, 0x1p-24);
    const double rad = sqrt(-2.0 * log(ua));
    double sn, cs;
    sincospi(2.0 * ub, &sn, &cs);
    zc = rad * cs;
    zs = rad * sn;
}

// Normals of component j for replicas r0 .. r0+RPT-1 (r0 a multiple of RPT;
// RPT in {1, 2, 4, 8}) at dof i, step n.
template <typename Real, int RPT>
__device__ __forceinline__ void normals(uint32_t k0, uint32_t k1, uint32_t stream, uint32_t i,
                                        uint32_t n, uint32_t j, uint32_t r0, Real* z) {
    if constexpr (RPT >= 4) {
#pragma unroll
        for (int g = 0; g < RPT / 4; ++g) {
            const Block4 b = philox4x32_10(i, n, (j << 16) | ((r0 >> 2) + g), stream, k0, k1);
            box_muller(b.w[0], b.w[1], z[4 * g + 0], z[4 * g + 1]);
            box_muller(b.w[2], b.w[3], z[4 * g + 2], z[4 * g + 3]);
        }
    } else {
        const Block4 b = philox4x32_10(i, n, (j << 16) | (r0 >> 2), stream, k0, k1);
        const bool hi = (r0 & 2u) != 0;
        Real zc, zs;
        box_muller(hi ? b.w[2] : b.w[0], hi ? b.w[3] : b.w[1], zc, zs);
        if constexpr (RPT == 2) {
            z[0] = zc;
            z[1] = zs;
        } else {
            z[0] = (r0 & 1u) ? zs : zc;
        }
    }
}

}  // namespace dev
}  // namespace fth
