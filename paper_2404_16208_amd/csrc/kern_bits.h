// kern_bits.h -- bit-matrix helpers shared by the sample-tiled kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranc {

// Sample (within its 32-sample group) of bit b of a history word. The order
// is the row order of the 32x32 MFMA result (lane l, element r is row
// 8*(r/4) + 4*(l/32) + r%4), so a lane's 16 results and its partner lane's
// form one word without reordering.
__device__ inline int sigma32(int b) { return 8 * ((b & 15) >> 2) + 4 * (b >> 4) + (b & 3); }

// Bit of sample i (within its 32-sample group) in a history word: the
// inverse of sigma32.
__device__ inline int sigma32_inv(int i) { return 16 * ((i & 7) >> 2) + 4 * (i >> 3) + (i & 3); }

// One stage of a recursive bit-matrix transpose: lanes whose index has bit K
// clear exchange the bits with index bit K set for their partner's (lane ^ K)
// bits with index bit K clear.
template <int K>
__device__ inline uint32_t transpose_stage(uint32_t x, int lane)
{
    constexpr uint32_t M = K == 16 ? 0x0000FFFFu : K == 8 ? 0x00FF00FFu : K == 4 ? 0x0F0F0F0Fu
                         : K == 2  ? 0x33333333u : 0x55555555u;
    // ds_swizzle bit-mask mode: partner = lane ^ K within each 32-lane half
    const uint32_t p = (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x1F | (K << 10));
    const bool up = (lane & K) != 0;
    const uint32_t r = __builtin_rotateright32(p, up ? K : 32 - K);
    const uint32_t keep = up ? ~M : M;
    return (x & keep) | (r & ~keep);
}

// 32 x 32 bit transpose within each half-wave: lane i of a half receives, as
// bit j, bit i of lane j of the same half. Every lane must be active.
__device__ inline uint32_t transpose32(uint32_t x, int lane)
{
    x = transpose_stage<16>(x, lane);
    x = transpose_stage<8>(x, lane);
    x = transpose_stage<4>(x, lane);
    x = transpose_stage<2>(x, lane);
    return transpose_stage<1>(x, lane);
}

}  // namespace ranc
