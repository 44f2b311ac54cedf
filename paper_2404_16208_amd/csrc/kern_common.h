// kern_common.h -- small device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranc {

// Sum of a 32-bit value over the 64 lanes of a wavefront (every lane gets it).
__device__ inline unsigned wave_sum(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += (unsigned)__shfl_xor((int)v, o, 64);
    return v;
}

// Potential update shared by every path (GPU-RANC Sec. II, LIF): the exact
// sum V + I + leak (64-bit) saturates to the potential range once per tick,
// the neuron fires when the result reaches its threshold and then takes its
// reset value.
__device__ inline bool lif_update(int32_t v, int32_t in, int32_t leak, int32_t thr, int32_t rst,
                                  int32_t vmin, int32_t vmax, int32_t &v_out)
{
    long long u = (long long)v + (long long)in + (long long)leak;
    u = u < vmin ? (long long)vmin : (u > vmax ? (long long)vmax : u);
    const bool fire = u >= (long long)thr;
    v_out = fire ? rst : (int32_t)u;
    return fire;
}

}  // namespace ranc
