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

// Workgroup barrier that orders LDS only: wait for this wave's LDS accesses,
// then s_barrier. __syncthreads() (and an LDS-scoped fence, which also covers
// global-to-LDS DMA) makes every wave wait for all of its outstanding global
// loads, including prefetches meant to stay in flight across the barrier.
// Kernels whose waves exchange data only through ordinary LDS accesses use
// this; the "memory" clobber keeps the compiler from moving memory accesses
// across it. A wave reading its own global-to-LDS DMA data waits for it
// separately (s_waitcnt vmcnt).
__device__ inline void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Compiler-only barrier: keeps issued memory operations where they are.
__device__ inline void compiler_fence()
{
    asm volatile("" ::: "memory");
}

// Potential update shared by every path (GPU-RANC Sec. II, LIF): the sum
// V + I + leak saturates to the potential range once per tick, the neuron
// fires when the result U reaches its threshold and then takes its reset
// value. |I| <= 512 * 256 and |leak| <= 2^30 (checked at load), so I + leak is
// exact in int32 and one saturating 32-bit add gives clamp(V + I + leak) to
// the int32 range exactly; clamping that to [vmin, vmax] equals clamping the
// exact sum to the P-bit range.
// Neuron-model options (the design space of Sec. I and Sec. V): a neuron in
// linear-reset mode keeps U - threshold on a spike (U >= threshold there, so
// the difference is >= 0 and only its upper end needs a clamp: one saturating
// subtraction, then vmax); a neuron that does not fire keeps at least its
// floor (fl = vmin: no floor).
__device__ inline int32_t lif_reset(int32_t u, int32_t thr, int32_t rst, int32_t vmax, bool lin)
{
    return lin ? min(__builtin_elementwise_sub_sat(u, thr), vmax) : rst;
}

__device__ inline bool lif_update(int32_t v, int32_t in, int32_t leak, int32_t thr, int32_t rst,
                                  int32_t vmin, int32_t vmax, int32_t fl, bool lin, int32_t &v_out)
{
    int32_t u = __builtin_elementwise_add_sat(v, in + leak);
    u = min(max(u, vmin), vmax);
    const bool fire = u >= thr;
    v_out = fire ? lif_reset(u, thr, rst, vmax, lin) : max(u, fl);
    return fire;
}

}  // namespace ranc
