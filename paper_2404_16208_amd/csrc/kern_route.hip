// kern_route.hip -- router + scheduler write of one tick, and state reset.
//
// GPU-RANC Sec. III-D writes each spike's bit straight into the destination
// core's scheduler SRAM at the packet's tick offset. Here that write is done
// from the destination side instead, so that no two lanes ever write the same
// word and no atomics are needed: the routing table is inverted at load time
// into, for every (destination core, axon word, delay), the list of source
// neurons that send there (rt_ptr / rt_src). The lane that owns destination
// word (core, w) of one sample gathers the spike bits of those sources, ORs
// them into a 32-bit word per delay d, and ORs each non-zero word into
// scheduler slot (t + d) % Q, which only it writes. Arrivals at the same
// (core, axon, tick) therefore merge into one bit (the scheduler SRAM holds
// booleans, Sec. III-E). The same lane clears slot t % Q, which this tick's
// integration has already read (the clear of the obsolete row that Sec.
// III-E does at the start of the next tick).
//
// The sample's current spike bitmap (C*N/32 words) is staged in LDS when it
// fits, so the gather reads LDS; otherwise it is read from global memory.
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int ROUTE_THREADS = 1024;
static constexpr int ROUTE_LDS_WORDS = 16384;  // 64 KiB

template <bool STAGE>
__global__ __launch_bounds__(ROUTE_THREADS) void k_route(DevNet n, int q_now)
{
    extern __shared__ uint32_t sp[];
    const int s = blockIdx.y;
    const size_t words = (size_t)n.C * n.NW;
    const uint32_t *src = n.spk + (size_t)s * words;
    if (STAGE) {
        for (size_t i = threadIdx.x; i < words; i += blockDim.x)
            sp[i] = src[i];
        __syncthreads();
    }
    const int CW = n.C * n.W;
    const size_t slot_stride = (size_t)n.S * CW;
    uint32_t *ring_s = n.ring + (size_t)s * CW;
    for (int dw = blockIdx.x * blockDim.x + threadIdx.x; dw < CW; dw += gridDim.x * blockDim.x) {
        ring_s[(size_t)q_now * slot_stride + dw] = 0u;
        const uint32_t *p = n.rt_ptr + (size_t)dw * n.D;
        uint32_t beg = p[0];
        for (int d = 1; d <= n.D; ++d) {
            const uint32_t end = p[d];
            uint32_t acc = 0;
            for (uint32_t e = beg; e < end; ++e) {
                const uint32_t ent = n.rt_src[e];
                const uint32_t g = ent >> 5;
                const uint32_t wd = STAGE ? sp[g >> 5] : src[g >> 5];
                acc |= ((wd >> (g & 31u)) & 1u) << (ent & 31u);
            }
            beg = end;
            if (acc) {
                int q = q_now + d;
                if (q >= n.Q)
                    q -= n.Q;
                ring_s[(size_t)q * slot_stride + dw] |= acc;
            }
        }
    }
}

hipError_t launch_route(const DevNet &n, int q_now, hipStream_t st)
{
    const int CW = n.C * n.W;
    const size_t words = (size_t)n.C * n.NW;
    if (n.S > 65535)
        return hipErrorInvalidValue;
    int per_sample = (CW + ROUTE_THREADS - 1) / ROUTE_THREADS;
    if (words <= (size_t)ROUTE_LDS_WORDS) {
        // Every block of a sample stages that sample's bitmap; use several
        // blocks per sample only while the grid is small.
        int want = (512 + n.S - 1) / n.S;
        int bx = want < per_sample ? want : per_sample;
        if (bx < 1)
            bx = 1;
        hipLaunchKernelGGL(k_route<true>, dim3(bx, n.S), dim3(ROUTE_THREADS), words * sizeof(uint32_t),
                           st, n, q_now);
    } else {
        hipLaunchKernelGGL(k_route<false>, dim3(per_sample, n.S), dim3(ROUTE_THREADS), 0, st, n, q_now);
    }
    return hipGetLastError();
}

__global__ void k_reset_potentials(DevNet n)
{
    const size_t total = (size_t)n.C * n.S * n.N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / ((size_t)n.S * n.N);
        const size_t j = i % n.N;
        n.V[i] = n.vinit[c * n.N + j];
    }
}

__global__ void k_fill_u32(uint32_t *p, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_reset_state(const DevNet &n, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_potentials, dim3(2048), dim3(256), 0, st, n);
    const size_t ring_words = (size_t)n.Q * n.S * n.C * n.W;
    const size_t spk_words = (size_t)n.S * n.C * n.NW;
    const size_t raster_words = (size_t)n.RT * n.S * n.Wout;
    const size_t cnt_words = (size_t)n.C * n.S * CNT_N * 2;
    hipLaunchKernelGGL(k_fill_u32, dim3(2048), dim3(256), 0, st, n.ring, ring_words);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, n.spk, spk_words);
    if (raster_words)
        hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, n.raster, raster_words);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, (uint32_t *)n.cnt, cnt_words);
    return hipGetLastError();
}

}  // namespace ranc
