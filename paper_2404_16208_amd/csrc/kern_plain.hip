// kern_plain.hip -- one tick of integrate + leak/threshold/reset, plain path.
//
// One workgroup per (core, sample), one lane per neuron (N = 64..512 lanes).
// The tick's axon spikes of the core (scheduler slot OR external input) are
// A/32 words that every lane needs, so they are loaded with uniform (scalar)
// loads and pre-masked per axon type. Each lane then reads its neuron's
// crossbar column as A/32 words (coalesced across lanes: colbits is
// [C][W][N]) and counts, per axon type, the spiking connected axons with
// popcount; the input is sum_g count_g * weight[g] (GPU-RANC Sec. II: the
// axon type selects the neuron's weight). Spikes are gathered with a
// wavefront ballot into 32-bit words; output-bus spikes go to the raster.
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

template <int W_, int G_>
__global__ __launch_bounds__(512) void k_integrate_plain(DevNet n, TickArgs ta)
{
    const int c = blockIdx.x;
    const int s = blockIdx.y;
    const int j = threadIdx.x;
    const int N = n.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ unsigned red[8][4];

    // Axon spikes of this tick: scheduler slot t%Q OR the external input.
    const uint32_t *slot = n.ring + (((size_t)ta.q_now * n.S + s) * n.C + c) * W_;
    const int ci = n.in_index[c];
    const uint32_t *ext = (ta.ext_t != nullptr && ci >= 0)
                              ? ta.ext_t + (size_t)s * ta.ext_sstride + (size_t)ci * W_
                              : nullptr;
    uint32_t xt[G_][W_];
    unsigned delivered = 0;
#pragma unroll
    for (int w = 0; w < W_; ++w) {
        const uint32_t r = slot[w];
        delivered += __popc(r);
        const uint32_t x = r | (ext ? ext[w] : 0u);
#pragma unroll
        for (int g = 0; g < G_; ++g)
            xt[g][w] = x & n.typemask[((size_t)c * G_ + g) * W_ + w];
    }

    // Integration: per-type counts of spiking connected axons.
    unsigned cnt[G_];
#pragma unroll
    for (int g = 0; g < G_; ++g)
        cnt[g] = 0;
    const uint32_t *col = n.colbits + (size_t)c * W_ * N + j;
#pragma unroll
    for (int w = 0; w < W_; ++w) {
        const uint32_t cw = col[(size_t)w * N];
#pragma unroll
        for (int g = 0; g < G_; ++g)
            cnt[g] += __popc(cw & xt[g][w]);
    }
    const int32_t *wt = n.wts + (size_t)c * G_ * N + j;
    int in = 0;
    unsigned ev = 0;
#pragma unroll
    for (int g = 0; g < G_; ++g) {
        in += __mul24((int)cnt[g], wt[(size_t)g * N]);
        ev += cnt[g];
    }

    // Leak, threshold, reset.
    const size_t cj = (size_t)c * N + j;
    const size_t vi = ((size_t)c * n.S + s) * N + j;
    int32_t vnew;
    const bool fire = lif_update(n.V[vi], in, n.leak[cj], n.thr[cj], n.rst[cj], n.vmin, n.vmax, vnew);
    n.V[vi] = vnew;

    // Spike words (ballot), counters, output raster.
    const unsigned long long b = __ballot(fire);
    ev = wave_sum(ev);
    if (lane == 0) {
        unsigned em = 0, ro = 0, ou = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int nw = wave * 2 + h;
            const uint32_t wd = (uint32_t)(b >> (32 * h));
            const size_t m = (size_t)c * n.NW + nw;
            n.spk[((size_t)s * n.C + c) * n.NW + nw] = wd;
            const uint32_t om = wd & n.outmask[m];
            em += __popc(wd);
            ro += __popc(wd & n.coremask[m]);
            ou += __popc(om);
            const int ow = n.outword[m];
            if (ow >= 0)
                n.raster[((size_t)ta.r_row * n.S + s) * n.Wout + ow] = om;
        }
        red[wave][0] = em;
        red[wave][1] = ro;
        red[wave][2] = ou;
        red[wave][3] = ev;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long em = 0, ro = 0, ou = 0, e = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            em += red[w][0];
            ro += red[w][1];
            ou += red[w][2];
            e += red[w][3];
        }
        unsigned long long *cp = n.cnt + ((size_t)c * n.S + s) * CNT_N;
        cp[CNT_EMITTED] += em;
        cp[CNT_ROUTED] += ro;
        cp[CNT_DELIVERED] += delivered;
        cp[CNT_OUT] += ou;
        cp[CNT_EVENTS] += e;
    }
}

template <int W_>
static hipError_t launch_plain_w(const DevNet &n, const TickArgs &a, hipStream_t st)
{
    const dim3 grid(n.C, n.S), block(n.N);
    switch (n.G) {
    case 1: hipLaunchKernelGGL((k_integrate_plain<W_, 1>), grid, block, 0, st, n, a); break;
    case 2: hipLaunchKernelGGL((k_integrate_plain<W_, 2>), grid, block, 0, st, n, a); break;
    case 4: hipLaunchKernelGGL((k_integrate_plain<W_, 4>), grid, block, 0, st, n, a); break;
    case 8: hipLaunchKernelGGL((k_integrate_plain<W_, 8>), grid, block, 0, st, n, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_integrate_plain(const DevNet &n, const TickArgs &a, hipStream_t st)
{
    if (n.N < 64 || n.N > 512 || n.N % 64 != 0 || n.S > 65535)
        return hipErrorInvalidValue;
    switch (n.W) {
    case 2: return launch_plain_w<2>(n, a, st);
    case 4: return launch_plain_w<4>(n, a, st);
    case 8: return launch_plain_w<8>(n, a, st);
    case 16: return launch_plain_w<16>(n, a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ranc
