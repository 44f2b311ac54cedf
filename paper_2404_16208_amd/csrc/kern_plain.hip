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

// One (core, sample) on a workgroup of at least N threads (threads past N
// take part in the ballots and the barrier only).
template <int W_, int G_>
__device__ __forceinline__ void integrate_plain_unit(const DevNet &n, const TickArgs &ta, int c, int s)
{
    const int N = n.N;
    const int jt = threadIdx.x;
    const bool live = jt < N;
    const int j = live ? jt : N - 1;   // idle threads mirror the last neuron's loads
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // Axon spikes of this tick: scheduler slot t%Q OR the external input.
    const uint32_t *slot = n.ring + (((size_t)tick_slot(n, ta.k) * n.S + s) * n.C + c) * W_;
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
    int32_t fl = n.vmin;
    bool lin = false;
    if (n.model_ext) {   // uniform
        fl = n.floor[cj];
        lin = (n.linmask[cj >> 5] >> (j & 31)) & 1u;
    }
    const bool fire = lif_update(n.V[vi], in, n.leak[cj], n.thr[cj], n.rst[cj], n.vmin, n.vmax, fl, lin, vnew) && live;
    if (live)
        n.V[vi] = vnew;
    if (!live)
        ev = 0;

    // Spike words (ballot), counters, output raster. Each wavefront adds its
    // 64 neurons' counts to its own counter row (no reduction across waves);
    // wave 0 also counts the core's delivered spikes.
    const unsigned long long b = __ballot(fire);
    ev = wave_sum(ev);
    if (lane == 0 && wave < (N >> 6)) {
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
                n.raster[((size_t)tick_row(n, ta.k) * n.S + s) * n.Wout + ow] = om;
        }
        // the core's delivered spikes are counted once, in row 0
        store_counts(n, ta.k, (size_t)c * (N >> 6) + wave, s, pack_counts(em, ro, ou, wave == 0 ? delivered : 0u, ev));
    }
}

template <int W_, int G_>
__global__ __launch_bounds__(512) void k_integrate_plain(DevNet n, TickArgs ta)
{
    integrate_plain_unit<W_, G_>(n, ta, blockIdx.x, blockIdx.y);
}

// The same tick for one 64-neuron block of one (core, sample) on a single
// wavefront (the batched launch, where networks of every N share one launch
// shape); the block's counts go to its own counter row.
template <int W_, int G_>
__device__ __forceinline__ void integrate_plain_wave(const DevNet &n, const TickArgs &ta, int c, int s, int nb)
{
    const int N = n.N;
    const int lane = threadIdx.x & 63;
    const uint32_t *slot = n.ring + (((size_t)tick_slot(n, ta.k) * n.S + s) * n.C + c) * W_;
    const int ci = n.in_index[c];
    const uint32_t *ext = (ta.ext_t != nullptr && ci >= 0)
                              ? ta.ext_t + (size_t)s * ta.ext_sstride + (size_t)ci * W_
                              : nullptr;
    const uint32_t *tmask = n.typemask + (size_t)c * G_ * W_;
    const int j = nb * 64 + lane;
    unsigned cnt[G_];
#pragma unroll
    for (int g = 0; g < G_; ++g)
        cnt[g] = 0;
    unsigned delivered = 0;
    const uint32_t *col = n.colbits + (size_t)c * W_ * N + j;
    // axon words and type masks are wave-uniform (scalar loads)
#pragma unroll 2
    for (int w = 0; w < W_; ++w) {
        const uint32_t r = slot[w];
        delivered += __popc(r);
        const uint32_t cw = col[(size_t)w * N] & (r | (ext ? ext[w] : 0u));
#pragma unroll
        for (int g = 0; g < G_; ++g)
            cnt[g] += __popc(cw & tmask[g * W_ + w]);
    }
    const int32_t *wt = n.wts + (size_t)c * G_ * N + j;
    int in = 0;
    unsigned e = 0;
#pragma unroll
    for (int g = 0; g < G_; ++g) {
        in += __mul24((int)cnt[g], wt[(size_t)g * N]);
        e += cnt[g];
    }
    const size_t cj = (size_t)c * N + j;
    const size_t vi = ((size_t)c * n.S + s) * N + j;
    int32_t vnew;
    int32_t fl = n.vmin;
    bool lin = false;
    if (n.model_ext) {   // uniform
        fl = n.floor[cj];
        lin = (n.linmask[cj >> 5] >> (j & 31)) & 1u;
    }
    const bool fire = lif_update(n.V[vi], in, n.leak[cj], n.thr[cj], n.rst[cj], n.vmin, n.vmax, fl, lin, vnew);
    n.V[vi] = vnew;
    const unsigned long long b = __ballot(fire);
    const unsigned ev = wave_sum(e);
    if (lane == 0) {
        unsigned em = 0, ro = 0, ou = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int nw = nb * 2 + h;
            const uint32_t wd = (uint32_t)(b >> (32 * h));
            const size_t m = (size_t)c * n.NW + nw;
            const uint32_t om = wd & n.outmask[m];
            em += __popc(wd);
            ro += __popc(wd & n.coremask[m]);
            ou += __popc(om);
            n.spk[((size_t)s * n.C + c) * n.NW + nw] = wd;
            const int ow = n.outword[m];
            if (ow >= 0)
                n.raster[((size_t)tick_row(n, ta.k) * n.S + s) * n.Wout + ow] = om;
        }
        store_counts(n, ta.k, (size_t)c * (N >> 6) + nb, s, pack_counts(em, ro, ou, nb == 0 ? delivered : 0u, ev));
    }
}

int plain_shape_code(int W, int G)
{
    const int wi = W == 2 ? 0 : W == 4 ? 1 : W == 8 ? 2 : 3;
    const int gi = G == 1 ? 0 : G == 2 ? 1 : G == 4 ? 2 : 3;
    return wi * 4 + gi;
}

// Several networks on the plain path, one tick, one launch: unit u is
// (64-neuron block, core, sample) of the network whose unit range holds u,
// on one wavefront.
__global__ __launch_bounds__(64) void k_integrate_plain_batch(const BatchEntry *__restrict__ tab, int num, int k)
{
    const int u = blockIdx.x;
    const BatchEntry &e = tab[batch_entry_of(tab, num, u, false)];
    const int local = u - e.unit_begin;
    const int nbs = e.n.N >> 6;
    const int nb = local % nbs, c = (local / nbs) % e.n.C, s = local / nbs / e.n.C;
    TickArgs ta;
    ta.k = k;
    ta.ext_t = e.ext_base ? e.ext_base + (size_t)k * e.tick_words : nullptr;
    ta.ext_sstride = e.ext_sstride;
    switch (e.code) {
#define RANC_PLAIN_CASE(WI, W, GI, G) \
    case WI * 4 + GI: integrate_plain_wave<W, G>(e.n, ta, c, s, nb); break;
        RANC_PLAIN_CASE(0, 2, 0, 1) RANC_PLAIN_CASE(0, 2, 1, 2) RANC_PLAIN_CASE(0, 2, 2, 4) RANC_PLAIN_CASE(0, 2, 3, 8)
        RANC_PLAIN_CASE(1, 4, 0, 1) RANC_PLAIN_CASE(1, 4, 1, 2) RANC_PLAIN_CASE(1, 4, 2, 4) RANC_PLAIN_CASE(1, 4, 3, 8)
        RANC_PLAIN_CASE(2, 8, 0, 1) RANC_PLAIN_CASE(2, 8, 1, 2) RANC_PLAIN_CASE(2, 8, 2, 4) RANC_PLAIN_CASE(2, 8, 3, 8)
        RANC_PLAIN_CASE(3, 16, 0, 1) RANC_PLAIN_CASE(3, 16, 1, 2) RANC_PLAIN_CASE(3, 16, 2, 4)
        RANC_PLAIN_CASE(3, 16, 3, 8)
#undef RANC_PLAIN_CASE
    default: break;
    }
}

hipError_t launch_integrate_plain_batch(const BatchEntry *tab, int num, int total, int k, hipStream_t st)
{
    if (num < 1 || total < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_integrate_plain_batch, dim3(total), dim3(64), 0, st, tab, num, k);
    return hipGetLastError();
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
