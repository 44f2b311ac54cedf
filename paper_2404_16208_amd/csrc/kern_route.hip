// kern_route.hip -- router + scheduler write of one tick, and state reset.
//
// GPU-RANC Sec. III-D writes each spike's bit straight into the destination
// core's scheduler SRAM at the packet's tick offset. Here that write is done
// from the destination side instead, so that no two lanes ever write the same
// word and no atomics are needed: the routing table is inverted at load time
// into one list per destination axon word (core, w) of the source neurons that
// send there, with their delays. The lane that owns (core, w) for a sample
// gathers the spike bits of those sources into a 32-bit word per delay d and
// ORs each non-zero word into scheduler slot (t + d) % Q, which only it
// writes. Arrivals at the same (core, axon, tick) therefore merge into one bit
// (the scheduler SRAM holds booleans, Sec. III-E). The same lane clears slot
// t % Q, which this tick's integration has already read (the clear of the
// obsolete row that Sec. III-E does at the start of the next tick).
//
// Layout for the MI355X: the lists are stored wave-interleaved (entry k of the
// 64 words of a wavefront are 64 consecutive u32), so each table load is one
// coalesced 256-byte access, and each list is sorted by delay with a count per
// delay, so a lane gathers every delay's word into its own register. A block
// serves SB samples at a time with their spike bitmaps staged in LDS, so every
// table entry fetched from L2 is used SB times. When the bitmaps do not fit in
// LDS the gather reads them from memory.
#include <algorithm>

#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int ROUTE_THREADS = 256;
static constexpr size_t ROUTE_LDS_BYTES = 128 * 1024;

// One destination word (core, w) for SB samples: gather every delay's word in
// registers (the per-delay loop is unrolled, so accumulators are indexed
// statically), then OR all non-zero words into their scheduler slots together
// so their read-modify-writes overlap.
template <int SB, int DMAX, bool STAGE>
__device__ __forceinline__ void route_unit(const DevNet &n, int k, int bx, int by, int gx, uint32_t *sp)
{
    const int q_now = tick_slot(n, k);
    const int s_base = by * SB;
    const int nsb = min(SB, n.S - s_base);
    const size_t words = (size_t)n.C * n.NW;
    const uint32_t *spk = n.spk + (size_t)s_base * words;
    if (STAGE) {
        for (size_t i = threadIdx.x; i < (size_t)nsb * words; i += blockDim.x)
            sp[i] = spk[i];
        __syncthreads();
    }
    const uint32_t *bits = STAGE ? sp : spk;
    const int CW = n.C * n.W;
    const size_t slot_stride = (size_t)n.S * CW;
    uint32_t *ring_b = n.ring + (size_t)s_base * CW;
    for (int dw = bx * ROUTE_THREADS + threadIdx.x; dw < CW; dw += gx * ROUTE_THREADS) {
#pragma unroll
        for (int b = 0; b < SB; ++b)
            if (b < nsb)
                ring_b[(size_t)q_now * slot_stride + (size_t)b * CW + dw] = 0u;
        const uint16_t *dcnt = n.rt_dcnt + (size_t)dw * DMAX;
        uint32_t cnt[DMAX];
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
            cnt[d] = dcnt[d];
        const uint32_t *e = n.rt_ent + n.rt_goff[dw >> 6] + (dw & 63);
        uint32_t acc[DMAX][SB];
        uint32_t k0 = 0;
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
#pragma unroll
            for (int b = 0; b < SB; ++b)
                acc[d][b] = 0u;
            const uint32_t kn = k0 + cnt[d];
#pragma unroll 4
            for (uint32_t k = k0; k < kn; ++k) {
                const uint32_t ent = e[(size_t)k * 64];
                const uint32_t g = ent >> RT_SRC_SHIFT;
                const uint32_t pos = ent & 31u;
                const uint32_t wi = g >> 5, bi = g & 31u;
#pragma unroll
                for (int b = 0; b < SB; ++b)
                    if (b < nsb)
                        acc[d][b] |= ((bits[(size_t)b * words + wi] >> bi) & 1u) << pos;
            }
            k0 = kn;
        }
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
            if (d >= n.D)
                break;
            int q = q_now + d + 1;
            if (q >= n.Q)
                q -= n.Q;
            uint32_t *dst = ring_b + (size_t)q * slot_stride + dw;
#pragma unroll
            for (int b = 0; b < SB; ++b)
                if (b < nsb && acc[d][b])
                    dst[(size_t)b * CW] |= acc[d][b];
        }
    }
}

template <int SB, int DMAX, bool STAGE>
__global__ __launch_bounds__(ROUTE_THREADS) void k_route(DevNet n, int k)
{
    extern __shared__ uint32_t sp[];
    route_unit<SB, DMAX, STAGE>(n, k, blockIdx.x, blockIdx.y, gridDim.x, sp);
}

// The same tick for one sample (blockIdx.y) with K lanes per destination
// word: lane r of a word's group walks entries r, r + K, ... of each delay's
// list, and the group ORs its partial words together with lane shuffles, so
// the serial walk is K times shorter and K times more lanes are in flight
// (used when the samples alone cannot fill the GPU). Lane 0 of the group is
// still the only writer of the word's scheduler slots. The loop bound is
// uniform across the block, so every lane reaches every shuffle. The spike
// bitmap is read in place: with one sample per block, copying all of it
// into every block's LDS cost more than the gather reads it saved (one
// MNIST-512c-shaped instance: 12.8 us per plain tick staged, 9.4 direct).
template <int DMAX, int K>
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_split(DevNet n, int k)
{
    static_assert(K >= 2 && K <= 64 && (K & (K - 1)) == 0, "K divides a wavefront");
    const int q_now = tick_slot(n, k);
    const int s = blockIdx.y;
    const size_t words = (size_t)n.C * n.NW;
    const uint32_t *bits = n.spk + (size_t)s * words;
    const int CW = n.C * n.W;
    const size_t slot_stride = (size_t)n.S * CW;
    uint32_t *ring_s = n.ring + (size_t)s * CW;
    const int r = threadIdx.x & (K - 1);
    constexpr int WPB = ROUTE_THREADS / K;   // destination words per block and pass
    for (int dw0 = blockIdx.x * WPB; dw0 < CW; dw0 += gridDim.x * WPB) {
        const int dw = dw0 + threadIdx.x / K;
        const bool own = dw < CW;
        uint32_t acc[DMAX];
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
            acc[d] = 0u;
        if (own) {
            if (r == 0)
                ring_s[(size_t)q_now * slot_stride + dw] = 0u;
            const uint16_t *dcnt = n.rt_dcnt + (size_t)dw * DMAX;
            const uint32_t *e = n.rt_ent + n.rt_goff[dw >> 6] + (dw & 63);
            uint32_t k0 = 0;
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                const uint32_t kn = k0 + dcnt[d];
#pragma unroll 2
                for (uint32_t j = k0 + r; j < kn; j += K) {
                    const uint32_t ent = e[(size_t)j * 64];
                    const uint32_t g = ent >> RT_SRC_SHIFT;
                    acc[d] |= ((bits[g >> 5] >> (g & 31u)) & 1u) << (ent & 31u);
                }
                k0 = kn;
            }
        }
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
#pragma unroll
            for (int off = 1; off < K; off <<= 1)
                acc[d] |= (uint32_t)__shfl_xor((int)acc[d], off, 64);
        }
        if (own && r == 0) {
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                if (d >= n.D)
                    break;
                int q = q_now + d + 1;
                if (q >= n.Q)
                    q -= n.Q;
                if (acc[d])
                    ring_s[(size_t)q * slot_stride + dw] |= acc[d];
            }
        }
    }
}

// Lanes per destination word of the split router.
static constexpr int ROUTE_SPLIT_K = 8;

int route_split_lanes() { return ROUTE_SPLIT_K; }

int route_auto_lanes(const DevNet &n, const RouteCfg &cfg)
{
    const long groups = (n.S + cfg.samples_per_block - 1) / cfg.samples_per_block;
    return (long)cfg.blocks_per_group * groups < 256 ? ROUTE_SPLIT_K : 1;
}

template <int DMAX>
static hipError_t launch_route_split(const DevNet &n, int k, hipStream_t st)
{
    constexpr int WPB = ROUTE_THREADS / ROUTE_SPLIT_K;
    const dim3 grid((n.C * n.W + WPB - 1) / WPB, n.S);
    hipLaunchKernelGGL((k_route_split<DMAX, ROUTE_SPLIT_K>), grid, dim3(ROUTE_THREADS), 0, st, n, k);
    return hipGetLastError();
}

int route_dmax(int D) { return D <= 4 ? 4 : D <= 8 ? 8 : 16; }

// Router variants usable in a batch launch: (samples per block, delay
// registers) with SB * DMAX <= 32, staged or not.
static constexpr int ROUTE_VARIANTS[9][2] = {{1, 4}, {1, 8}, {1, 16}, {2, 4}, {2, 8}, {2, 16}, {4, 4}, {4, 8}, {8, 4}};

int route_shape_code(const RouteCfg &cfg, int max_delay)
{
    const int dmax = route_dmax(max_delay);
    for (int i = 0; i < 9; ++i)
        if (ROUTE_VARIANTS[i][0] == cfg.samples_per_block && ROUTE_VARIANTS[i][1] == dmax)
            return i * 2 + (cfg.stage ? 1 : 0);
    return -1;
}

// Several plain-path networks routed in one launch: unit u is block
// (x, y) of the network whose router unit range holds u.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_batch(const BatchEntry *__restrict__ tab, int num, int k)
{
    extern __shared__ uint32_t sp[];
    const int u = blockIdx.x;
    const BatchEntry &e = tab[batch_entry_of(tab, num, u, true)];
    const int local = u - e.route_begin;
    const int bx = local % e.route_split, by = local / e.route_split;
    switch (e.route_code) {
#define RANC_ROUTE_CASE(I, SB, D)                                                      \
    case 2 * I: route_unit<SB, D, false>(e.n, k, bx, by, e.route_split, sp); break; \
    case 2 * I + 1: route_unit<SB, D, true>(e.n, k, bx, by, e.route_split, sp); break;
        RANC_ROUTE_CASE(0, 1, 4) RANC_ROUTE_CASE(1, 1, 8) RANC_ROUTE_CASE(2, 1, 16) RANC_ROUTE_CASE(3, 2, 4)
        RANC_ROUTE_CASE(4, 2, 8) RANC_ROUTE_CASE(5, 2, 16) RANC_ROUTE_CASE(6, 4, 4) RANC_ROUTE_CASE(7, 4, 8)
        RANC_ROUTE_CASE(8, 8, 4)
#undef RANC_ROUTE_CASE
    default: break;
    }
}

hipError_t launch_route_batch(const BatchEntry *tab, int num, int total, int k, size_t lds_bytes, hipStream_t st)
{
    if (num < 1 || total < 1 || lds_bytes > ROUTE_LDS_BYTES)
        return hipErrorInvalidValue;
    if (lds_bytes > 64 * 1024) {
        static bool raised = false;
        if (!raised) {
            hipError_t e = hipFuncSetAttribute((const void *)k_route_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)ROUTE_LDS_BYTES);
            if (e != hipSuccess)
                return e;
            raised = true;
        }
    }
    hipLaunchKernelGGL(k_route_batch, dim3(total), dim3(ROUTE_THREADS), lds_bytes, st, tab, num, k);
    return hipGetLastError();
}

// End of a batch call: every network's tick moves forward, and the batch
// queue counters are cleared for the next call.
__global__ void k_advance_batch(const BatchEntry *tab, int num, int num_ticks, unsigned *queue)
{
    for (int i = threadIdx.x; i < num; i += blockDim.x) {
        int *t = tab[i].n.tick;
        t[0] = (t[0] + num_ticks) % tab[i].n.Q;
        t[1] = (t[1] + num_ticks) % tab[i].n.RT;
        const unsigned long long v = ((unsigned long long)(unsigned)t[3] << 32 | (unsigned)t[2]) + (unsigned)num_ticks;
        t[2] = (int)(unsigned)v;
        t[3] = (int)(unsigned)(v >> 32);
    }
    if (threadIdx.x == 0) {
        queue[0] = 0u;
        queue[1] = 0u;
    }
}

hipError_t launch_advance_batch(const BatchEntry *tab, int num, int num_ticks, unsigned *queue, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_batch, dim3(1), dim3(256), 0, st, tab, num, num_ticks, queue);
    return hipGetLastError();
}

RouteCfg route_default_cfg(const DevNet &n)
{
    RouteCfg c;
    const size_t bitmap = (size_t)n.C * n.NW * 4;
    const int dmax = route_dmax(n.D);
    int sb = 1;
    // two samples per block measured fastest on the 512-core net (1024 samples)
    while (sb < 8 && bitmap * (size_t)(sb * 2) <= 64 * 1024 && sb * 2 <= n.S && dmax * sb * 2 <= 16)
        sb *= 2;
    c.samples_per_block = sb;
    c.stage = bitmap * (size_t)sb <= 64 * 1024;
    const int groups = (n.S + sb - 1) / sb;
    const int CW = n.C * n.W;
    const int max_split = (CW + ROUTE_THREADS - 1) / ROUTE_THREADS;
    int split = (2048 + groups - 1) / groups;
    if (split > max_split)
        split = max_split;
    if (split < 1)
        split = 1;
    c.blocks_per_group = split;
    c.lanes = route_auto_lanes(n, c);
    return c;
}

template <int SB, int DMAX, bool STAGE>
static hipError_t launch_route_v(const DevNet &n, int k, const RouteCfg &cfg, hipStream_t st)
{
    const size_t lds = STAGE ? (size_t)n.C * n.NW * 4 * SB : 0;
    const dim3 grid(cfg.blocks_per_group, (n.S + SB - 1) / SB);
    if (lds > 64 * 1024) {
        static bool raised = false;
        if (!raised) {
            hipError_t e = hipFuncSetAttribute((const void *)k_route<SB, DMAX, STAGE>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)ROUTE_LDS_BYTES);
            if (e != hipSuccess)
                return e;
            raised = true;
        }
    }
    hipLaunchKernelGGL((k_route<SB, DMAX, STAGE>), grid, dim3(ROUTE_THREADS), lds, st, n, k);
    return hipGetLastError();
}

template <int SB, int DMAX>
static hipError_t launch_route_sd(const DevNet &n, int k, const RouteCfg &cfg, hipStream_t st)
{
    // more than 32 accumulators per lane would spill
    if constexpr (SB * DMAX <= 32)
        return cfg.stage ? launch_route_v<SB, DMAX, true>(n, k, cfg, st)
                         : launch_route_v<SB, DMAX, false>(n, k, cfg, st);
    else
        return hipErrorInvalidValue;
}

template <int SB>
static hipError_t launch_route_s(const DevNet &n, int k, const RouteCfg &cfg, hipStream_t st)
{
    switch (route_dmax(n.D)) {
    case 4: return launch_route_sd<SB, 4>(n, k, cfg, st);
    case 8: return launch_route_sd<SB, 8>(n, k, cfg, st);
    default: return launch_route_sd<SB, 16>(n, k, cfg, st);
    }
}

hipError_t launch_route(const DevNet &n, int k, const RouteCfg &cfg, hipStream_t st)
{
    if (cfg.lanes == ROUTE_SPLIT_K) {
        if (n.S > 65535)
            return hipErrorInvalidValue;   // one sample per grid row
        switch (route_dmax(n.D)) {
        case 4: return launch_route_split<4>(n, k, st);
        case 8: return launch_route_split<8>(n, k, st);
        default: return launch_route_split<16>(n, k, st);
        }
    }
    if (cfg.lanes != 1 || cfg.blocks_per_group < 1)
        return hipErrorInvalidValue;
    if (cfg.stage && (size_t)n.C * n.NW * 4 * cfg.samples_per_block > ROUTE_LDS_BYTES)
        return hipErrorInvalidValue;
    if ((n.S + cfg.samples_per_block - 1) / cfg.samples_per_block > 65535)
        return hipErrorInvalidValue;
    switch (cfg.samples_per_block) {
    case 1: return launch_route_s<1>(n, k, cfg, st);
    case 2: return launch_route_s<2>(n, k, cfg, st);
    case 4: return launch_route_s<4>(n, k, cfg, st);
    case 8: return launch_route_s<8>(n, k, cfg, st);
    default: return hipErrorInvalidValue;
    }
}

__global__ void k_reset_potentials(DevNet n)
{
    const bool brick = n.vlayout == VLAYOUT_BRICK;
    const size_t SV = n.vlayout == VLAYOUT_CSN ? (size_t)n.S : (size_t)n.S64;   // samples per core
    const size_t total = (size_t)n.C * SV * n.N;
    const int NB = n.N / 32;
    const size_t groups = (size_t)n.S64 / 32;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        size_t c, j;
        if (brick) {
            // [C][N/32][S64/32][4][64][4]: 1024 values per brick
            const size_t lane = (i >> 2) & 63;
            const size_t cnb = (i >> 10) / groups;   // c * NB + nb
            c = cnb / NB;
            j = (cnb % NB) * 32 + (lane & 31);
        } else if (n.vlayout == VLAYOUT_SPARSE) {
            // [C][N][S64]
            c = i / (SV * n.N);
            j = (i / SV) % n.N;
        } else {
            c = i / (SV * n.N);
            j = i % n.N;
        }
        n.V[i] = n.vinit[c * n.N + j];
    }
}

__global__ void k_fill_u32(uint32_t *p, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_reset_state(const DevNet &n, const LinkArgs &l, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_potentials, dim3(2048), dim3(256), 0, st, n);
    const bool hist = n.vlayout != VLAYOUT_CSN;
    const size_t ring_words = hist ? 0 : (size_t)n.Q * n.S * n.C * n.W;
    const size_t spk_words = hist ? 0 : (size_t)n.S * n.C * n.NW;
    const size_t hist_words = hist ? (size_t)n.Q * n.C * n.N * (n.S64 / 64) * 2 : 0;
    const size_t raster_words = hist ? (size_t)n.RT * n.Nout * (n.S64 / 64) * 2 : (size_t)n.RT * n.S * n.Wout;
    const size_t cnt_words = (size_t)n.C * n.cnt_rows * n.S * CNT_N * 2;
    if (ring_words)
        hipLaunchKernelGGL(k_fill_u32, dim3(2048), dim3(256), 0, st, n.ring, ring_words);
    if (spk_words)
        hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, n.spk, spk_words);
    if (hist_words)
        hipLaunchKernelGGL(k_fill_u32, dim3(2048), dim3(256), 0, st, (uint32_t *)n.hist, hist_words);
    if (raster_words)
        hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, n.raster, raster_words);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, (uint32_t *)n.cnt, cnt_words);
    if (l.d)
        hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, (uint32_t *)l.d, (size_t)4 * n.C * n.S64 * 2);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)n.tick, (size_t)4);
    return hipGetLastError();
}

// End of a call of num_ticks ticks: move the device tick forward.
__global__ void k_advance_tick(DevNet n, int num_ticks)
{
    if (threadIdx.x == 0) {
        n.tick[0] = (n.tick[0] + num_ticks) % n.Q;
        n.tick[1] = (n.tick[1] + num_ticks) % n.RT;
        const unsigned long long t =
            ((unsigned long long)(unsigned)n.tick[3] << 32 | (unsigned)n.tick[2]) + (unsigned)num_ticks;
        n.tick[2] = (int)(unsigned)t;
        n.tick[3] = (int)(unsigned)(t >> 32);
    }
}

// Add the packed per-tick counts of the call's num_ticks ticks (ring rows
// from the call's first raster row on) into the 64-bit totals. Runs before
// the tick advance, which moves that row.
__global__ void k_fold_counts(DevNet n, int num_ticks)
{
    const size_t R = (size_t)n.C * n.cnt_rows * n.S;   // counter rows x samples
    const int r0 = n.tick[1];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < R; i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long em = 0, ro = 0, ou = 0, de = 0, ev = 0;
        for (int k = 0; k < num_ticks; ++k) {
            const unsigned long long w = n.cring[(size_t)((r0 + k) % n.RT) * R + i];
            em += w & 1023u;
            ro += (w >> 10) & 1023u;
            ou += (w >> 20) & 1023u;
            de += (w >> 30) & 1023u;
            ev += w >> 40;
        }
        unsigned long long *cp = n.cnt + i * CNT_N;
        cp[CNT_EMITTED] += em;
        cp[CNT_ROUTED] += ro;
        cp[CNT_OUT] += ou;
        cp[CNT_DELIVERED] += de;
        cp[CNT_EVENTS] += ev;
    }
}

// The same fold with one wavefront per counter row (few rows, e.g. a single
// sample): lane l adds ticks l, l + 64, ..., and the wavefront sums the five
// totals with shuffles before lane 0 adds them in.
__global__ __launch_bounds__(256) void k_fold_counts_wave(DevNet n, int num_ticks)
{
    const size_t R = (size_t)n.C * n.cnt_rows * n.S;
    const int r0 = n.tick[1];
    const int lane = threadIdx.x & 63;
    const size_t i = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= R)
        return;   // whole wavefronts leave together
    unsigned long long em = 0, ro = 0, ou = 0, de = 0, ev = 0;
    for (int k = lane; k < num_ticks; k += 64) {
        const unsigned long long w = n.cring[(size_t)((r0 + k) % n.RT) * R + i];
        em += w & 1023u;
        ro += (w >> 10) & 1023u;
        ou += (w >> 20) & 1023u;
        de += (w >> 30) & 1023u;
        ev += w >> 40;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        em += __shfl_xor(em, off, 64);
        ro += __shfl_xor(ro, off, 64);
        ou += __shfl_xor(ou, off, 64);
        de += __shfl_xor(de, off, 64);
        ev += __shfl_xor(ev, off, 64);
    }
    if (lane == 0) {
        unsigned long long *cp = n.cnt + i * CNT_N;
        cp[CNT_EMITTED] += em;
        cp[CNT_ROUTED] += ro;
        cp[CNT_OUT] += ou;
        cp[CNT_DELIVERED] += de;
        cp[CNT_EVENTS] += ev;
    }
}

hipError_t launch_fold_counts(const DevNet &n, int num_ticks, hipStream_t st)
{
    if (num_ticks < 1 || num_ticks > n.RT)
        return hipErrorInvalidValue;
    const size_t R = (size_t)n.C * n.cnt_rows * n.S;
    if (R <= 16384 && num_ticks >= 8) {
        // fewer rows than a thread per row would spread over the GPU
        hipLaunchKernelGGL(k_fold_counts_wave, dim3((unsigned)((R + 3) / 4)), dim3(256), 0, st, n, num_ticks);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)std::min<size_t>((R + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fold_counts, dim3(blocks), dim3(256), 0, st, n, num_ticks);
    return hipGetLastError();
}

hipError_t launch_advance_tick(const DevNet &n, int num_ticks, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_tick, dim3(1), dim3(64), 0, st, n, num_ticks);
    return hipGetLastError();
}

}  // namespace ranc
