// kern_sparse.hip -- one tick of the event-driven path: delivery of the
// spikes scheduled for this tick, integration by scattering each spiking
// axon's weights to its connected neurons, leak/threshold/reset, and the
// scheduler write of this tick's spikes.
//
// Integration (GPU-RANC Sec. II) visits only spiking axons: for every axon a
// that spikes in a sample, every neuron n connected to it adds its weight for
// a's type. With spike rates of a few percent this is a few hundred additions
// per (core, sample) instead of the dense A x N contraction, and it needs
// neither the weight planes of the MFMA path nor the per-neuron crossbar
// columns of the plain path: only the core's crossbar rows (A x N bits), its
// axon-type masks and the neurons' G weights, all held on chip for the
// workgroup's whole chunk of samples.
//
// Scheduler and delivery are those of the MFMA path (same layouts): a
// sample-sliced spike history of the last Q = D + 1 ticks, gathered by the
// destination core for each of its axons at tick t - d, and the output raster
// as neuron-major history words. Bits within a 32-sample group follow the
// order sigma32 of kern_bits.h, so both paths read and write the same words.
//
// Mapping: one workgroup of 8 wavefronts per (core, chunk of samples), 64
// samples per tile; wave w handles samples w, w + 8, ..., w + 56 of the tile,
// one at a time, with lane l owning neurons l, l + 64, ... (N/64 per lane). A
// sample's axon words are wave-uniform, so the loop over its spiking axons
// (per axon type, so the type is static inside the loop) runs in scalar
// registers; per spiking axon each lane reads its part of the crossbar row
// from LDS and adds bit * weight for its neurons. The neurons' spike bits of
// the wave's samples are collected per lane and ORed across the eight waves
// in LDS, giving each neuron's 64-sample history word of the tile.
#include <type_traits>

#include "kern_bits.h"
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int SP_TS = 64;        // samples per tile
static constexpr int SP_SPW_MAX = 512;  // samples per workgroup (LDS counters)

template <int A_, int N_, int G_>
__global__ __launch_bounds__(512) void k_integrate_sparse(DevNet n, TickArgs ta, int spw)
{
    constexpr int W_ = A_ / 32;          // axon words
    constexpr int NW_ = N_ / 32;         // neuron words per crossbar row
    constexpr int NPL = N_ / 64;         // neurons per lane: lane + 64 j
    constexpr int APW = A_ / 64;         // 64-axon blocks of the gather
    constexpr int GPW = APW == 8 ? 2 : 1;  // 32-sample groups gathered per wave
    typedef typename std::conditional<GPW == 2, uint64_t, uint32_t>::type RawT;

    // crossbar rows, lane-friendly: xr[a][h][j] = row word h + 2j (neurons
    // 32h + 64j .. +31), so lane l reads its NPL words at (a, l / 32)
    __shared__ __attribute__((aligned(16))) uint32_t xr[A_ * NW_];
    __shared__ uint32_t tm[G_ * W_];                   // axon-type masks
    __shared__ uint16_t dg[A_];                        // connected neurons per axon
    __shared__ uint32_t x_lds[2][SP_TS][W_ + 1];        // delivered axon words per sample
    __shared__ unsigned long long hacc[N_];            // the tile's spike words per neuron
    // per sample of the chunk: [0] emitted | routed << 10 | out << 20,
    // [1] events | delivered << 18
    __shared__ unsigned s_cnt[2][SP_SPW_MAX];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int sig = sigma32(lane & 31);
    const int c = blockIdx.x % n.C;
    const int chunk = blockIdx.x / n.C;
    const int s_begin = chunk * spw;
    const int s_end = min(n.S, s_begin + spw);

    for (int i = threadIdx.x; i < A_ * NW_; i += blockDim.x) {
        const int a = i / NW_, w = i % NW_;
        xr[a * NW_ + (w & 1) * NPL + (w >> 1)] = n.xrow[((size_t)c * A_ + a) * NW_ + w];
    }
    for (int i = threadIdx.x; i < G_ * W_; i += blockDim.x)
        tm[i] = n.typemask[(size_t)c * G_ * W_ + i];
    for (int a = threadIdx.x; a < A_; a += blockDim.x) {
        unsigned d = 0;
        for (int w = 0; w < NW_; ++w)
            d += __popc(n.xrow[((size_t)c * A_ + a) * NW_ + w]);
        dg[a] = (uint16_t)d;
    }
    for (int i = threadIdx.x; i < N_; i += blockDim.x)
        hacc[i] = 0ull;
    for (int i = threadIdx.x; i < 2 * SP_SPW_MAX; i += blockDim.x)
        (&s_cnt[0][0])[i] = 0u;

    // neuron parameters of this lane
    int32_t wt[G_][NPL], lk[NPL], th[NPL], rs[NPL];
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
        const size_t cj = (size_t)c * N_ + lane + 64 * j;
        lk[j] = n.leak[cj];
        th[j] = n.thr[cj];
        rs[j] = n.rst[cj];
#pragma unroll
        for (int g = 0; g < G_; ++g)
            wt[g][j] = n.wts[((size_t)c * G_ + g) * N_ + lane + 64 * j];
    }
    const int32_t vmin = n.vmin, vmax = n.vmax;

    const int ci = n.in_index[c];
    const uint32_t *ext_c = (ta.ext_t != nullptr && ci >= 0) ? ta.ext_t + (size_t)ci * W_ : nullptr;
    const int q_now = tick_slot(n, ta.k), r_row = tick_row(n, ta.k);
    const size_t HG = (size_t)n.S64 / 64;
    const size_t CN = (size_t)n.C * N_;
    int32_t *vc = n.V + (size_t)c * n.S64 * N_ + lane;

    // ---- history gather (as on the MFMA path): wave w collects, for axon
    // block w % APW, group w / APW of each tile's history bits.
    const bool gatherer = wave < 2 * APW;
    const int axb = wave % APW;
    const int grp = GPW == 2 ? 0 : wave / APW;
    const int ga = axb * 64 + lane;
    uint32_t e_beg = 0, e_end = 0;
    if (gatherer) {
        e_beg = n.rtx_ptr[(size_t)c * A_ + ga];
        e_end = n.rtx_ptr[(size_t)c * A_ + ga + 1];
    }
    constexpr int FMAX = 4;
    const uint64_t *src_row[FMAX];
#pragma unroll
    for (int k = 0; k < FMAX; ++k) {
        src_row[k] = n.hist_zero;
        if (e_beg + k < e_end) {
            const uint32_t ent = n.rtx_ent[e_beg + k];
            int slot = q_now - (int)(ent & 15u) - 1;
            if (slot < 0)
                slot += n.Q;
            src_row[k] = n.hist + ((size_t)slot * CN + (ent >> 4)) * HG;
        }
    }
    const bool multi = __ballot(e_end - e_beg > 1) != 0;
    const bool long_lists = __ballot(e_end - e_beg > FMAX) != 0;
    auto raw_word = [&](const uint64_t *row, int tile) -> RawT {
        if constexpr (GPW == 2)
            return row[tile];
        else
            return reinterpret_cast<const uint32_t *>(row + tile)[grp];
    };
    auto load_mask = [&](int s0, RawT (&raw)[FMAX]) {
        const int tile = (s0 < s_end ? s0 : s_begin) / SP_TS;
        raw[0] = raw_word(src_row[0], tile);
        if (multi) {
#pragma unroll
            for (int k = 1; k < FMAX; ++k)
                raw[k] = raw_word(src_row[k], tile);
            for (uint32_t e = e_beg + FMAX; long_lists && e < e_end; ++e) {
                const uint32_t ent = n.rtx_ent[e];
                int slot = q_now - (int)(ent & 15u) - 1;
                if (slot < 0)
                    slot += n.Q;
                raw[1] |= raw_word(n.hist + ((size_t)slot * CN + (ent >> 4)) * HG, tile);
            }
        }
    };
    auto mask_of = [&](const RawT (&raw)[FMAX]) -> RawT {
        RawT m = raw[0];
        if (multi) {
#pragma unroll
            for (int k = 1; k < FMAX; ++k)
                m |= raw[k];
        }
        return m;
    };
    auto transpose_store = [&](RawT m, int buf) {
#pragma unroll
        for (int g = 0; g < GPW; ++g) {
            const uint32_t t = transpose32((uint32_t)(m >> (32 * g)), lane);
            x_lds[buf][32 * (GPW == 2 ? g : grp) + sig][2 * axb + h] = t;
        }
    };

    RawT mraw[FMAX] = {};
    if (gatherer) {
        load_mask(s_begin, mraw);
        transpose_store(mask_of(mraw), 0);
        load_mask(s_begin + SP_TS, mraw);
    }
    __syncthreads();

    int it = 0;
    for (int s0 = s_begin; s0 < s_end; s0 += SP_TS, ++it) {
        const int buf = it & 1;
        const int tile = s0 / SP_TS;
        uint64_t hw[NPL];
#pragma unroll
        for (int j = 0; j < NPL; ++j)
            hw[j] = 0ull;
        // potentials of the wave's first sample of the tile
        int32_t vnext[NPL];
        {
            const int s = min(s0 + wave, s_end - 1);
#pragma unroll
            for (int j = 0; j < NPL; ++j)
                vnext[j] = vc[(size_t)s * N_ + 64 * j];
        }
        for (int t = wave; t < SP_TS; t += 8) {
            const int s = s0 + t;
            if (s >= s_end)
                break;   // wave-uniform
            int32_t vcur[NPL];
#pragma unroll
            for (int j = 0; j < NPL; ++j)
                vcur[j] = vnext[j];
            if (t + 8 < SP_TS && s + 8 < s_end) {
#pragma unroll
                for (int j = 0; j < NPL; ++j)
                    vnext[j] = vc[(size_t)(s + 8) * N_ + 64 * j];
            }
            // the sample's axon words: delivered | external input
            uint32_t xw[W_];
            unsigned delivered = 0;
#pragma unroll
            for (int w = 0; w < W_; ++w) {
                const uint32_t xd = __builtin_amdgcn_readfirstlane(x_lds[buf][t][w]);
                delivered += __popc(xd);
                xw[w] = xd | (ext_c ? ext_c[(size_t)s * ta.ext_sstride + w] : 0u);
            }
            int32_t acc[NPL];
#pragma unroll
            for (int j = 0; j < NPL; ++j)
                acc[j] = lk[j];
            unsigned events = 0;
            const int lj = lane & 31;
#pragma unroll
            for (int g = 0; g < G_; ++g) {
#pragma unroll
                for (int w = 0; w < W_; ++w) {
                    uint32_t bits = xw[w] & tm[g * W_ + w];   // wave-uniform
                    // up to four spiking axons per round, their row reads in flight together
                    while (bits) {
                        int a[4];
                        bool v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            v[u] = bits != 0u;
                            a[u] = v[u] ? 32 * w + __builtin_ctz(bits) : 0;
                            bits &= bits - 1u;
                        }
                        uint32_t row[4][NPL];
                        unsigned d[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            d[u] = dg[a[u]];
#pragma unroll
                            for (int j = 0; j < NPL; ++j)
                                row[u][j] = xr[a[u] * NW_ + h * NPL + j];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (v[u]) {   // wave-uniform
                                events += d[u];
#pragma unroll
                                for (int j = 0; j < NPL; ++j)
                                    acc[j] += (int32_t)((row[u][j] >> lj) & 1u) * wt[g][j];
                            }
                        }
                    }
                }
            }
            // leak was the accumulator's start; threshold, reset
            unsigned emitted = 0, routed = 0, out = 0;
            const int pos = 32 * (t >> 5) + sigma32_inv(t & 31);
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                int32_t vn;
                const bool fire = lif_update(vcur[j], acc[j], 0, th[j], rs[j], vmin, vmax, vn);
                vc[(size_t)s * N_ + 64 * j] = vn;
                hw[j] |= fire ? (1ull << pos) : 0ull;
                const unsigned long long m = __ballot(fire);
                const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
                const size_t mw = (size_t)c * NW_ + 2 * j;
                emitted += __popc(lo) + __popc(hi);
                routed += __popc(lo & n.coremask[mw]) + __popc(hi & n.coremask[mw + 1]);
                out += __popc(lo & n.outmask[mw]) + __popc(hi & n.outmask[mw + 1]);
            }
            if (lane == 0) {
                s_cnt[0][s - s_begin] = emitted | (routed << 10) | (out << 20);
                s_cnt[1][s - s_begin] = events | (delivered << 18);
            }
        }
        // the tile's spike words of every neuron: OR of the eight waves' bits
#pragma unroll
        for (int j = 0; j < NPL; ++j)
            if (hw[j])
                atomicOr(&hacc[lane + 64 * j], hw[j]);
        __syncthreads();
        for (int i = threadIdx.x; i < N_; i += blockDim.x) {
            const uint64_t w = hacc[i];
            hacc[i] = 0ull;
            const size_t cj = (size_t)c * N_ + i;
            n.hist[((size_t)q_now * CN + cj) * HG + tile] = w;
            const int oi = n.outidx[cj];
            if (oi >= 0)
                reinterpret_cast<uint64_t *>(n.raster)[((size_t)r_row * n.Nout + oi) * HG + tile] = w;
        }
        if (s0 + SP_TS < s_end && gatherer) {
            transpose_store(mask_of(mraw), (it + 1) & 1);
            load_mask(s0 + 2 * SP_TS, mraw);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < s_end - s_begin; i += blockDim.x) {
        unsigned long long *cp = n.cnt + ((size_t)c * n.S + s_begin + i) * CNT_N;
        const unsigned sp = s_cnt[0][i], ev = s_cnt[1][i];
        cp[CNT_EMITTED] += sp & 1023u;
        cp[CNT_ROUTED] += (sp >> 10) & 1023u;
        cp[CNT_OUT] += sp >> 20;
        cp[CNT_DELIVERED] += ev >> 18;
        cp[CNT_EVENTS] += ev & ((1u << 18) - 1u);
    }
}

int sparse_max_samples_per_wg() { return SP_SPW_MAX; }

bool sparse_shape_supported(int A, int N, int G)
{
    const bool ok_a = A == 64 || A == 128 || A == 256 || A == 512;
    const bool ok_n = N == 64 || N == 128 || N == 256 || N == 512;
    const bool ok_g = G == 1 || G == 2 || G == 4 || G == 8;
    // per-lane weights take G * N / 64 VGPRs
    return ok_a && ok_n && ok_g && G * N <= 2048;
}

template <int A_, int N_>
static hipError_t launch_sparse_an(const DevNet &n, const TickArgs &a, int spw, hipStream_t st)
{
    const int chunks = (n.S + spw - 1) / spw;
    const dim3 grid(n.C * chunks), block(512);
    switch (n.G) {
    case 1: hipLaunchKernelGGL((k_integrate_sparse<A_, N_, 1>), grid, block, 0, st, n, a, spw); break;
    case 2: hipLaunchKernelGGL((k_integrate_sparse<A_, N_, 2>), grid, block, 0, st, n, a, spw); break;
    case 4:
        if constexpr (N_ <= 512)
            hipLaunchKernelGGL((k_integrate_sparse<A_, N_, 4>), grid, block, 0, st, n, a, spw);
        break;
    case 8:
        if constexpr (N_ <= 256)
            hipLaunchKernelGGL((k_integrate_sparse<A_, N_, 8>), grid, block, 0, st, n, a, spw);
        else
            return hipErrorInvalidValue;
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int A_>
static hipError_t launch_sparse_a(const DevNet &n, const TickArgs &a, int spw, hipStream_t st)
{
    switch (n.N) {
    case 64: return launch_sparse_an<A_, 64>(n, a, spw, st);
    case 128: return launch_sparse_an<A_, 128>(n, a, spw, st);
    case 256: return launch_sparse_an<A_, 256>(n, a, spw, st);
    case 512: return launch_sparse_an<A_, 512>(n, a, spw, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_integrate_sparse(const DevNet &n, const TickArgs &a, int samples_per_wg, hipStream_t st)
{
    if (!sparse_shape_supported(n.A, n.N, n.G) || samples_per_wg <= 0 || samples_per_wg % SP_TS ||
        samples_per_wg > SP_SPW_MAX || n.vlayout != VLAYOUT_SPARSE || n.S64 % SP_TS || n.S > n.S64)
        return hipErrorInvalidValue;
    switch (n.A) {
    case 64: return launch_sparse_a<64>(n, a, samples_per_wg, st);
    case 128: return launch_sparse_a<128>(n, a, samples_per_wg, st);
    case 256: return launch_sparse_a<256>(n, a, samples_per_wg, st);
    case 512: return launch_sparse_a<512>(n, a, samples_per_wg, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ranc
