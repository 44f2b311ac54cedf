// kern_sparse.hip -- one tick of the event-driven path: delivery of the
// spikes scheduled for this tick, integration by scattering each spiking
// axon's weights to its connected neurons, leak/threshold/reset, and the
// scheduler write of this tick's spikes.
//
// Integration (GPU-RANC Sec. II) touches only the spiking axons' part of the
// crossbar: a neuron's input is the sum over axon types g of (number of
// spiking axons of type g connected to it) * its weight for g, and the count
// is a popcount of (the neuron's crossbar column word) AND (the sample's
// spiking axons of type g) per 32-axon word. Words with no spiking axon, and
// types with no spiking axon in a word, are skipped (wave-uniform tests), so
// the work follows the activity: with spike rates of a few percent most of
// the A/32 x G buckets are empty. It needs neither the weight planes of the
// MFMA path nor LDS tiles per sample: the core's crossbar columns, type masks
// and the neurons' G weights are loaded once per workgroup.
//
// Scheduler and delivery are those of the MFMA path (same layouts): a
// sample-sliced spike history of the last Q = D + 1 ticks, gathered by the
// destination core for each of its axons at tick t - d, and the output raster
// as neuron-major history words. Bits within a 32-sample group follow the
// order sigma32 of kern_bits.h, so both paths read and write the same words.
//
// Mapping: one workgroup per (core, chunk of samples), 64 samples per tile,
// of 4 wavefronts (8 when A = 512, whose history gather needs 8); wave w of
// the workgroup's nw waves handles samples w, w + nw, ... of the tile, one at
// a time, with lane l owning neurons l, l + 64, ... (N/64 per lane). Small
// workgroups keep several independent workgroups per compute unit: with few
// samples per core a workgroup is a short chain of dependent memory
// accesses, and the chains of different workgroups overlap. A sample's axon
// words are wave-uniform, so the bucket tests run on scalar
// registers; per non-empty word each lane reads its neurons' column words
// from LDS, per non-empty bucket it adds popcounts. The neurons' spike bits
// of the wave's samples are collected per lane and ORed across the
// workgroup's waves in LDS, giving each neuron's 64-sample history word of
// the tile.
#include <type_traits>

#include "kern_bits.h"
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int SP_TS = 64;        // samples per tile
static constexpr int SP_SPW_MAX = 512;  // samples per workgroup (LDS counters)

template <int A_> constexpr int sp_waves() { return A_ == 512 ? 8 : 4; }

// Four waves per SIMD where the per-lane weights, type counts and prefetched
// potentials fit in 128 VGPRs without spilling.
template <int A_, int N_, int G_>
__global__ __launch_bounds__(64 * sp_waves<A_>()) __attribute__((amdgpu_waves_per_eu(N_ <= 128 || (N_ == 256 && A_ == 256 && G_ <= 4) ? 4 : 2)))
void k_integrate_sparse(DevNet n, TickArgs ta, int spw)
{
    constexpr int NWV = sp_waves<A_>();  // wavefronts per workgroup
    constexpr int W_ = A_ / 32;          // axon words
    constexpr int NW_ = N_ / 32;         // neuron words per crossbar row
    constexpr int NPL = N_ / 64;         // neurons per lane: lane + 64 j
    constexpr int APW = A_ / 64;         // 64-axon blocks of the gather
    // 32-sample groups gathered per wave: both when the (block, group) pairs
    // outnumber the waves
    constexpr int GPW = 2 * APW > NWV ? 2 : 1;
    static_assert(APW * 2 / GPW <= NWV, "gather roles exceed the workgroup's waves");
    typedef typename std::conditional<GPW == 2, uint64_t, uint32_t>::type RawT;

    // crossbar columns: bit b of col[w][n] = crossbar(32w + b, n)
    __shared__ uint32_t col[W_][N_];
    __shared__ uint32_t tm[G_ * W_];                   // axon-type masks
    __shared__ uint32_t x_lds[2][SP_TS][W_ + 1];        // delivered axon words per sample
    __shared__ uint32_t xe_lds[2][SP_TS][W_ + 1];       // external input words per sample
    __shared__ unsigned long long hacc[N_];            // the tile's spike words per neuron
    // per sample of the chunk: [0] emitted | routed << 10 | out << 20,
    // [1] events | delivered << 19 (events <= 512 * 512 = 2^18)
    __shared__ unsigned s_cnt[2][SP_SPW_MAX];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int sig = sigma32(lane & 31);
    int c, chunk;   // XCD-grouped (core_unit_of)
    core_unit_of(blockIdx.x, n.C, (n.S + spw - 1) / spw, c, chunk);
    const int s_begin = chunk * spw;
    const int s_end = min(n.S, s_begin + spw);

    for (int i = threadIdx.x; i < W_ * N_; i += blockDim.x)
        (&col[0][0])[i] = n.colbits[(size_t)c * W_ * N_ + i];
    for (int i = threadIdx.x; i < G_ * W_; i += blockDim.x)
        tm[i] = n.typemask[(size_t)c * G_ * W_ + i];
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
    // block w % APW, group w / APW of each tile's history bits (both groups
    // with GPW = 2).
    const bool gatherer = wave < 2 * APW / GPW;
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

    // external input words of a tile into LDS (all threads, coalesced per sample)
    auto stage_ext = [&](int s0, int buf) {
        for (int i = threadIdx.x; i < SP_TS * W_; i += blockDim.x) {
            const int t = i / W_, w = i % W_;
            const int s = s0 + t;
            xe_lds[buf][t][w] = (ext_c && s < s_end) ? ext_c[(size_t)s * ta.ext_sstride + w] : 0u;
        }
    };

    RawT mraw[FMAX] = {};
    if (gatherer) {
        load_mask(s_begin, mraw);
        transpose_store(mask_of(mraw), 0);
        load_mask(s_begin + SP_TS, mraw);
    }
    stage_ext(s_begin, 0);
    __syncthreads();

    int it = 0;
    for (int s0 = s_begin; s0 < s_end; s0 += SP_TS, ++it) {
        const int buf = it & 1;
        const int tile = s0 / SP_TS;
        uint64_t hw[NPL];
#pragma unroll
        for (int j = 0; j < NPL; ++j)
            hw[j] = 0ull;
        // the potentials of PF of the wave's samples of the tile are loaded
        // together, ahead of their use
        constexpr int PF = NPL >= 4 ? 4 : 8;
        constexpr int SPW = SP_TS / NWV;   // samples per wave per tile
        for (int i0 = 0; i0 < SPW; i0 += PF) {
        int32_t vbuf[PF][NPL];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int s = min(s0 + wave + NWV * (i0 + i), s_end - 1);
#pragma unroll
            for (int j = 0; j < NPL; ++j)
                vbuf[i][j] = vc[(size_t)s * N_ + 64 * j];
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int t = wave + NWV * (i0 + i);
            const int s = s0 + t;
            if (s >= s_end)
                break;   // wave-uniform
            // the sample's axon words: delivered | external input
            uint32_t xw[W_];
            unsigned delivered = 0;
#pragma unroll
            for (int w = 0; w < W_; ++w) {
                const uint32_t xd = __builtin_amdgcn_readfirstlane(x_lds[buf][t][w]);
                delivered += __popc(xd);
                xw[w] = xd | __builtin_amdgcn_readfirstlane(xe_lds[buf][t][w]);
            }
            // per type, spiking connected axons of each of this lane's neurons
            unsigned cnt[G_][NPL];
#pragma unroll
            for (int g = 0; g < G_; ++g)
#pragma unroll
                for (int j = 0; j < NPL; ++j)
                    cnt[g][j] = 0u;
#pragma unroll
            for (int w = 0; w < W_; ++w) {
                if (!xw[w])
                    continue;   // wave-uniform
                uint32_t cw[NPL];
#pragma unroll
                for (int j = 0; j < NPL; ++j)
                    cw[j] = col[w][lane + 64 * j];
#pragma unroll
                for (int g = 0; g < G_; ++g) {
                    const uint32_t m = xw[w] & tm[g * W_ + w];   // wave-uniform
                    if (!m)
                        continue;
#pragma unroll
                    for (int j = 0; j < NPL; ++j)
                        cnt[g][j] += (unsigned)__popc(cw[j] & m);
                }
            }
            int32_t acc[NPL];
            unsigned ev = 0;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                acc[j] = lk[j];
#pragma unroll
                for (int g = 0; g < G_; ++g) {
                    acc[j] += __mul24((int)cnt[g][j], wt[g][j]);
                    ev += cnt[g][j];
                }
            }
            const unsigned events = wave_sum(ev);
            // leak was the accumulator's start; threshold, reset
            unsigned emitted = 0, routed = 0, out = 0;
            const int pos = 32 * (t >> 5) + sigma32_inv(t & 31);
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                int32_t vn;
                const bool fire = lif_update(vbuf[i][j], acc[j], 0, th[j], rs[j], vmin, vmax, vn);
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
                s_cnt[1][s - s_begin] = events | (delivered << 19);
            }
        }
        }
        // the tile's spike words of every neuron: OR of the waves' bits
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
        if (s0 + SP_TS < s_end) {
            if (gatherer) {
                transpose_store(mask_of(mraw), (it + 1) & 1);
                load_mask(s0 + 2 * SP_TS, mraw);
            }
            stage_ext(s0 + SP_TS, (it + 1) & 1);
        }
        __syncthreads();
    }
    unsigned long long *cw_out = n.cring + ((size_t)r_row * n.C + c) * n.S + s_begin;   // one counter row per core
    for (int i = threadIdx.x; i < s_end - s_begin; i += blockDim.x) {
        const unsigned sp = s_cnt[0][i], ev = s_cnt[1][i];
        cw_out[i] = pack_counts(sp & 1023u, (sp >> 10) & 1023u, sp >> 20, ev >> 19, ev & ((1u << 19) - 1u));
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
    const dim3 grid(n.C * chunks), block(64 * sp_waves<A_>());
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
