// kern_sparse.hip -- one tick of the event-driven path: delivery of the
// spikes scheduled for this tick, integration by scattering each spiking
// axon's weights to its connected neurons, leak/threshold/reset, and the
// scheduler write of this tick's spikes.
//
// Integration (GPU-RANC Sec. II) touches only the spiking axons' part of the
// crossbar. The core's connections are kept as compressed rows, one per
// (neuron slice, axon): the connected neurons of the slice, each entry with
// the neuron's weight for the axon's type already in it (16 bits: neuron
// within the slice in 7, signed 9-bit weight in 9). For every spiking axon
// of a sample the row's weights are added to the sample's input currents,
// so the work is the number of synaptic events, not A x N per sample.
//
// Mapping: one workgroup of 4 wavefronts per (core, slice of <= 128 neurons,
// tile of 64 samples); a lane is a sample. Phases:
//   0. every lane starts loading the potentials of its wave's neurons for
//      its sample (V is neuron-major, [C][N][S64], so a wave's load of one
//      neuron is 256 contiguous bytes); they are in flight during 1 and 2;
//      the slice's rows are staged in LDS;
//   1. delivery: for each axon, the OR of its sources' history words at
//      t - d (the scheduler rows of Sec. III-E, kept as the last Q = D + 1
//      ticks of every neuron's spikes, 64 samples per word, bit i = sample
//      i of the tile); the per-axon sample words are bit-transposed into
//      per-sample axon words;
//   2. scatter: each lane walks the spiking axons of its sample in its
//      wave's axon words and, flat over (axon, entry), adds every entry's
//      weight to its sample's current of that neuron in LDS (LDS atomic
//      add: waves share neurons);
//   3. update: per neuron of the wave, leak, threshold and reset for all 64
//      samples at once (lif_update); the wave's ballot of the spikes is the
//      neuron's 64-sample history word; potentials are stored back.
// Every scheduler word has one writer (the workgroup of the neuron's slice
// and tile) and no global atomics are used.
#include "kern_bits.h"
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int EV_TS = 64;          // samples per workgroup (one history word)
static constexpr int EV_NS = 128;         // neurons per slice, at most
static constexpr int EV_WAVES = 4;        // wavefronts per workgroup
static constexpr int EV_CSR_LDS = 4096;   // row entries staged in LDS (8 KiB)

int sparse_max_samples_per_wg() { return EV_TS; }
int sparse_slice_width(int N) { return N < EV_NS ? N : EV_NS; }
int sparse_row_align() { return 8; }

bool sparse_shape_supported(int A, int N, int G)
{
    const bool ok_a = A == 64 || A == 128 || A == 256 || A == 512;
    const bool ok_n = N == 64 || N == 128 || N == 256 || N == 512;
    const bool ok_g = G == 1 || G == 2 || G == 4 || G == 8;
    return ok_a && ok_n && ok_g;
}

// acc index of (sample s, neuron j of the slice): the neuron index is XORed
// with the sample's low five bits, so the 32 samples a half-wave reads for
// one neuron fall in 32 different banks.
template <int NS_> __device__ inline int acc_index(int s, int j) { return s * NS_ + (j ^ (s & 31)); }

// Scatter of one axon word of this lane's sample: a flat loop over
// (spiking axon, row entry), so lanes with short rows move on to their next
// axon instead of idling until the wave's longest row ends.
template <int NS_, typename RowPtr>
__device__ __forceinline__ void scatter_word(uint32_t bits, int word, int s, const uint32_t *rp, RowPtr rows,
                                             int32_t *acc, unsigned &events)
{
    uint32_t e = 0, ee = 0;
    for (;;) {
        if (e >= ee) {
            if (!bits)
                break;
            const int a = 32 * word + __builtin_ctz(bits);
            bits &= bits - 1u;
            e = rp[a];
            ee = rp[a + 1];
            events += ee - e;
            continue;
        }
        const uint32_t ent = rows[e++];
        const int j = (int)(ent & 127u);
        const int w = (int)(ent << 16) >> 23;   // bits 7..15, sign-extended
        atomicAdd(&acc[acc_index<NS_>(s, j)], w);
    }
}

template <int A_, int NS_, bool EXT>
__global__ __launch_bounds__(64 * EV_WAVES) void k_integrate_event(DevNet n, TickArgs ta)
{
    constexpr int W_ = A_ / 32;                             // axon words
    constexpr int NPW = NS_ / EV_WAVES;                      // neurons per wave in the update
    constexpr int WPW = (W_ + EV_WAVES - 1) / EV_WAVES;      // axon words per wave in the scatter
    constexpr int APW = A_ / 64;                             // 64-axon blocks of the gather
    constexpr int BPW = (APW + EV_WAVES - 1) / EV_WAVES;     // gather blocks per wave
    constexpr int FMAX = 4;                                  // sources gathered without a loop

    __shared__ __attribute__((aligned(16))) int32_t acc[EV_TS * NS_];
    __shared__ uint32_t xw[EV_TS][W_ + 1];                   // delivered axon words per sample
    __shared__ uint32_t rp[A_ + 1];                          // row starts, relative to the slice's first entry
    __shared__ __attribute__((aligned(16))) uint16_t rows[EV_CSR_LDS];
    // per sample: [0] emitted | routed << 10 | out << 20, [1] events | delivered << 20
    __shared__ unsigned s_cnt[2][EV_TS];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tiles = n.S64 / EV_TS;
    int c, v;   // XCD-grouped (core_unit_of)
    core_unit_of(blockIdx.x, n.C, n.slices * tiles, c, v);
    const int slice = v % n.slices;
    const int tile = v / n.slices;
    const int s = tile * EV_TS + lane;   // this lane's sample
    const bool svalid = s < n.S;
    const size_t CN = (size_t)n.C * n.N;
    const size_t HG = (size_t)n.S64 / 64;
    const int q_now = tick_slot(n, ta.k), r_row = tick_row(n, ta.k);
    const int j0 = slice * NS_ + wave * NPW;   // first neuron (within the core) of this wave's update

    // ---- 0. loads that start the chains: gather table heads, the slice's
    // rows, then the potentials of this wave's neurons (used in phase 3)
    uint32_t g_beg[BPW], g_end[BPW];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int axb = wave + EV_WAVES * b;
        g_beg[b] = g_end[b] = 0u;
        if (axb < APW) {
            const size_t a = (size_t)c * A_ + axb * 64 + lane;
            g_beg[b] = n.rtx_ptr[a];
            g_end[b] = n.rtx_ptr[a + 1];
        }
    }
    const uint32_t *rp_g = n.ecsr_ptr + ((size_t)c * n.slices + slice) * (A_ + 1);
    const uint32_t e_base = rp_g[0];
    const uint32_t e_count = rp_g[A_] - e_base;
    const uint32_t e_pad = (e_count + 7u) & ~7u;   // each slice's rows are padded to 8 entries
    const bool staged = e_pad <= (uint32_t)EV_CSR_LDS;   // uniform
    for (int i = threadIdx.x; i <= A_; i += 64 * EV_WAVES)
        rp[i] = rp_g[i] - e_base;
    if (staged) {
        const uint4 *src = reinterpret_cast<const uint4 *>(n.ecsr_ent + e_base);
        for (int i = threadIdx.x; i < (int)(e_pad / 8); i += 64 * EV_WAVES)
            reinterpret_cast<uint4 *>(rows)[i] = src[i];
    }
    int32_t vreg[NPW];
    const int32_t *vin = n.V + ((size_t)c * n.N + j0) * n.S64 + s;
#pragma unroll
    for (int k = 0; k < NPW; ++k)
        vreg[k] = __builtin_nontemporal_load(vin + (size_t)k * n.S64);
    compiler_fence();

    // external input words of this lane's sample for the wave's scatter words
    uint32_t xe[WPW];
    const int ci = n.in_index[c];
    const uint32_t *ext = (ta.ext_t != nullptr && ci >= 0 && svalid)
                              ? ta.ext_t + (size_t)s * ta.ext_sstride + (size_t)ci * W_
                              : nullptr;
#pragma unroll
    for (int k = 0; k < WPW; ++k) {
        const int wi = wave + EV_WAVES * k;
        xe[k] = (ext && wi < W_) ? ext[wi] : 0u;
    }

    for (int i = threadIdx.x; i < EV_TS * NS_ / 4; i += 64 * EV_WAVES)
        reinterpret_cast<int4 *>(acc)[i] = int4{0, 0, 0, 0};
    if (threadIdx.x < 2 * EV_TS)
        (&s_cnt[0][0])[threadIdx.x] = 0u;

    // ---- 1. delivery: lane = axon 64 axb + lane; its sources' history words
    // at t - d (up to FMAX of them as independent loads, the rest in a loop)
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int axb = wave + EV_WAVES * b;
        if (axb >= APW)
            break;   // wave-uniform
        auto row_of = [&](uint32_t e) -> const uint64_t * {
            int slot = q_now - (int)(e & 15u) - 1;
            if (slot < 0)
                slot += n.Q;
            return n.hist + ((size_t)slot * CN + (e >> 4)) * HG + tile;
        };
        uint32_t ent[FMAX];
#pragma unroll
        for (int k = 0; k < FMAX; ++k)
            ent[k] = g_beg[b] + k < g_end[b] ? n.rtx_ent[g_beg[b] + k] : 0xFFFFFFFFu;
        uint64_t m = 0;
#pragma unroll
        for (int k = 0; k < FMAX; ++k)
            if (ent[k] != 0xFFFFFFFFu)
                m |= *row_of(ent[k]);
        for (uint32_t e = g_beg[b] + FMAX; e < g_end[b]; ++e)
            m |= *row_of(n.rtx_ent[e]);
        // lane (h, j) holds axon 64 axb + 32 h + j; after the transpose lane
        // (h, i) holds axon word 2 axb + h of sample 32 g + i
#pragma unroll
        for (int g = 0; g < 2; ++g)
            xw[32 * g + (lane & 31)][2 * axb + (lane >> 5)] = transpose32((uint32_t)(m >> (32 * g)), lane);
    }
    __syncthreads();

    // ---- 2. scatter: lane = sample; wave w takes axon words w, w + 4, ...
    unsigned events = 0, delivered = 0;
#pragma unroll
    for (int k = 0; k < WPW; ++k) {
        const int wi = wave + EV_WAVES * k;
        if (wi >= W_)
            break;   // wave-uniform
        const uint32_t xd = svalid ? xw[lane][wi] : 0u;
        delivered += (unsigned)__popc(xd);
        const uint32_t bits = xd | xe[k];
        if (staged)
            scatter_word<NS_>(bits, wi, lane, rp, (const uint16_t *)rows, acc, events);
        else
            scatter_word<NS_>(bits, wi, lane, rp, n.ecsr_ent + e_base, acc, events);
    }
    if (svalid && (events | delivered))
        atomicAdd(&s_cnt[1][lane], events | (slice == 0 ? delivered << 20 : 0u));   // delivered counted once per core
    __syncthreads();

    // ---- 3. update, one neuron of the wave at a time for all 64 samples
    unsigned em = 0, ro = 0, ou = 0;
    uint64_t myword = 0;   // lane k < NPW: the history word of neuron j0 + k
    int32_t *vout = n.V + ((size_t)c * n.N + j0) * n.S64 + s;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
        const int jl = wave * NPW + k;                // within the slice
        const size_t cj = (size_t)c * n.N + j0 + k;   // uniform
        const int32_t in = acc[acc_index<NS_>(lane, jl)];
        int32_t fl = n.vmin;
        bool lin = false;
        if constexpr (EXT) {
            fl = n.floor[cj];
            lin = (n.linmask[cj >> 5] >> (cj & 31)) & 1u;
        }
        int32_t vn;
        const bool fire = lif_update(vreg[k], in, n.leak[cj], n.thr[cj], n.rst[cj], n.vmin, n.vmax, fl, lin, vn) &&
                          svalid;
        __builtin_nontemporal_store(vn, vout + (size_t)k * n.S64);
        const uint64_t word = __ballot(fire);
        myword = lane == k ? word : myword;
        const uint32_t bit = 1u << (cj & 31);
        em += fire;
        ro += fire && (n.coremask[cj >> 5] & bit);
        ou += fire && (n.outmask[cj >> 5] & bit);
    }
    if (lane < NPW) {
        const size_t g = (size_t)c * n.N + j0 + lane;
        n.hist[((size_t)q_now * CN + g) * HG + tile] = myword;
        const int oi = n.outidx[g];
        if (oi >= 0)
            reinterpret_cast<uint64_t *>(n.raster)[((size_t)r_row * n.Nout + oi) * HG + tile] = myword;
    }
    if (svalid && (em | ro | ou))
        atomicAdd(&s_cnt[0][lane], em | (ro << 10) | (ou << 20));
    __syncthreads();
    if (wave == 0 && svalid) {
        const unsigned a0 = s_cnt[0][lane], a1 = s_cnt[1][lane];
        n.cring[((size_t)r_row * n.C * n.cnt_rows + (size_t)c * n.cnt_rows + slice) * n.S + s] =
            pack_counts(a0 & 1023u, (a0 >> 10) & 1023u, a0 >> 20, a1 >> 20, a1 & 0xFFFFFu);
    }
}

template <int A_, int NS_>
static void launch_event_k(const DevNet &n, const TickArgs &a, hipStream_t st)
{
    const dim3 grid(n.C * n.slices * (n.S64 / EV_TS)), block(64 * EV_WAVES);
    if (n.model_ext)
        hipLaunchKernelGGL((k_integrate_event<A_, NS_, true>), grid, block, 0, st, n, a);
    else
        hipLaunchKernelGGL((k_integrate_event<A_, NS_, false>), grid, block, 0, st, n, a);
}

template <int A_>
static hipError_t launch_event_a(const DevNet &n, const TickArgs &a, hipStream_t st)
{
    switch (sparse_slice_width(n.N)) {
    case 64: launch_event_k<A_, 64>(n, a, st); break;
    case 128: launch_event_k<A_, 128>(n, a, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_integrate_sparse(const DevNet &n, const TickArgs &a, int samples_per_wg, hipStream_t st)
{
    if (!sparse_shape_supported(n.A, n.N, n.G) || samples_per_wg != EV_TS || n.vlayout != VLAYOUT_SPARSE ||
        n.S64 % EV_TS || n.S > n.S64 || n.slices != n.N / sparse_slice_width(n.N) || n.cnt_rows != n.slices)
        return hipErrorInvalidValue;
    switch (n.A) {
    case 64: return launch_event_a<64>(n, a, st);
    case 128: return launch_event_a<128>(n, a, st);
    case 256: return launch_event_a<256>(n, a, st);
    case 512: return launch_event_a<512>(n, a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ranc
