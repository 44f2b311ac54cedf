// kern_sparse.hip -- one tick of the event-driven path, as two kernels:
// delivery of the spikes scheduled for this tick, then integration by
// scattering each spiking axon's weights to its connected neurons,
// leak/threshold/reset, and the scheduler write of this tick's spikes.
//
// Scheduler (Sec. III-E): the spikes of the last Q = D + 1 ticks of every
// neuron are kept as a sample-sliced history, 64 samples per word (bit i =
// sample i of the word's 64-sample tile). A spike sent at tick t with offset d
// is read by its destination axon at tick t + d from the history slot of
// tick t, so every scheduler word has one writer (the firing neuron's
// workgroup) and no atomics are needed.
//
// k_deliver_event: one lane per destination axon and 64-sample tile ORs the
// history words of the axon's sources at t - d (the routing table keyed by
// destination axon) and, after a 32 x 32 bit transpose within each half
// wavefront, writes each sample's axon words of the tick to the delivery
// buffer [C][S64][A/32] (the scheduler row the tick reads). These are random
// 8-byte reads with few per lane; kept out of the integration kernel they run
// at the occupancy of a small kernel, and the integration kernel becomes a
// stream over the potentials.
//
// k_integrate_event (Sec. II): integration touches only the spiking axons'
// part of the crossbar. The core's connections are kept as compressed rows,
// one per (neuron slice, axon): the connected neurons of the slice, each
// entry with the neuron's weight for the axon's type already in it (16 bits:
// neuron within the slice in 7, signed 9-bit weight in 9). For every spiking
// axon of a sample the row's weights are added to the sample's input
// currents, so the work is the number of synaptic events, not A x N per
// sample. One workgroup of 8 wavefronts per (core, slice of <= 128 neurons,
// 64-sample tile); a lane is a sample:
//   0. loads that do not depend on each other are issued first and together:
//      the slice's row starts and rows (for LDS), the lane's delivered and
//      external input words;
//   1. scatter: each lane walks the spiking axons of its sample in its wave's
//      axon words and, flat over (axon, entry), adds every entry's weight to
//      its sample's current of that neuron in LDS (LDS atomic add: waves
//      share neurons); with at most EV_SMALL_S samples the wavefront instead
//      takes the samples in turn and its lanes take a row's entries, 64 at a
//      time (one instance of MNIST-12c: 11.8 instead of 47.0 us per tick);
//   2. update: the potentials of the wave's neurons are loaded (V is
//      neuron-major, [C][N][S64], so a wave's load of one neuron is 256
//      contiguous bytes), then per neuron leak, threshold and reset for all
//      64 samples at once (lif_update); the wave's ballot of the spikes is the
//      neuron's 64-sample history word; potentials are stored back.
// Loading the potentials only for the update keeps them out of the registers
// during the scatter: the kernel then fits 64 VGPRs, so four workgroups (32
// wavefronts, as many as the LDS holds) share a CU, and their potential
// loads and scatters overlap (6% faster on the 16384-core mesh than loading
// them in step 0 with three workgroups per CU). Barriers order LDS only
// (lds_barrier), so no wave waits for the potential loads of the others.
#include "kern_bits.h"
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int EV_TS = 64;          // samples per workgroup (one history word)
static constexpr int EV_NS = 128;         // neurons per slice, at most
static constexpr int EV_WAVES = 8;        // wavefronts per integration workgroup
static constexpr int EV_CSR_LDS = 3072;   // row entries staged in LDS (6 KiB)
static constexpr int DV_WAVES = 4;        // wavefronts per delivery workgroup
static constexpr int EV_SMALL_S = 8;      // at most this many samples: the small-batch scatter

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

// ---------------------------------------------------------------------------
// Delivery: wave (core c, tile, 64-axon block axb), lane = axon 64 axb + lane.

template <int A_>
__global__ __launch_bounds__(64 * DV_WAVES) void k_deliver_event(DevNet n, TickArgs ta)
{
    constexpr int W_ = A_ / 32;
    constexpr int APB = A_ / 64;   // 64-axon blocks per core
    constexpr int FMAX = 4;        // sources gathered without a loop
    const int HG = n.S64 / 64;
    const long long wv = (long long)blockIdx.x * DV_WAVES + (threadIdx.x >> 6);
    if (wv >= (long long)n.C * HG * APB)
        return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int axb = (int)(wv % APB);
    const long long ct = wv / APB;
    const int tile = (int)(ct % HG);
    const int c = (int)(ct / HG);
    const size_t CN = (size_t)n.C * n.N;
    const int q_now = tick_slot(n, ta.k);
    const size_t a = (size_t)c * A_ + axb * 64 + lane;
    const uint32_t b = n.rtx_ptr[a], e = n.rtx_ptr[a + 1];
    auto word_of = [&](uint32_t x) -> uint64_t {
        int slot = q_now - (int)(x & 15u) - 1;   // history slot of tick t - d
        if (slot < 0)
            slot += n.Q;
        return n.hist[((size_t)slot * CN + (x >> 4)) * HG + tile];
    };
    uint32_t ent[FMAX];
#pragma unroll
    for (int k = 0; k < FMAX; ++k)
        ent[k] = b + k < e ? n.rtx_ent[b + k] : 0xFFFFFFFFu;
    uint64_t m = 0;
#pragma unroll
    for (int k = 0; k < FMAX; ++k)
        if (ent[k] != 0xFFFFFFFFu)
            m |= word_of(ent[k]);
    for (uint32_t k = b + FMAX; k < e; ++k)
        m |= word_of(n.rtx_ent[k]);
    // lane (h, j) holds the 64-sample word of axon 64 axb + 32 h + j; after
    // the transpose of half g, lane (h, i) holds axon word 2 axb + h of
    // sample 32 g + i of the tile
    uint32_t *out = n.ring + ((size_t)c * n.S64 + (size_t)tile * 64) * W_;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const uint32_t t = transpose32((uint32_t)(m >> (32 * g)), lane);
        out[(size_t)(32 * g + (lane & 31)) * W_ + 2 * axb + (lane >> 5)] = t;
    }
}

// ---------------------------------------------------------------------------
// Integration.

// acc index of (sample s, neuron j of the slice): neuron-major, so the
// scatter's lanes (one sample each) always hit the bank of their own sample,
// whatever neurons they add to, and the update's read of one neuron for the
// wave's 64 samples is 256 contiguous bytes.
__device__ inline int acc_index(int s, int j) { return j * EV_TS + s; }

// Scatter of one axon word of this lane's sample: a flat loop over
// (spiking axon, row entry), so lanes with short rows move on to their next
// axon instead of idling until the wave's longest row ends.
template <typename RowPtr>
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
        atomicAdd(&acc[acc_index(s, j)], w);
    }
}

// SMALL: a few samples (n.S <= EV_SMALL_S, one tile): with a lane per sample
// most lanes would idle and one lane would walk every row entry of its
// sample, so instead the wavefront takes the samples in turn and its 64 lanes
// take 64 entries of a spiking axon's row at a time.
template <int A_, int NS_, bool EXT, bool SMALL>
__global__ __launch_bounds__(64 * EV_WAVES) __attribute__((amdgpu_waves_per_eu(8)))
void k_integrate_event(DevNet n, TickArgs ta)
{
    constexpr int W_ = A_ / 32;                             // axon words
    constexpr int NPW = NS_ / EV_WAVES;                      // neurons per wave in the update
    constexpr int WPW = (W_ + EV_WAVES - 1) / EV_WAVES;      // axon words per wave in the scatter
    constexpr int NT = 64 * EV_WAVES;                        // threads
    constexpr int RPT = (A_ + 1 + NT - 1) / NT;              // row starts per thread
    constexpr int CPT = (EV_CSR_LDS / 8 + NT - 1) / NT;      // 16-byte row chunks per thread

    __shared__ __attribute__((aligned(16))) int32_t acc[EV_TS * NS_];
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

    // ---- 0. independent loads, in the order they are needed
    const uint32_t *rp_g = n.ecsr_ptr + ((size_t)c * n.slices + slice) * (A_ + 1);
    const uint32_t e_base = rp_g[0];
    const uint32_t e_count = rp_g[A_] - e_base;
    const uint32_t e_pad = (e_count + 7u) & ~7u;   // each slice's rows are padded to 8 entries
    const bool staged = e_pad <= (uint32_t)EV_CSR_LDS;   // uniform
    uint32_t rpv[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = threadIdx.x + r * NT;
        rpv[r] = i <= A_ ? rp_g[i] - e_base : 0u;
    }
    uint4 rv[CPT];
    const uint4 *src = reinterpret_cast<const uint4 *>(n.ecsr_ent + e_base);
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        const int i = threadIdx.x + r * NT;
        rv[r] = staged && i < (int)(e_pad / 8) ? src[i] : uint4{0u, 0u, 0u, 0u};
    }
    // delivered (scheduler row of the tick) and external input words of this
    // lane's sample for the wave's scatter words w = wave, wave + EV_WAVES, ...
    uint32_t xd[WPW], xe[WPW];
    const int ci = n.in_index[c];
    const uint32_t *dlv = n.ring + ((size_t)c * n.S64 + s) * W_;
    const uint32_t *ext = (ta.ext_t != nullptr && ci >= 0 && svalid)
                              ? ta.ext_t + (size_t)s * ta.ext_sstride + (size_t)ci * W_
                              : nullptr;
#pragma unroll
    for (int k = 0; k < WPW; ++k) {
        const int wi = wave + EV_WAVES * k;
        xd[k] = (svalid && wi < W_) ? dlv[wi] : 0u;
        xe[k] = (ext && wi < W_) ? ext[wi] : 0u;
    }
    // parameters of the wave's neurons, lane k holding neuron j0 + k (one
    // load each, broadcast per neuron in the update): the kernel stores
    // through other pointers, so per-neuron loads inside the update would be
    // vector loads waited for one neuron at a time
    const size_t cw = (size_t)c * n.N + j0;   // first neuron of the wave (a multiple of NPW)
    const size_t cl = cw + (lane < NPW ? lane : 0);
    const int32_t p_leak = n.leak[cl], p_thr = n.thr[cl], p_rst = n.rst[cl];
    int32_t p_fl = n.vmin;
    if constexpr (EXT)
        p_fl = n.floor[cl];
    // the wave's NPW neurons lie in one 32-neuron word of the masks, from bit cw % 32
    const uint32_t cm_w = n.coremask[cw >> 5] >> (cw & 31), om_w = n.outmask[cw >> 5] >> (cw & 31);
    const uint32_t lin_w = EXT ? n.linmask[cw >> 5] >> (cw & 31) : 0u;
    compiler_fence();

    for (int i = threadIdx.x; i < EV_TS * NS_ / 4; i += NT)
        reinterpret_cast<int4 *>(acc)[i] = int4{0, 0, 0, 0};
    if (threadIdx.x < 2 * EV_TS)
        (&s_cnt[0][0])[threadIdx.x] = 0u;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = threadIdx.x + r * NT;
        if (i <= A_)
            rp[i] = rpv[r];
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        const int i = threadIdx.x + r * NT;
        if (staged && i < (int)(e_pad / 8))
            reinterpret_cast<uint4 *>(rows)[i] = rv[r];
    }
    lds_barrier();

    // ---- 1. scatter: lane = sample; wave w takes axon words w, w + EV_WAVES, ...
    unsigned events = 0, delivered = 0;
#pragma unroll
    for (int k = 0; k < WPW; ++k) {
        const int wi = wave + EV_WAVES * k;
        if (wi >= W_)
            break;   // wave-uniform
        delivered += (unsigned)__popc(xd[k]);
        if constexpr (!SMALL) {
            const uint32_t bits = xd[k] | xe[k];
            if (staged)
                scatter_word(bits, wi, lane, rp, (const uint16_t *)rows, acc, events);
            else
                scatter_word(bits, wi, lane, rp, n.ecsr_ent + e_base, acc, events);
        }
    }
    if constexpr (SMALL) {
        auto walk = [&](auto rowsrc) {
            for (int ss = 0; ss < n.S; ++ss) {   // wave-uniform
#pragma unroll
                for (int k = 0; k < WPW; ++k) {
                    const int wi = wave + EV_WAVES * k;
                    if (wi >= W_)
                        break;   // wave-uniform
                    uint32_t bits = (uint32_t)__builtin_amdgcn_readlane((int)(xd[k] | xe[k]), ss);
                    while (bits) {
                        const int a = 32 * wi + __builtin_ctz(bits);
                        bits &= bits - 1u;
                        const uint32_t e0 = rp[a], e1 = rp[a + 1];
                        if (lane == ss)
                            events += e1 - e0;
                        for (uint32_t e = e0 + lane; e < e1; e += 64) {
                            const uint32_t ent = rowsrc[e];
                            atomicAdd(&acc[acc_index(ss, (int)(ent & 127u))], (int)(ent << 16) >> 23);
                        }
                    }
                }
            }
        };
        if (staged)
            walk((const uint16_t *)rows);
        else
            walk(n.ecsr_ent + e_base);
    }
    if (svalid && (events | delivered))
        atomicAdd(&s_cnt[1][lane], events | (slice == 0 ? delivered << 20 : 0u));   // delivered counted once per core
    lds_barrier();

    // ---- 2. update, one neuron of the wave at a time for all 64 samples
    int32_t vreg[NPW];
    const int32_t *vin = n.V + ((size_t)c * n.N + j0) * n.S64 + s;
    // (small batches: only the valid samples' potentials move; the padding
    // lanes of the tile are never read)
#pragma unroll
    for (int k = 0; k < NPW; ++k)
        vreg[k] = (!SMALL || svalid) ? __builtin_nontemporal_load(vin + (size_t)k * n.S64) : 0;
    uint32_t fm = 0;       // bit k: this lane's sample fired on neuron j0 + k
    uint64_t myword = 0;   // lane k < NPW: the history word of neuron j0 + k
    int32_t *vout = n.V + ((size_t)c * n.N + j0) * n.S64 + s;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
        const int jl = wave * NPW + k;                // within the slice
        const int32_t in = acc[acc_index(lane, jl)];
        const int32_t lk = __builtin_amdgcn_readlane(p_leak, k), th = __builtin_amdgcn_readlane(p_thr, k);
        const int32_t rs = __builtin_amdgcn_readlane(p_rst, k);
        int32_t vn;
        bool fire;
        if constexpr (EXT) {
            const int32_t fl = __builtin_amdgcn_readlane(p_fl, k);
            fire = lif_update(vreg[k], in, lk, th, rs, n.vmin, n.vmax, fl, (lin_w >> k) & 1u, vn);
        } else {
            // 32-bit potentials, absolute reset, no floor: the saturating add
            // is the whole clamp (the same arithmetic as lif_update)
            const int32_t u = __builtin_elementwise_add_sat(vreg[k], in + lk);
            fire = u >= th;
            vn = fire ? rs : u;
        }
        fire = fire && svalid;
        if (!SMALL || svalid)
            __builtin_nontemporal_store(vn, vout + (size_t)k * n.S64);
        const uint64_t word = __ballot(fire);
        myword = lane == k ? word : myword;
        fm |= (uint32_t)fire << k;
    }
    const unsigned em = (unsigned)__popc(fm), ro = (unsigned)__popc(fm & cm_w), ou = (unsigned)__popc(fm & om_w);
    if (lane < NPW) {
        const size_t g = (size_t)c * n.N + j0 + lane;
        n.hist[((size_t)q_now * CN + g) * HG + tile] = myword;
        const int oi = n.outidx[g];
        if (oi >= 0)
            reinterpret_cast<uint64_t *>(n.raster)[((size_t)r_row * n.Nout + oi) * HG + tile] = myword;
    }
    if (svalid && (em | ro | ou))
        atomicAdd(&s_cnt[0][lane], em | (ro << 10) | (ou << 20));
    lds_barrier();
    if (wave == 0 && svalid) {
        const unsigned a0 = s_cnt[0][lane], a1 = s_cnt[1][lane];
        n.cring[((size_t)r_row * n.C * n.cnt_rows + (size_t)c * n.cnt_rows + slice) * n.S + s] =
            pack_counts(a0 & 1023u, (a0 >> 10) & 1023u, a0 >> 20, a1 >> 20, a1 & 0xFFFFFu);
    }
}

template <int A_, int NS_>
static void launch_event_k(const DevNet &n, const TickArgs &a, hipStream_t st)
{
    const long long dv_waves = (long long)n.C * (n.S64 / 64) * (A_ / 64);
    hipLaunchKernelGGL((k_deliver_event<A_>), dim3((unsigned)((dv_waves + DV_WAVES - 1) / DV_WAVES)),
                       dim3(64 * DV_WAVES), 0, st, n, a);
    const dim3 grid(n.C * n.slices * (n.S64 / EV_TS)), block(64 * EV_WAVES);
    const bool small = n.S <= EV_SMALL_S;
    if (n.model_ext && small)
        hipLaunchKernelGGL((k_integrate_event<A_, NS_, true, true>), grid, block, 0, st, n, a);
    else if (n.model_ext)
        hipLaunchKernelGGL((k_integrate_event<A_, NS_, true, false>), grid, block, 0, st, n, a);
    else if (small)
        hipLaunchKernelGGL((k_integrate_event<A_, NS_, false, true>), grid, block, 0, st, n, a);
    else
        hipLaunchKernelGGL((k_integrate_event<A_, NS_, false, false>), grid, block, 0, st, n, a);
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
        n.S64 % EV_TS || n.S > n.S64 || n.slices != n.N / sparse_slice_width(n.N) || n.cnt_rows != n.slices ||
        !n.ring)
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
