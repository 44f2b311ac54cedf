// kern_mfma.hip -- one tick of the batched path on int8 MFMA: delivery of the
// spikes scheduled for this tick, integration, leak/threshold/reset, and the
// scheduler write of this tick's spikes.
//
// Integration. With many samples, the integration of one core (GPU-RANC
// Sec. II: sum over spiking connected axons of the neuron's weight for the
// axon's type) is the dense product X[samples x A] * B[A x N] with X the 0/1
// axon spikes and B[a][n] = crossbar(a, n) * weight(n, type(a)). It runs on
// V_MFMA_I32_32X32X32_I8 with int32 accumulation, which is exact:
//   - weights of up to 8 bits are int8 as they are (one B plane);
//   - 9-bit weights w in [-256, 255] are split as w = 128*hi + lo with
//     hi = w >> 7 in [-2, 1] and lo = w & 127 in [0, 127]; the two planes
//     accumulate separately and combine as lo + 128*hi;
//   |sum| <= 512 * 256 < 2^31, so int32 never overflows. The lo accumulator
//   starts at the neuron's leak, so the products give I + leak directly.
//
// Scheduler. A spike fired at tick t by neuron g with destination
// (core, axon, delay d) must reach that axon at tick t + d (Sec. III-D/E;
// several spikes to one (core, axon, tick) merge into one bit). On this path
// the scheduler holds the last Q = D + 1 ticks of every neuron's spikes,
// sample-sliced (one u64 = 64 samples of one neuron), and delivery is done by
// the destination: at tick t the workgroup of a core ORs, for each of its
// axons, the history bits of its sources at tick t - d. Every scheduler word
// has exactly one writer (the firing neuron's wavefront, at tick t, slot
// t % Q) and no atomics are used.
//
// Mapping: one workgroup of 8 wavefronts per (core, neuron slice, chunk of
// samples), a slice being 128 or 256 of the core's neurons; wave w owns the
// 32 neurons of block w % (slice/32), whose B tiles stay in VGPRs for the
// whole chunk (A*planes/8 VGPRs per lane; with 512 axons and two planes the
// two wavefronts of a block hold one plane each, see integrate_mfma_unit).
// Samples go 64 at a time (two 32-sample sub-tiles) through a software
// pipeline:
//   - the potentials of tile i+1 travel from HBM straight into LDS
//     (global_load_lds) while tile i is processed; history bits of tile i+2
//     are loaded and those of tile i+1 transposed into LDS meanwhile;
//   - the axon spikes of tile i (delivered OR external input) are expanded,
//     one lane per sample, to an int8 [64 x A] tile in LDS, double-buffered
//     so one barrier per tile suffices; delivered spikes and synaptic events
//     (sum over spiking axons of their connected-neuron counts, by dot4) are
//     counted in the same pass;
//   - products, potential update, and the neuron's 32-sample spike word
//     (16 bits per lane, two lanes combined); a 32 x 32 bit transpose of the
//     wave's spike words gives each sample's spike word, whose popcounts are
//     the per-sample spike counters;
//   - the results of tile i (potentials, counter updates in LDS, and the
//     spike history and raster words, which collect in LDS and go out every
//     few tiles as runs of consecutive words per neuron) are written at the
//     top of iteration i+1, so the stores have a whole iteration to drain
//     before the next wait.
// Waves exchange data only through LDS, so barriers order LDS alone
// (lds_barrier); the single wait for vector memory per iteration is explicit.
//
// MFMA operand convention used for both A and B: in k-step k, lane l holds 16
// bytes for row/column l % 32 and axons 32k + 16*(l/32) + [0, 16). Result:
// lane l, element r is row 8*(r/4) + 4*(l/32) + r%4, column l % 32. Bit
// p = r + 16*(l/32) of a neuron's 32-sample spike word is therefore sample
// sigma(p) = 8*((p%16)/4) + 4*(p/16) + p%4 of the 32-sample group.
#include "kern_mfma_unit.h"

namespace ranc {

int mfma_max_samples_per_wg() { return MFMA_SPW_MAX; }

// ---------------------------------------------------------------------------
// Several networks (shapes may differ) advanced by one tick in one persistent
// launch: a grid of one workgroup per CU pulls units (network, workgroup of
// that network's tick grid) from a queue counter until every unit is done.
// Units are numbered network after network in the order of the batch table,
// which the host sorts by decreasing cost per unit, so the largest units go
// first. LDS is sized for the largest shape; each unit uses it through views
// of its own shape.

int mfma_shape_code(int A, int N, int two_planes)
{
    const int ai = A == 64 ? 0 : A == 128 ? 1 : A == 256 ? 2 : 3;
    return (ai * 2 + (N == 256 ? 1 : 0)) * 2 + (two_planes ? 1 : 0);
}

template <int A_, int N_, bool TWO>
__device__ __forceinline__ void batch_unit(const BatchEntry &e, const TickArgs &ta, int bid, int8_t *a_raw,
                                           v4i *v_raw, uint32_t *x_raw, unsigned (*s_cnt)[MFMA_SPW_MAX])
{
    typedef MfmaLds<A_, N_> L;
    // the plane-split exchange sits in the potential staging area past this
    // shape's eight VTiles (it holds eight VTiles of the widest shape)
    static_assert(!(TWO && A_ == 512) ||
                  8 * sizeof(typename L::VTile) + sizeof(typename L::Xch) <= 8 * sizeof(MfmaLds<512, 256>::VTile),
                  "exchange does not fit the staging area");
    // Units store each tile's history words at once (no LDS history buffer).
    // A buffer carved for the widest shape would not serve the others: the
    // buffer of a shape with 256 axons or fewer (HB = 8) is twice the widest
    // shape's (HB = 4), so those shapes would index past its end.
    constexpr bool kHistBuf = false;
    static_assert(!kHistBuf || sizeof(typename L::HBuf) <= sizeof(MfmaLds<512, 256>::HBuf),
                  "this shape's history buffer is larger than the widest shape's");
    integrate_mfma_unit<A_, N_, TWO, true, kHistBuf, false>(e.n, ta, e.spw, bid, reinterpret_cast<typename L::ATile *>(a_raw),
                                                  reinterpret_cast<typename L::VTile *>(v_raw),
                                                  reinterpret_cast<typename L::XTile *>(x_raw), nullptr,
                                                  reinterpret_cast<typename L::Xch *>(
                                                      reinterpret_cast<int8_t *>(v_raw) + 8 * sizeof(typename L::VTile)),
                                                  s_cnt);
}

__global__ __launch_bounds__(512) void k_integrate_mfma_batch(const BatchEntry *__restrict__ tab, int num, int total, int k,
                                                              unsigned *queue)
{
    typedef MfmaLds<512, 256> Lmax;
    __shared__ __attribute__((aligned(16))) int8_t a_raw[2 * sizeof(Lmax::ATile)];
    __shared__ __attribute__((aligned(16))) v4i v_raw[8 * sizeof(Lmax::VTile) / sizeof(v4i)];
    __shared__ uint32_t x_raw[2 * sizeof(Lmax::XTile) / 4];
    __shared__ unsigned s_cnt[2][MFMA_SPW_MAX];
    __shared__ int s_unit;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        queue[(k + 1) & 1] = 0u;   // the next tick's counter (no unit of this launch uses it)
    for (;;) {
        if (threadIdx.x == 0)
            s_unit = (int)atomicAdd(&queue[k & 1], 1u);
        __syncthreads();
        const int u = __builtin_amdgcn_readfirstlane(s_unit);
        __syncthreads();
        if (u >= total)
            break;
        const BatchEntry &e = tab[batch_entry_of(tab, num, u, false)];   // network of unit u
        TickArgs ta;
        ta.k = k;
        ta.ext_t = e.ext_base ? e.ext_base + (size_t)k * e.tick_words : nullptr;
        ta.ext_sstride = e.ext_sstride;
        const int bid = u - e.unit_begin;
        switch (e.code) {
        case 0: batch_unit<64, 128, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 1: batch_unit<64, 128, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 2: batch_unit<64, 256, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 3: batch_unit<64, 256, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 4: batch_unit<128, 128, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 5: batch_unit<128, 128, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 6: batch_unit<128, 256, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 7: batch_unit<128, 256, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 8: batch_unit<256, 128, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 9: batch_unit<256, 128, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 10: batch_unit<256, 256, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 11: batch_unit<256, 256, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 12: batch_unit<512, 128, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 13: batch_unit<512, 128, true>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        case 14: batch_unit<512, 256, false>(e, ta, bid, a_raw, v_raw, x_raw, s_cnt); break;
        default: break;
        }
        __syncthreads();
    }
}

hipError_t launch_integrate_mfma_batch(const BatchEntry *tab, int num, int total, int k, unsigned *queue,
                                       int workgroups, hipStream_t st)
{
    if (num < 1 || total < 1 || workgroups < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_integrate_mfma_batch, dim3(workgroups), dim3(512), 0, st, tab, num, total, k, queue);
    return hipGetLastError();
}

hipError_t launch_integrate_mfma_group(const MfmaGroupArgs &g, int total, int k, int code, int ext, int compact,
                                       hipStream_t st)
{
    static_assert(sizeof(MfmaGroupArgs) + sizeof(int) <= 4096, "kernel arguments exceed 4 KiB");
    if (g.num < 1 || g.num > MFMA_GROUP_MAX || total < 1)
        return hipErrorInvalidValue;
    return compact ? launch_integrate_mfma_group_cb(g, total, k, code, ext, st)
                   : launch_group_code<false>(g, total, k, code, ext, st);
}

// B source of a launch by default. The compact crossbar when one workgroup covers all
// samples of a core (it alone reads the core's B tiles in the tick) and the
// planes it replaces are large (A x planes >= 256 bytes per neuron, cores of
// >= 256 neurons) and the launch has a workgroup per CU or more; otherwise
// the int8 planes. With one 64-sample tile per workgroup the expansion's
// VALU work is latency nothing hides: measured per network of the 64-variant
// sweep, 512-neuron cores with 512 axons run 8-24% faster, while 64- and
// 128-neuron cores and networks of fewer workgroups than CUs run 2-20%
// slower with the compact source.
bool mfma_compact_b(const DevNet &n, int two_planes, int samples_per_wg)
{
    return n.S <= samples_per_wg && n.N >= 256 && n.A * (two_planes ? 2 : 1) >= 256 && n.C * n.slices >= 256;
}

bool mfma_shape_supported(int A, int N, int two_planes)
{
    const bool ok_a = A == 64 || A == 128 || A == 256 || A == 512;
    // 32-neuron blocks over 8 wavefronts (4 or 8 blocks per slice, 512
    // neurons as two slices, 64 as a slice of 128 with two dead blocks); the
    // B tiles take A * planes / 8 VGPRs per lane, at most 64 (A = 512 with
    // two planes: one plane per wavefront, in 128-neuron slices).
    return ok_a && (N == 64 || N == 128 || N == 256 || N == 512) && A * (two_planes ? 2 : 1) <= 1024;
}

int mfma_width(int A, int N, int two_planes)
{
    // 128 neurons per workgroup for small cores and for the plane split
    return N <= 128 || A * (two_planes ? 2 : 1) > 512 ? 128 : 256;
}
int mfma_slices(int A, int N, int two_planes)
{
    const int w = mfma_width(A, N, two_planes);
    return N > w ? N / w : 1;
}

hipError_t launch_integrate_mfma(const DevNet &n, const TickArgs &a, int two_planes, int samples_per_wg, int compact,
                                 hipStream_t st)
{
    if (!mfma_shape_supported(n.A, n.N, two_planes) || n.slices != mfma_slices(n.A, n.N, two_planes) ||
        n.cnt_rows != n.slices ||
        samples_per_wg <= 0 || samples_per_wg % MFMA_TS ||
        samples_per_wg > MFMA_SPW_MAX || n.vlayout != VLAYOUT_BRICK || n.S64 % MFMA_TS || n.S > n.S64 ||
        (compact ? !n.colbits : !n.planes))
        return hipErrorInvalidValue;
    if (compact)
        return launch_integrate_mfma_cb(n, a, two_planes, samples_per_wg, st);
    return launch_mfma_shape<false>(n, a, two_planes, samples_per_wg, st);
}

}  // namespace ranc
