// ranc_internal.h -- device data layout shared by the host runtime and the kernels.
//
// Notation: C cores, A axons and N neurons per core, G axon types,
// W = A/32 axon words, NW = N/32 neuron words, D = max delay, Q = D + 1
// scheduler slots, S samples (S64: S rounded up to 64), HG = S64/64,
// RT retained raster ticks, Wout output words, Nout output neurons.
//
// Parameters (written once at load):
//   colbits  u32 [C][W][N]     bit b of colbits[c][w][n] = crossbar(c, 32w+b, n)   (plain, sparse)
//   typemask u32 [C][G][W]     bit b of typemask[c][g][w] = (type(c, 32w+b) == g)
//   wts      i32 [C][G][N]     weight of neuron n for axon type g
//   leak, thr, rst, vinit i32 [C][N]
//   floor    i32 [C][N]        lowest potential a neuron that does not fire keeps (vmin: none)
//   linmask  u32 [C][NW]       neurons whose spike subtracts the threshold (linear reset)
//   coremask, outmask u32 [C][NW]  neurons whose destination is a core / the output bus
//   outword  i32 [C][NW]       raster column of that neuron word, -1 if it has no output neuron
//   outidx   i32 [C][N]        (MFMA path) index of the neuron among output-bus neurons, -1 if none
//   in_index i32 [C]           input slot of the core, -1 if it takes no external input
//   routing table (plain path; destination-owned, one list per destination axon
//   word dw = c*W + w), stored wave-interleaved: words are grouped by 64; group
//   g holds its words' lists as rt_ent[rt_goff[g] + k*64 + (dw % 64)], each
//   list sorted by delay; rt_dcnt u16 [C*W][DMAX] counts the entries of each
//   delay (DMAX = max delay rounded up to 4, 8 or 16). Entry bits: [0,5)
//   destination axon % 32, [5,9) delay - 1, [9,32) source neuron c*N + n.
//   degb     u32 [C][2][A/4]   (MFMA path) connected neurons per axon, low byte
//                              plane then high byte plane, 4 axons per word
//   planes   int8 MFMA B operand tiles (MFMA path), see kern_mfma.hip
//   ecsr_ptr u32 [C][slices][A+1], ecsr_ent u16  (sparse path) per (core, slice of <= 128
//                              neurons) one row per axon: its connected neurons of the slice,
//                              entry = neuron within the slice | weight for the axon's type << 7
//   rtx_ptr  u32 [C*A + 1], rtx_ent u32 [E]  (MFMA and sparse) the same routing table keyed by
//                              destination axon: entries (source neuron c*N + n) << 4 | (delay - 1)
//   linkrec  int2 [C][N]       mesh path ends of each neuron's packets (kern_links.hip): x = -1
//                              if the packet takes no x hop, else 2 * (core at (xd, ys)) + (dx < 0);
//                              y = -1 if it takes no y hop, else 2 * (core at (xd, yd)) + (dy < 0)
// State:
//   V        i32, layout by path:
//              plain: [C][S][N]
//              MFMA:  [C][N/32][S64/32][4][64][4]: brick (c, nb, g) holds 32 samples
//                     x 32 neurons; element (q, lane l, e) = sample 32g + 8q + 4(l/32) + e,
//                     neuron 32nb + l%32 (the MFMA result layout)
//              sparse: [C][N][S64] (a neuron's samples contiguous)
//   plain path:
//   ring     u32 [Q][S][C][W]  scheduler: slot t%Q holds the axon spikes of tick t
//   spk      u32 [S][C][NW]    spikes of the current tick
//   raster   u32 [RT][S][Wout] output-bus spikes of tick t in row t%RT
//   sparse path:
//   ring     u32 [C][S64][W]   delivered axon spikes of the tick being integrated (the
//                              scheduler row it reads), written by the delivery kernel
//   MFMA and sparse paths:
//   hist     u64 [Q][C*N][HG]  spikes of tick t in slot t%Q; word (slot, neuron, i)
//                              covers samples 64i .. 64i+63; MFMA: bit p = sample
//                              64i + 32(p/32) + sigma(p%32) with
//                              sigma(b) = 8((b%16)/4) + 4(b/16) + b%4; sparse: bit p =
//                              sample 64i + p
//   raster   u64 [RT][Nout][HG] output-bus spikes of tick t in row t%RT, words as hist
//   both:
//   cnt      u64 [C*cnt_rows][S][5]  emitted, routed, delivered, out, events (summed over
//                              the rows of a core when read)
//   linkd    i64 [4][C][S64]   difference arrays of the packets per mesh link (+x, -x, +y, -y),
//                              summed along mesh rows / columns when read
//   tick     i32 [4]           scheduler slot (t % Q) and raster row (t % RT) of the
//                              first tick of the next call, and t as two u32 halves;
//                              kept on the device so a captured tick loop replays
//                              correctly from any starting tick
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranc {

enum { CNT_EMITTED = 0, CNT_ROUTED, CNT_DELIVERED, CNT_OUT, CNT_EVENTS, CNT_N };
enum { VLAYOUT_CSN = 0, VLAYOUT_BRICK = 1, VLAYOUT_SPARSE = 2 };

// Routing entry fields.
static constexpr int RT_POS_BITS = 5, RT_DELAY_SHIFT = 5, RT_SRC_SHIFT = 9;
static constexpr long long RT_MAX_NEURONS = 1LL << 23;

struct DevNet {
    int C, A, N, G, W, NW, D, Q, S, S64, RT, Wout, Nout, Cin, vlayout;
    int cnt_rows;   // counter rows per core, summed when read (plain: one per 64 neurons, MFMA: one per slice)
    int slices;     // neuron slices per core, one workgroup each (MFMA: N / slices <= 256; sparse: <= 128)
    int32_t vmin, vmax;
    int model_ext;  // extended potential update: clamp to [vmin, vmax], floor, linear reset
    // parameters
    const uint32_t *colbits, *typemask;
    const int32_t *wts, *leak, *thr, *rst, *vinit;
    const int32_t *floor;      // [C][N] (vmin where the neuron has none)
    const uint32_t *linmask;   // [C][NW] neurons in linear-reset mode
    const uint32_t *coremask, *outmask;
    const int32_t *outword, *in_index;
    const uint16_t *rt_dcnt;
    const uint32_t *rt_goff, *rt_ent;
    const int32_t *outidx;
    const uint32_t *degb;
    const uint4 *planes;
    const uint32_t *rtx_ptr, *rtx_ent;
    const uint64_t *hist_zero;   // HG zero words (a history row with no spikes)
    const uint32_t *ecsr_ptr;    // sparse path: row starts [C][slices][A+1]
    const uint16_t *ecsr_ent;    // sparse path: row entries (neuron in slice | weight << 7)
    // state
    int32_t *V;
    uint32_t *ring, *spk, *raster;
    uint64_t *hist;
    unsigned long long *cnt;     // totals [C][cnt_rows][S][CNT_N]
    unsigned long long *cring;   // per-tick packed counts [RT][C * cnt_rows][S], folded per call
    int *tick;
};

// Mesh link statistics (kern_links.hip); kept out of DevNet, which travels
// in batched kernels' arguments.
struct LinkArgs {
    const int2 *rec;         // linkrec [C][N]
    long long *d;            // linkd [4][C][S64]
    const uint32_t *rows;    // sample-tiled paths: row starts [4 C + 1] of the entries per (direction, core)
    const uint32_t *ents;    // entries: source neuron << 1 | (1: the run ends here, 0: it starts here)
};

// Per-tick launch arguments: the tick's position k in the call (the tick is
// the device tick of the call's start plus k, k < RT).
struct TickArgs {
    int k;
    const uint32_t *ext_t;  // external input of this tick for sample 0, or nullptr
    long long ext_sstride;  // words between consecutive samples of the input block
};

// Arguments of the state-resident MFMA tick loop (kern_resident.hip): the
// call's external input (sample s, tick k, input core i, word w at
// ext_base[s * ext_sstride + k * tick_words + i * W + w], or nullptr) and
// its number of ticks.
struct ResidentArgs {
    const uint32_t *ext_base;
    long long ext_sstride;
    long long tick_words;
    int num_ticks;
};

// Grid synchronization words of the state-resident loop: arrival counter and
// give-up flag (zeroed before each launch), and the longest wait, in ticks of
// the device's constant-rate wall clock.
struct ResSync {
    unsigned *ctr;
    unsigned *abort;
    unsigned long long wait_ticks;
};

// Scheduler slot and raster row of the tick at position k of the call.
__device__ inline int tick_slot(const DevNet &n, int k) { return (n.tick[0] + k) % n.Q; }
__device__ inline int tick_row(const DevNet &n, int k) { return (n.tick[1] + k) % n.RT; }

// Core c and unit v (0 <= v < U) of workgroup `bid` of a grid of C * U
// workgroups. The GPU spreads consecutive workgroups over its 8 XCDs (each
// with its own L2) round robin, so with a multiple of 8 cores the units of a
// core are numbered 8 apart inside a run of 8 cores: they are dispatched
// together on XCD c % 8 and share the core's weights in its L2. (Putting
// runs of 4 neighbouring cores on one XCD as well, so that they share the
// cache lines of their input words, measured 0.8% slower on the 512-core
// net and no faster on the 16384-core mesh.) Otherwise cores run fastest.
__device__ inline void core_unit_of(int bid, int C, int U, int &c, int &v)
{
    if ((C & 7) == 0) {
        const int t = bid >> 3;
        c = (t / U) << 3 | (bid & 7);
        v = t % U;
    } else {
        c = bid % C;
        v = bid / C;
    }
}

// One tick's counts of one counter row and sample, packed into 64 bits:
// emitted, routed, output-bus and delivered spikes in 10 bits each (at most
// 512 per row and tick) and synaptic events in 24 bits (at most 512 * 512).
// A tick writes its word at the tick's raster row of `cring`; the call's
// words are added into the 64-bit totals once, after its last tick.
__device__ inline unsigned long long pack_counts(unsigned emitted, unsigned routed, unsigned out,
                                                 unsigned delivered, unsigned events)
{
    return (unsigned long long)emitted | (unsigned long long)routed << 10 | (unsigned long long)out << 20 |
           (unsigned long long)delivered << 30 | (unsigned long long)events << 40;
}
__device__ inline void store_counts(const DevNet &n, int k, size_t row, int s, unsigned long long packed)
{
    n.cring[((size_t)tick_row(n, k) * n.C * n.cnt_rows + row) * n.S + s] = packed;
}

// One network of a batch advanced together (several networks per launch).
// unit_begin: the network's first unit in the launch's numbering; code:
// kernel variant of the network's shape (path specific).
struct BatchEntry {
    DevNet n;
    const uint32_t *ext_base;   // inputs of the call ([S][T][Cin][W]), or nullptr
    long long tick_words;       // Cin * W
    long long ext_sstride;      // num_ticks * tick_words
    int spw;                    // samples per workgroup (MFMA path)
    int code;
    int unit_begin, units;      // integration units
    int route_begin, route_units, route_code, route_split;   // plain path: router units and shape
    int phase;                  // cache-sized phase of the batch (host bookkeeping)
    int compact;                // MFMA path: B tiles built from the compact crossbar (host bookkeeping)
};

// Networks of one MFMA shape class in one launch, passed by value as kernel
// arguments (at most 4 KiB): pointers read from kernel arguments are known
// to address global memory, so the kernel's accesses through them are
// global (not flat) loads and stores, as in the single-network kernel.
constexpr int MFMA_GROUP_MAX = 11;
struct MfmaGroupEntry {
    DevNet n;
    const uint32_t *ext_base;   // inputs of the call ([S][T][Cin][W]), or nullptr
    long long tick_words;       // Cin * W
    long long ext_sstride;      // num_ticks * tick_words
    int spw;                    // samples per workgroup
    int unit_begin;             // first unit of the network in the launch
};
struct MfmaGroupArgs {
    int num;
    MfmaGroupEntry e[MFMA_GROUP_MAX];
};

// Index of the last entry of tab[0, num) whose first unit (unit_begin, or
// route_begin with `route`) is <= u; the first units increase along the
// table and entry 0 starts at 0. Each lane of the wavefront compares one
// entry, so the lookup is one round of parallel loads instead of a chain of
// dependent ones. The result is wave-uniform.
__device__ inline int batch_entry_of(const BatchEntry *tab, int num, int u, bool route)
{
    const int lane = threadIdx.x & 63;
    int count = 0;
    for (int base = 0; base < num; base += 64) {
        const int i = base + lane;
        const int first = i < num ? (route ? tab[i].route_begin : tab[i].unit_begin) : INT32_MAX;
        count += __popcll(__ballot(first <= u));
    }
    return __builtin_amdgcn_readfirstlane(count - 1);
}

// Route launch shape (chosen per network by the runtime).
struct RouteCfg {
    int samples_per_block;  // 1, 2, 4 or 8 spike bitmaps per block
    int blocks_per_group;   // blocks sharing one group of samples (split of the destination words)
    int stage;              // stage the bitmaps in LDS
    int lanes;              // lanes per destination word: 1 (k_route, the fields above apply) or
                            // route_split_lanes() (k_route_split: one sample per block row)
};

// Launchers (return the first HIP error, hipSuccess otherwise).
hipError_t launch_integrate_plain(const DevNet &n, const TickArgs &a, hipStream_t st);
hipError_t launch_integrate_sparse(const DevNet &n, const TickArgs &a, int samples_per_wg, hipStream_t st);
bool sparse_shape_supported(int A, int N, int G);
int sparse_max_samples_per_wg();
int sparse_slice_width(int N);   // neurons per sparse-path workgroup
int sparse_row_align();          // entries each slice's rows are aligned to
// compact: B tiles built from the compact crossbar (R_BSRC), else read from the planes
hipError_t launch_integrate_mfma(const DevNet &n, const TickArgs &a, int two_planes, int samples_per_wg, int compact,
                                 hipStream_t st);
// State-resident MFMA tick loop (N = 256 in one slice, A <= 256, at most
// resident_max_cores_per_wg() cores per workgroup): zeroes the sync words,
// then launches `grid` workgroups cooperatively.
hipError_t launch_mfma_resident(const DevNet &n, const ResidentArgs &ra, const ResSync &sy, int grid, int two_planes,
                                hipStream_t st);
int resident_blocks_per_cu(int A, int two_planes, int ext);   // 0: the shape is not built
int resident_max_cores_per_wg();
hipError_t launch_route(const DevNet &n, int k, const RouteCfg &cfg, hipStream_t st);
hipError_t launch_reset_state(const DevNet &n, const LinkArgs &l, hipStream_t st);
hipError_t launch_advance_tick(const DevNet &n, int num_ticks, hipStream_t st);
hipError_t launch_fold_counts(const DevNet &n, int num_ticks, hipStream_t st);
hipError_t launch_link_counts(const DevNet &n, const LinkArgs &l, int k, hipStream_t st);
// Output-bus spikes of ticks [t0, t0 + T) (all retained) into dst, by neuron
// (u64 [T][Nout][S64/64]) or by sample (u32 [T][S][ceil(Nout/32)]), bits in
// sample order (kern_raster.hip). Plain path tables: outcol[ow] = (index
// c * NW + w of raster column ow's neuron word, output index of its first
// output neuron); opos[o] = raster column of output neuron o << 5 | its bit.
hipError_t launch_pack_raster(const DevNet &n, const int2 *outcol, const int32_t *opos, int by_sample, long long t0,
                              int T, void *dst, hipStream_t st);
bool mfma_shape_supported(int A, int N, int two_planes);
int mfma_width(int A, int N, int two_planes);   // neurons per MFMA workgroup (128 or 256)
int mfma_slices(int A, int N, int two_planes);  // MFMA workgroups per core and sample chunk
int mfma_shape_code(int A, int N, int two_planes);
int plain_shape_code(int W, int G);
int route_shape_code(const RouteCfg &cfg, int max_delay);
hipError_t launch_integrate_plain_batch(const BatchEntry *tab, int num, int total, int k, hipStream_t st);
hipError_t launch_route_batch(const BatchEntry *tab, int num, int total, int k, size_t lds_bytes, hipStream_t st);
hipError_t launch_advance_batch(const BatchEntry *tab, int num, int num_ticks, unsigned *queue, hipStream_t st);
hipError_t launch_integrate_mfma_batch(const BatchEntry *tab, int num, int total, int k, unsigned *queue,
                                       int workgroups, hipStream_t st);
// Whether a launch of this network should build its B tiles from the compact
// crossbar (R_BSRC) rather than read the int8 weight planes (kern_mfma.hip)
bool mfma_compact_b(const DevNet &n, int two_planes, int samples_per_wg);
// compact: B tiles built from the compact crossbar (chosen for every network
// of the group), else read from the weight planes
hipError_t launch_integrate_mfma_group(const MfmaGroupArgs &g, int total, int k, int code, int ext, int compact,
                                       hipStream_t st);
// the compact-B forms (kern_mfma_cb.hip); arguments validated by the callers above
hipError_t launch_integrate_mfma_cb(const DevNet &n, const TickArgs &a, int two_planes, int samples_per_wg,
                                    hipStream_t st);
hipError_t launch_integrate_mfma_group_cb(const MfmaGroupArgs &g, int total, int k, int code, int ext,
                                          hipStream_t st);
RouteCfg route_default_cfg(const DevNet &n);
int route_split_lanes();
// Lanes per word chosen for a configuration: the lane-split router when the
// one-lane launch would have fewer blocks than the GPU has compute units.
int route_auto_lanes(const DevNet &n, const RouteCfg &cfg);
int route_dmax(int max_delay);
int mfma_max_samples_per_wg();

// The library-held workspace of ranc_load_network_static (static_ws.hip).
// static_ws_claim looks up the device address of device `dev`'s array (the
// first time, with `dev` current) and claims it for one handle; *held is set
// (and *addr left null) while another handle holds it.
constexpr int STATIC_WS_MAX_DEVICES = 64;
hipError_t static_ws_claim(int dev, void **addr, bool *held);
void static_ws_release(int dev);

}  // namespace ranc
