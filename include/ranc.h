/*
 * ranc.h -- C ABI of the MI355X RANC tick engine.
 *
 * A RANC network (GPU-RANC Sec. II) is a 2-D mesh of cores. Each core has A
 * axons, N neurons, a binary crossbar of synaptic connections, an axon type
 * per axon and a set of G signed weights per neuron (the axon's type selects
 * the weight), plus per-neuron leak, threshold, reset potential and a
 * destination for its spikes. Time advances in ticks. One tick (Algorithm 1)
 * reads each core's scheduled axon spikes for the tick, integrates them
 * through the crossbar and weights, applies leak, threshold and reset, and
 * routes every spike to a destination (core, axon) at a future tick through
 * that core's scheduler (Sec. III-D, III-E) or to the output bus (Sec. IV).
 *
 * The library simulates S independent instances ("samples") of one network
 * side by side on one GPU. All device memory it uses lives in a
 * caller-provided workspace (or, for ranc_load_network_static, in a
 * fixed-size workspace held in the library's code object); the library never
 * allocates device memory.
 *
 * Conventions for every call:
 *   - the return value is a ranc_status; on failure ranc_last_error() gives a
 *     thread-local message that names the offending field;
 *   - validation failures change nothing and allocate nothing;
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream);
 *     calls that launch work return before it finishes; errors raised by the
 *     device surface as RANC_EDEVICE at the next call that synchronizes.
 */
#ifndef RANC_H
#define RANC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RANC_ABI_VERSION 2u

typedef enum ranc_status {
    RANC_OK = 0,
    RANC_EINVAL = -1,       /* malformed argument (null pointer, bad size, bad enum) */
    RANC_ERANGE = -2,       /* a value outside its allowed range (weight, delay, destination...) */
    RANC_ENOMEM = -3,       /* workspace too small, or a host allocation failed */
    RANC_EDEVICE = -4,      /* a HIP call or a kernel failed */
    RANC_ESTATE = -5,       /* call not valid in the handle's state (e.g. ticks no longer retained) */
    RANC_ETRUNC = -6,       /* output buffer too small; the required size is reported */
    RANC_EUNSUPPORTED = -7, /* shape or option the library does not implement */
    RANC_ETIMEOUT = -8      /* a bounded wait inside a persistent launch gave up (the state is
                               undefined until ranc_reset_state) */
} ranc_status;

/* Destination kinds of a neuron's spikes. */
enum { RANC_DEST_NONE = 0, RANC_DEST_CORE = 1, RANC_DEST_OUT = 2 };

/* What a spike does to the firing neuron's potential (Sec. II lists resetting
 * the potential among the per-tick neuron operations; Sec. I and Sec. V make
 * the reset potential's width a configurable axis). */
enum {
    RANC_RESET_ABSOLUTE = 0,  /* the potential becomes the neuron's reset value */
    RANC_RESET_LINEAR = 1     /* the potential becomes U - threshold (what exceeded the
                                 threshold is kept), clamped to the potential range */
};

/* Integration paths (fixed at load time; they differ in device data layout). */
enum {
    RANC_PATH_AUTO = 0,   /* pick per shape */
    RANC_PATH_PLAIN = 1,  /* per (core, sample) workgroups, crossbar words and popcounts */
    RANC_PATH_MFMA = 2,   /* per-core workgroups over sample tiles, exact int8 MFMA;
                             every supported core shape (512 neurons run as 256-neuron
                             workgroups, 64 as a 128-neuron workgroup with half its
                             wavefronts idle, 512 axons with 9-bit weights as
                             128-neuron workgroups with one weight plane per
                             wavefront) */
    RANC_PATH_SPARSE = 3  /* per-core workgroups over sample tiles, event-driven: only spiking
                             axons are visited (never chosen by RANC_PATH_AUTO) */
};

/* Flags of ranc_run_ticks. */
#define RANC_INPUTS_ON_DEVICE 1u
/* Run the call's ticks as one HIP graph: the tick loop for a given
 * (num_ticks, input address) is captured on first use (on a stream the
 * library owns, never on the caller's) and replayed with one graph launch on
 * `stream` afterwards. The scheduler slot and raster row of each tick are
 * read from a tick counter kept in the workspace, so a replay is exact from
 * any starting tick. Results are identical to the per-launch form. A handle
 * keeps at most 16 captured loops; capturing another drops the least recently
 * replayed one (after synchronizing the handle's stream). */
#define RANC_RUN_GRAPH 2u
/* With several networks per call: run the MFMA-path networks of each tick in
 * one persistent launch (one workgroup per compute unit pulls units from a
 * work queue, largest first; LDS sized for the largest shape) instead of one
 * launch per shape class. Results are identical. */
#define RANC_BATCH_PERSISTENT 4u
/* State-resident run (one network per call; MFMA path, cores of 256 neurons
 * and at most 256 axons, no link counting): all ticks of the call in one
 * persistent launch. Each workgroup keeps up to two cores' weight planes in
 * registers and, for one 64-sample group after another, the group's
 * potentials of its cores in LDS across all ticks of the call, so the
 * potentials cross HBM once per call instead of once per tick; the grid
 * synchronizes after every tick (spikes of tick t reach their destinations
 * at t + d, d >= 1, through the spike history in HBM). The grid is launched
 * cooperatively (every workgroup resident at once); every wait at a grid
 * barrier is bounded (2 s, or RANC_RESIDENT_WAIT_US microseconds from the
 * environment), and a wait that gives up ends the launch and the call
 * returns RANC_ETIMEOUT. The call synchronizes `stream` to read that
 * outcome. RANC_RUN_GRAPH is ignored with this flag (one launch per call
 * already). Results are identical to the per-tick forms; calls may mix
 * them on one handle. Networks it cannot run are refused with
 * RANC_EUNSUPPORTED (nothing is queued). */
#define RANC_RUN_RESIDENT 8u

/*
 * Network description (host memory; the library copies it during
 * ranc_load_network, so the caller may free it afterwards).
 * Core c sits at mesh position (x, y) = (c % grid_w, c / grid_w).
 * Supported shapes: num_axons, num_neurons in {64, 128, 256, 512};
 * num_types in {1, 2, 4, 8}; 2 <= weight_bits <= 9; 2 <= potential_bits <= 32;
 * 1 <= max_delay <= 15; num_cores * num_neurons <= 2^23.
 * The neuron-model widths and options at the end of the struct (leak_bits,
 * reset_bits, floor, reset_mode) cover the design space of Sec. I and Sec. V
 * (configurable widths of weight, leak, potential and reset); zero / NULL
 * keeps the defaults (32-bit leak and reset, no floor, absolute reset).
 */
typedef struct ranc_net_desc {
    uint32_t abi_version;      /* must be RANC_ABI_VERSION */
    int32_t num_cores;         /* C = grid_w * grid_h */
    int32_t num_axons;         /* A */
    int32_t num_neurons;       /* N */
    int32_t num_types;         /* G: weights per neuron, one per axon type */
    int32_t weight_bits;       /* weights lie in [-2^(b-1), 2^(b-1) - 1] */
    int32_t potential_bits;    /* P: potentials saturate to [-2^(P-1), 2^(P-1) - 1] once per tick */
    int32_t max_delay;         /* largest tick offset a spike packet may carry */
    int32_t grid_w, grid_h;    /* mesh size */
    const uint32_t *crossbar;  /* [C][A][N/32]: bit n%32 of word n/32 set = axon a connects to neuron n */
    const uint8_t *axon_type;  /* [C][A]: type in [0, G) */
    const int16_t *weight;     /* [C][N][G] */
    const int32_t *leak;       /* [C][N]: added every tick; within [-2^30, 2^30] */
    const int32_t *threshold;  /* [C][N]: a neuron fires when its potential reaches it (>=) */
    const int32_t *reset;      /* [C][N]: potential after a spike; within the P-bit range */
    const int32_t *v_init;     /* [C][N]: initial potential; within the P-bit range */
    const uint8_t *dest_kind;  /* [C][N]: RANC_DEST_* */
    const int16_t *dest_dx;    /* [C][N]: destination core at mesh offset (dx, dy) (CORE only) */
    const int16_t *dest_dy;
    const uint16_t *dest_axon; /* [C][N]: destination axon, < A (CORE only) */
    const uint8_t *dest_delay; /* [C][N]: tick offset in [1, max_delay] (CORE only) */
    int32_t num_input_cores;   /* C_in >= 0 */
    const int32_t *input_cores;/* [C_in]: distinct cores that take external input */
    int32_t leak_bits;         /* leaks are signed leak_bits-bit values, 2..32 (0: 32) */
    int32_t reset_bits;        /* reset values are signed reset_bits-bit values, 2..32 (0: 32);
                                  they must also lie in the potential range */
    const int32_t *floor;      /* [C][N] or NULL (none): a neuron that does not fire and whose
                                  saturated potential U lies below its floor keeps the floor
                                  instead (a negative threshold); within the potential range;
                                  not applied to the value a spike resets to */
    const uint8_t *reset_mode; /* [C][N] RANC_RESET_*, or NULL (all absolute) */
} ranc_net_desc;

/* An output-bus spike. */
typedef struct ranc_spike {
    int64_t tick;
    int32_t core;
    int32_t neuron;
} ranc_spike;

/* Per-sample totals since load or the last reset. */
typedef struct ranc_counters {
    uint64_t emitted;    /* spikes fired */
    uint64_t routed;     /* spikes sent to a (core, axon) */
    uint64_t delivered;  /* scheduler bits set by routed spikes and read at their tick
                            (several spikes to one (core, axon, tick) count once) */
    uint64_t out;        /* spikes sent to the output bus */
    uint64_t events;     /* synaptic events: sum over ticks and cores of
                            (spiking axon, connected neuron) pairs */
} ranc_counters;

typedef struct ranc_net ranc_net;  /* opaque handle */

/* Thread-local description of the last failure in this thread ("" if none). */
const char *ranc_last_error(void);

/*
 * Bytes of device workspace ranc_load_network needs for this network,
 * num_samples instances, at most max_ticks_per_call ticks per
 * ranc_run_ticks call (the output-spike raster and the input staging area
 * hold that many ticks) and the given path. Host-only computation; validates
 * the description like ranc_load_network.
 */
ranc_status ranc_workspace_bytes(const ranc_net_desc *desc, int32_t num_samples,
                                 int32_t max_ticks_per_call, int32_t path, size_t *bytes);

/*
 * Load a network (Sec. II: cores of axons, neurons, a binary crossbar and
 * per-neuron weights selected by axon type, leak, threshold and reset;
 * Sec. III-B: the per-core SRAM that holds these parameters and each
 * neuron's destination packet fields; Algorithm 1: the initial state before
 * the tick loop).
 * Validate the description, lay it out in the workspace (a device buffer of
 * at least ranc_workspace_bytes bytes, 256-byte aligned, owned by the caller
 * and kept alive until ranc_free), upload it on `stream`, and set every
 * instance to its initial state: potentials = v_init, empty schedulers,
 * tick 0. Synchronizes `stream` before returning. *out receives a handle
 * owned by the library until ranc_free.
 */
ranc_status ranc_load_network(const ranc_net_desc *desc, int32_t num_samples,
                              int32_t max_ticks_per_call, int32_t path, void *workspace,
                              size_t workspace_bytes, void *stream, ranc_net **out);

/*
 * The tick loop of Algorithm 1, num_ticks iterations: per tick, scheduler
 * rows advance and the tick's external input spikes are written; every
 * neuron integrates its spiking connected axons' weights, leaks, compares
 * with its threshold and resets (Sec. II, Sec. III-C); every spike is routed
 * to its destination (core, axon) at its tick offset (Sec. III-D, III-E) or
 * to the output bus (Sec. IV).
 * Advance every instance of each of the num_nets networks by num_ticks
 * ticks (1 <= num_ticks <= max_ticks_per_call). inputs[i] (may be NULL for
 * no external input) holds network i's external spikes as
 * [S][num_ticks][C_in][A/32] uint32 bitmaps (bit a%32 of word a/32 = axon a
 * of input core k spikes at that tick), in device memory when flags has
 * RANC_INPUTS_ON_DEVICE, else in host memory (copied to the workspace's
 * staging area first). Consecutive calls continue the same simulation:
 * spikes whose delivery tick lies beyond the call stay scheduled.
 * flags: RANC_INPUTS_ON_DEVICE, RANC_RUN_GRAPH, RANC_BATCH_PERSISTENT,
 * RANC_RUN_RESIDENT (see above); other bits are rejected with RANC_EINVAL. After a
 * call that returned RANC_ETIMEOUT, runs of that handle return RANC_ESTATE until
 * ranc_reset_state. With RANC_RUN_GRAPH and device inputs, the
 * input buffer must stay at the same address to reuse a captured loop.
 *
 * With num_nets > 1 the networks (any shapes, paths and sample counts; each
 * at most once) advance together: per tick, one launch per MFMA shape class
 * (axons, neurons per workgroup, weight planes, potential clamp) runs every
 * MFMA-path network of that class (or, with RANC_BATCH_PERSISTENT, one
 * persistent launch runs all of them from a work queue), and one launch each
 * integrates and routes every plain-path network. The batch tables are kept in the workspace of nets[0] (at most
 * 128 networks per path); they are rebuilt, with a synchronization of
 * `stream`, whenever the list of networks, the input addresses or num_ticks
 * change. Results are identical to running each network alone.
 * Returns after queueing the work on `stream`.
 */
ranc_status ranc_run_ticks(ranc_net *const *nets, int32_t num_nets,
                           const uint32_t *const *inputs, uint32_t flags, int32_t num_ticks,
                           void *stream);

/*
 * The output file of Sec. IV (the spikes the network sends to its output
 * bus, compared one to one between the serial and the GPU simulator):
 * output-bus spikes of one sample with tick_begin <= tick < tick_end, sorted
 * by (tick, core, neuron). Ticks must lie in the retained window: the last
 * max_ticks_per_call ticks run (else RANC_ESTATE). If capacity is too small,
 * *count receives the required number and RANC_ETRUNC is returned.
 * Synchronizes the stream of the last run.
 */
ranc_status ranc_read_spikes(ranc_net *net, int32_t sample, int64_t tick_begin, int64_t tick_end,
                             ranc_spike *out, int64_t capacity, int64_t *count);

/*
 * The same output file in bulk, for every sample at once, so that a long run
 * can be drained chunk by chunk while the next chunk runs (streaming, Sec. V:
 * an application's inputs pass through one instance tick after tick, and its
 * output spikes leave the same way) and decoded away from the critical path.
 * ranc_copy_raster queues on `stream` a kernel that writes the output-bus
 * spikes of ticks [tick_begin, tick_end) (T ticks) into dst, in one of two
 * layouts:
 *   RANC_RASTER_BY_NEURON: uint64 words [T][Nout][ceil(S/64)]; bit i of word
 *     (t, o, w) is set if sample 64 w + i sent a spike from output neuron o to
 *     the output bus at tick tick_begin + t;
 *   RANC_RASTER_BY_SAMPLE: uint32 words [T][S][ceil(Nout/32)]; bit o % 32 of
 *     word (t, s, o / 32) is set for the same event (compact for few samples).
 * Output neurons are numbered in ascending (core, neuron) order among the
 * neurons whose destination is the output bus (ranc_output_neurons lists
 * them). Bits past S samples or Nout neurons are zero; every word of the
 * range is written. dst is any memory the device can write: device memory,
 * or pinned host memory (hipHostMalloc), which the kernel then writes across
 * the bus with no further copy. The ticks must lie in the retained window
 * (the last max_ticks_per_call ticks queued; else RANC_ESTATE) when the call
 * is made, the range must not be empty, and the kernel must run after the
 * runs that produced them (same stream, or ordered by events) and before
 * later runs overwrite them (a run of k ticks reuses the rows of the k oldest
 * retained ticks). RANC_ENOMEM if dst_bytes is below
 * ranc_raster_bytes(net, T, layout); RANC_EINVAL for another layout. Returns
 * after queueing.
 */
#define RANC_RASTER_BY_NEURON 0u
#define RANC_RASTER_BY_SAMPLE 1u
ranc_status ranc_raster_bytes(const ranc_net *net, int64_t num_ticks, uint32_t layout, size_t *bytes);
ranc_status ranc_copy_raster(ranc_net *net, int64_t tick_begin, int64_t tick_end, uint32_t layout, void *dst,
                             size_t dst_bytes, void *stream);
/* (core, neuron) of output neuron o at out[2 o], out[2 o + 1]; *count = Nout.
 * RANC_ETRUNC (with *count set) if capacity < Nout. Host only. */
ranc_status ranc_output_neurons(const ranc_net *net, int32_t *out, int64_t capacity, int64_t *count);

/* Current potentials of one sample into out[C][N] (host). Synchronizes. */
ranc_status ranc_read_potentials(ranc_net *net, int32_t sample, int32_t *out);

/* Counters of one sample. Synchronizes. */
ranc_status ranc_read_counters(ranc_net *net, int32_t sample, ranc_counters *out);

/*
 * Packets per mesh link. In RANC a spike packet reaches its destination core
 * hop by hop through the routers of the cores between, along x first, then
 * along y (Sec. III-D, Fig. 2); the library delivers it directly, and counts,
 * when asked, the links such a route takes.
 * ranc_link_counts_enable: count (1) or stop counting (0) on every tick that
 * later calls of ranc_run_ticks run on this handle (alone or in a batch).
 * Counting adds one small kernel per tick. Changing the setting drops the
 * handle's captured tick loops. Counts start at zero at load and at
 * ranc_reset_state, and accumulate over the ticks run while enabled.
 * ranc_read_links: the counts of one sample into out[C][4] (host): out[c][d]
 * is the number of packets that left core c over its link in direction d
 * (RANC_LINK_XPLUS, _XMINUS, _YPLUS, _YMINUS; +x is towards the core at
 * x + 1, +y towards y + 1). Their sum is the total number of hops. A packet to
 * a neuron's own core takes no link. Synchronizes the stream of the last run.
 */
enum { RANC_LINK_XPLUS = 0, RANC_LINK_XMINUS = 1, RANC_LINK_YPLUS = 2, RANC_LINK_YMINUS = 3 };
ranc_status ranc_link_counts_enable(ranc_net *net, int32_t enable);
ranc_status ranc_read_links(ranc_net *net, int32_t sample, int64_t *out);

/* Next tick to be simulated (ticks run since load or reset). */
ranc_status ranc_current_tick(const ranc_net *net, int64_t *tick);

/* Integration path chosen at load (RANC_PATH_PLAIN or RANC_PATH_MFMA). */
ranc_status ranc_get_path(const ranc_net *net, int32_t *path);

/* Kernel timing, recorded with HIP events on the launch stream around every
 * integration and routing launch (per-launch form) or every tick-loop graph
 * launch (RANC_RUN_GRAPH) while enabled. */
typedef struct ranc_profile {
    double integrate_ms;         /* summed duration of integration launches */
    double route_ms;             /* summed duration of routing launches */
    int64_t integrate_launches;
    int64_t route_launches;
    double graph_ms;             /* summed duration of tick-loop graph launches */
    int64_t graph_launches;
    int64_t graphs_held;         /* captured tick loops the handle holds now (at most 16: the
                                    least recently replayed one is dropped to capture another) */
    int64_t graphs_dropped;      /* captured tick loops dropped since load */
    double resident_ms;          /* summed duration of state-resident launches (RANC_RUN_RESIDENT) */
    int64_t resident_launches;
} ranc_profile;

/* Enable (1) or disable (0) timing; enabling clears the totals. Host-side only. */
ranc_status ranc_profile_enable(ranc_net *net, int32_t enable);

/* Totals since timing was enabled. Synchronizes the stream of the last run. */
ranc_status ranc_profile_read(ranc_net *net, ranc_profile *out);

/* Launch shape of a handle (path specific; fields of the other path are 0). */
typedef struct ranc_tune {
    int32_t samples_per_wg;          /* MFMA path: samples per workgroup (multiple of 64, <= 512) */
    int32_t route_samples_per_block; /* plain path router: samples per block (1, 2, 4, 8) */
    int32_t route_split;             /* plain path router: blocks sharing one group of samples */
    int32_t route_stage;             /* plain path router: spike bitmaps staged in LDS (0/1) */
    double ms_per_tick;              /* ranc_autotune: time per tick of the chosen shape */
    int32_t candidates;              /* ranc_autotune: number of shapes timed */
    int32_t route_lanes_per_word;    /* plain path router: 1 = one lane per destination word
                                        (the three router fields above apply); 8 = eight lanes
                                        per word, one sample per block row (they do not); 0 in
                                        ranc_set_launch_shape = chosen automatically (8 when
                                        the one-lane launch would have fewer blocks than the
                                        GPU has compute units). Batched routing of several
                                        networks always runs one lane per word. */
} ranc_tune;

/*
 * Autotuner: time every candidate launch shape of the handle's path (MFMA:
 * samples per workgroup; plain: router samples per block x split x LDS
 * staging) on num_ticks ticks of `inputs` (as for ranc_run_ticks; flags may
 * hold RANC_INPUTS_ON_DEVICE), each from the initial state after one untimed
 * pass, and keep the fastest. Results never depend on the shape. Leaves every
 * instance in its initial state (as ranc_reset_state) and drops captured
 * tick loops. Synchronizes `stream`; *out receives the chosen shape.
 */
ranc_status ranc_autotune(ranc_net *net, const uint32_t *inputs, uint32_t flags, int32_t num_ticks,
                          void *stream, ranc_tune *out);

/* Set a launch shape (e.g. one cached from an earlier ranc_autotune) or read
 * the current one. Setting validates the shape (RANC_EINVAL) and drops
 * captured tick loops; the simulation state is unchanged. */
ranc_status ranc_set_launch_shape(ranc_net *net, const ranc_tune *shape);
ranc_status ranc_get_launch_shape(const ranc_net *net, ranc_tune *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): load a
 * network as ranc_load_network does, into a workspace the library holds
 * instead of a caller-provided one. The library keeps one such workspace of
 * RANC_STATIC_WORKSPACE_BYTES bytes per device, in its code object (each
 * device the library runs on holds it until the process ends); the network
 * goes to the current device's. Allocates no device memory and calls no
 * allocating HIP or library routine.
 * Errors: RANC_ENOMEM if the network, num_samples and max_ticks_per_call
 * need more than RANC_STATIC_WORKSPACE_BYTES (ranc_workspace_bytes gives the
 * need); RANC_ESTATE while another handle loaded this way on the same device
 * has not been freed (one handle per device at a time; ranc_free releases the
 * workspace); RANC_EUNSUPPORTED for a device index >= 64; otherwise as
 * ranc_load_network. The workspace keeps what the previous handle left in
 * it; loading overwrites everything the simulation reads. Calls on a handle
 * loaded this way behave exactly as on any other handle, and as for any
 * handle, calls that overlap on it (from several threads or streams) race.
 */
#define RANC_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
ranc_status ranc_load_network_static(const ranc_net_desc *desc, int32_t num_samples,
                                     int32_t max_ticks_per_call, int32_t path, void *stream,
                                     ranc_net **out);

/* Return every instance to its initial state (queued on `stream`). */
ranc_status ranc_reset_state(ranc_net *net, void *stream);

/* Release the handle (the workspace stays the caller's). NULL is a no-op. */
void ranc_free(ranc_net *net);

#ifdef __cplusplus
}
#endif

#endif /* RANC_H */
