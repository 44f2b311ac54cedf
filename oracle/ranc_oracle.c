/*
 * ranc_oracle.c -- serial, tick-accurate RANC simulator used as the oracle.
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's shared object; the simulation library
 * never does, and this file shares no code, header or table with it.
 *
 * What it computes follows the RANC simulator algorithm of GPU-RANC
 * (Algorithm 1, "RANC Simulator Algorithm", and Sec. II), for ONE independent
 * network instance ("sample"), one tick at a time:
 *
 *   1. every core: clear its scheduler-SRAM row of the previous tick and
 *      advance the index of the current tick's row (Sec. III-E, scheduler);
 *   2. every external input packet of this tick: write its spike bit into the
 *      destination core's current row (Algorithm 1, packet loop);
 *   3. neuron block, every core and neuron: accumulate, over all axons whose
 *      current-row bit is set and that are connected to the neuron, the
 *      neuron's weight for that axon's type; then add the leak, compare with
 *      the threshold, and reset on a spike (Sec. II: LIF model, four weights
 *      per neuron selected by axon type; Algorithm 1 neuron loop and "additional
 *      computation / checks");
 *   4. router, every core and neuron that spiked: build the packet, move it one
 *      mesh hop at a time (along x first, then along y) to its
 *      destination core, counting the mesh link each hop takes (Fig. 2: a
 *      packet reaches its core through the routers of the cores between), and
 *      set the destination axon's bit in that core's
 *      scheduler row at the packet's tick offset (Sec. II, Sec. III-D); a
 *      neuron whose destination is the output bus records (tick, core, neuron)
 *      instead (Sec. IV, output file).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - a neuron fires when its post-leak potential is >= its threshold;
 *   - leak is applied to every neuron on every tick;
 *   - the sum V + I + leak is formed exactly (int64) and clamped once per tick
 *     to a signed potential_bits-bit range;
 *   - on a spike the potential becomes the neuron's reset value (absolute
 *     reset) or, for a neuron in linear-reset mode, U - threshold clamped to
 *     the potential range;
 *   - a neuron that does not fire and whose U lies below its floor (a
 *     negative threshold) keeps the floor instead; the floor does not apply
 *     to the value a spike resets to;
 *   - leaks, reset potentials and weights are signed values of leak_bits,
 *     reset_bits and weight_bits bits (Sec. I and Sec. V name these widths as
 *     configurable); a value outside its width is rejected;
 *   - several packets to the same (core, axon, tick) set one bit (the scheduler
 *     SRAM is an array of booleans), so they count once;
 *   - a packet with tick offset d written during tick t is read at tick t+d,
 *     1 <= d <= max_delay, and the scheduler has max_delay+1 rows;
 *   - external input for tick t is read at tick t;
 *   - packets still pending when a run call ends stay in the scheduler and are
 *     read by a later call.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_TRUNCATED 1
#define ORC_EBADNET (-1)
#define ORC_EROUTE (-2)
#define ORC_ENOMEM (-3)

/* counters */
enum { ORC_EMITTED = 0, ORC_ROUTED, ORC_DELIVERED, ORC_OUT, ORC_EVENTS, ORC_HOPS, ORC_NCOUNTERS };

enum { ORC_DEST_NONE = 0, ORC_DEST_CORE = 1, ORC_DEST_OUT = 2 };

enum { ORC_RESET_ABSOLUTE = 0, ORC_RESET_LINEAR = 1 };

/* Directions of the mesh link a hop takes, out of the core it leaves. */
enum { ORC_LINK_XPLUS = 0, ORC_LINK_XMINUS, ORC_LINK_YPLUS, ORC_LINK_YMINUS, ORC_NLINKS };

typedef struct orc_net {
    int32_t num_cores, num_axons, num_neurons, num_types;
    int32_t weight_bits, potential_bits, max_delay, grid_w, grid_h;
    const uint32_t *crossbar;   /* [C][A][ceil(N/32)] */
    const uint8_t *axon_type;   /* [C][A] */
    const int16_t *weight;      /* [C][N][G] */
    const int32_t *leak, *threshold, *reset, *v_init; /* [C][N] */
    const uint8_t *dest_kind;   /* [C][N] */
    const int16_t *dest_dx, *dest_dy;
    const uint16_t *dest_axon;
    const uint8_t *dest_delay;
    int32_t num_input_cores;
    const int32_t *input_cores; /* [C_in] */
    int32_t leak_bits, reset_bits;
    const int32_t *floor;       /* [C][N] lowest potential kept without firing, or NULL (none) */
    const uint8_t *reset_mode;  /* [C][N] ORC_RESET_*, or NULL (all absolute) */
} orc_net;

typedef struct orc_sim {
    orc_net net;
    int32_t rows;          /* scheduler rows per core */
    int64_t tick;          /* next tick to simulate */
    int32_t *potential;    /* [C][N] */
    uint8_t *sram;         /* scheduler SRAM [C][rows][A] of booleans */
    int32_t *curr;         /* [C] row of the current tick */
    uint8_t *spiked;       /* [C][N] spike flags of the current tick */
    int32_t *active;       /* [A] axons of the core being integrated that hold a spike */
    int64_t *links;        /* [C][ORC_NLINKS] packets that left core c over each of its links */
    int64_t counters[ORC_NCOUNTERS];
} orc_sim;

static int connected(const orc_net *n, int c, int a, int j)
{
    int words = (n->num_neurons + 31) / 32;
    uint32_t w = n->crossbar[((size_t)c * n->num_axons + a) * words + j / 32];
    return (int)((w >> (j % 32)) & 1u);
}

static int input_bit(const uint32_t *ext, const orc_net *n, int k, int i, int a)
{
    int words = (n->num_axons + 31) / 32;
    uint32_t w = ext[((size_t)k * n->num_input_cores + i) * words + a / 32];
    return (int)((w >> (a % 32)) & 1u);
}

static uint8_t *sram_row(orc_sim *s, int c, int row)
{
    return s->sram + ((size_t)c * s->rows + row) * s->net.num_axons;
}

/* Move a packet hop by hop across the mesh; returns the destination core or
 * -1 if it would leave the grid. Each hop is counted in *hops and, if links
 * is not NULL, on the link it takes out of the core it leaves. */
static int route_hops(const orc_net *n, int core, int dx, int dy, int64_t *hops, int64_t *links)
{
    int x = core % n->grid_w, y = core / n->grid_w;
    while (dx != 0) {
        int step = dx > 0 ? 1 : -1;   /* along x */
        if (links)
            ++links[((size_t)y * n->grid_w + x) * ORC_NLINKS + (step > 0 ? ORC_LINK_XPLUS : ORC_LINK_XMINUS)];
        x += step;
        dx -= step;
        ++*hops;
        if (x < 0 || x >= n->grid_w)
            return -1;
    }
    while (dy != 0) {
        int step = dy > 0 ? 1 : -1;   /* along y */
        if (links)
            ++links[((size_t)y * n->grid_w + x) * ORC_NLINKS + (step > 0 ? ORC_LINK_YPLUS : ORC_LINK_YMINUS)];
        y += step;
        dy -= step;
        ++*hops;
        if (y < 0 || y >= n->grid_h)
            return -1;
    }
    return y * n->grid_w + x;
}

int orc_check(const orc_net *n)
{
    if (n->num_cores < 1 || n->num_axons < 1 || n->num_neurons < 1 || n->num_types < 1)
        return ORC_EBADNET;
    if (n->grid_w < 1 || n->grid_h < 1 || n->grid_w * n->grid_h != n->num_cores)
        return ORC_EBADNET;
    if (n->max_delay < 1 || n->potential_bits < 2 || n->potential_bits > 32)
        return ORC_EBADNET;
    for (int c = 0; c < n->num_cores; ++c)
        for (int a = 0; a < n->num_axons; ++a)
            if (n->axon_type[(size_t)c * n->num_axons + a] >= n->num_types)
                return ORC_EBADNET;
    if (n->leak_bits < 2 || n->leak_bits > 32 || n->reset_bits < 2 || n->reset_bits > 32)
        return ORC_EBADNET;
    {
        const int64_t lmax = ((int64_t)1 << (n->leak_bits - 1)) - 1, lmin = -((int64_t)1 << (n->leak_bits - 1));
        const int64_t rmax = ((int64_t)1 << (n->reset_bits - 1)) - 1, rmin = -((int64_t)1 << (n->reset_bits - 1));
        const int64_t vmax = ((int64_t)1 << (n->potential_bits - 1)) - 1, vmin = -((int64_t)1 << (n->potential_bits - 1));
        for (size_t i = 0; i < (size_t)n->num_cores * n->num_neurons; ++i) {
            if (n->leak[i] < lmin || n->leak[i] > lmax)
                return ORC_EBADNET;
            if (n->reset[i] < rmin || n->reset[i] > rmax)
                return ORC_EBADNET;
            if (n->floor && (n->floor[i] < vmin || n->floor[i] > vmax))
                return ORC_EBADNET;
            if (n->reset_mode && n->reset_mode[i] > ORC_RESET_LINEAR)
                return ORC_EBADNET;
        }
    }
    for (size_t i = 0; i < (size_t)n->num_cores * n->num_neurons; ++i) {
        if (n->dest_kind[i] == ORC_DEST_CORE) {
            int64_t hops = 0;
            int c = (int)(i / n->num_neurons);
            if (n->dest_delay[i] < 1 || n->dest_delay[i] > n->max_delay)
                return ORC_EBADNET;
            if (n->dest_axon[i] >= n->num_axons)
                return ORC_EBADNET;
            if (route_hops(n, c, n->dest_dx[i], n->dest_dy[i], &hops, NULL) < 0)
                return ORC_EROUTE;
        }
    }
    for (int i = 0; i < n->num_input_cores; ++i)
        if (n->input_cores[i] < 0 || n->input_cores[i] >= n->num_cores)
            return ORC_EBADNET;
    return ORC_OK;
}

orc_sim *orc_new(const orc_net *n)
{
    if (orc_check(n) != ORC_OK)
        return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s)
        return NULL;
    s->net = *n;
    s->rows = n->max_delay + 1;
    size_t cn = (size_t)n->num_cores * n->num_neurons;
    s->potential = (int32_t *)malloc(cn * sizeof(int32_t));
    s->spiked = (uint8_t *)calloc(cn, 1);
    s->sram = (uint8_t *)calloc((size_t)n->num_cores * s->rows * n->num_axons, 1);
    s->curr = (int32_t *)malloc((size_t)n->num_cores * sizeof(int32_t));
    s->active = (int32_t *)malloc((size_t)n->num_axons * sizeof(int32_t));
    s->links = (int64_t *)calloc((size_t)n->num_cores * ORC_NLINKS, sizeof(int64_t));
    if (!s->potential || !s->spiked || !s->sram || !s->curr || !s->active || !s->links) {
        free(s->potential); free(s->spiked); free(s->sram); free(s->curr); free(s->active); free(s->links); free(s);
        return NULL;
    }
    memcpy(s->potential, n->v_init, cn * sizeof(int32_t));
    /* Before tick 0 the "previous" row is the last one, so the first advance
     * makes row 0 the current row. */
    for (int c = 0; c < n->num_cores; ++c)
        s->curr[c] = s->rows - 1;
    s->tick = 0;
    return s;
}

void orc_free(orc_sim *s)
{
    if (!s)
        return;
    free(s->potential); free(s->spiked); free(s->sram); free(s->curr); free(s->active); free(s->links); free(s);
}

/*
 * Advance the instance by T ticks.
 *   ext          external input bitmaps [T][C_in][ceil(A/32)] (may be NULL: no input)
 *   out_events   output-bus spikes as int64 triples (tick, core, neuron), in the
 *                order the router visits them, which is (tick, core, neuron)
 *   cap          capacity of out_events in triples; *n_out receives the total
 *                count even when it exceeds cap (then ORC_TRUNCATED)
 *   spike_trace  optional [T][C][N] spike flags
 *   v_trace      optional [T][C][N] potentials after each tick
 */
int orc_run(orc_sim *s, const uint32_t *ext, int32_t T, int64_t *out_events, int64_t cap,
            int64_t *n_out, uint8_t *spike_trace, int32_t *v_trace)
{
    const orc_net *n = &s->net;
    const int C = n->num_cores, A = n->num_axons, N = n->num_neurons, G = n->num_types;
    const int64_t vmax = ((int64_t)1 << (n->potential_bits - 1)) - 1;
    const int64_t vmin = -((int64_t)1 << (n->potential_bits - 1));
    int64_t count = 0;

    for (int32_t k = 0; k < T; ++k, ++s->tick) {
        /* Scheduler: drop the previous tick's row, advance to this tick's row. */
        for (int c = 0; c < C; ++c) {
            memset(sram_row(s, c, s->curr[c]), 0, (size_t)A);
            s->curr[c] = (s->curr[c] + 1) % s->rows;
        }
        /* Spikes that earlier ticks' packets left in this tick's rows. */
        for (int c = 0; c < C; ++c) {
            const uint8_t *row = sram_row(s, c, s->curr[c]);
            for (int a = 0; a < A; ++a)
                s->counters[ORC_DELIVERED] += row[a];
        }
        /* External input packets of this tick (tick offset 0). */
        if (ext) {
            for (int i = 0; i < n->num_input_cores; ++i) {
                int c = n->input_cores[i];
                uint8_t *row = sram_row(s, c, s->curr[c]);
                for (int a = 0; a < A; ++a)
                    if (input_bit(ext, n, k, i, a))
                        row[a] = 1;
            }
        }
        /* Neuron block. */
        for (int c = 0; c < C; ++c) {
            const uint8_t *row = sram_row(s, c, s->curr[c]);
            /* An axon without a spike adds nothing to any neuron's sum, so the
             * accumulation visits only the axons whose bit is set. */
            int nact = 0;
            for (int a = 0; a < A; ++a)
                if (row[a])
                    s->active[nact++] = a;
            for (int j = 0; j < N; ++j) {
                size_t cj = (size_t)c * N + j;
                int64_t acc = 0;
                int64_t events = 0;
                for (int k = 0; k < nact; ++k) {
                    const int a = s->active[k];
                    /* a term counts iff the axon holds a spike and is connected */
                    int hit = row[a] & connected(n, c, a, j);
                    int type = n->axon_type[(size_t)c * A + a];
                    acc += hit * n->weight[cj * G + type];
                    events += hit;
                }
                s->counters[ORC_EVENTS] += events;
                int64_t u = (int64_t)s->potential[cj] + acc + n->leak[cj];
                if (u > vmax) u = vmax;
                if (u < vmin) u = vmin;
                if (u >= n->threshold[cj]) {
                    s->spiked[cj] = 1;
                    if (n->reset_mode && n->reset_mode[cj] == ORC_RESET_LINEAR) {
                        /* linear reset: keep what exceeded the threshold */
                        int64_t r = u - n->threshold[cj];
                        if (r > vmax) r = vmax;
                        if (r < vmin) r = vmin;
                        s->potential[cj] = (int32_t)r;
                    } else {
                        s->potential[cj] = n->reset[cj];
                    }
                    s->counters[ORC_EMITTED] += 1;
                } else {
                    /* below its floor a neuron that does not fire stops at the floor */
                    if (n->floor && u < n->floor[cj])
                        u = n->floor[cj];
                    s->spiked[cj] = 0;
                    s->potential[cj] = (int32_t)u;
                }
            }
        }
        /* Router. */
        for (int c = 0; c < C; ++c) {
            for (int j = 0; j < N; ++j) {
                size_t cj = (size_t)c * N + j;
                if (!s->spiked[cj])
                    continue;
                if (n->dest_kind[cj] == ORC_DEST_OUT) {
                    if (count < cap && out_events) {
                        out_events[3 * count + 0] = s->tick;
                        out_events[3 * count + 1] = c;
                        out_events[3 * count + 2] = j;
                    }
                    ++count;
                    s->counters[ORC_OUT] += 1;
                } else if (n->dest_kind[cj] == ORC_DEST_CORE) {
                    int dest = route_hops(n, c, n->dest_dx[cj], n->dest_dy[cj], &s->counters[ORC_HOPS], s->links);
                    if (dest < 0)
                        return ORC_EROUTE;
                    int row = (s->curr[dest] + n->dest_delay[cj]) % s->rows;
                    sram_row(s, dest, row)[n->dest_axon[cj]] = 1;
                    s->counters[ORC_ROUTED] += 1;
                }
            }
        }
        if (spike_trace)
            memcpy(spike_trace + (size_t)k * C * N, s->spiked, (size_t)C * N);
        if (v_trace)
            memcpy(v_trace + (size_t)k * C * N, s->potential, (size_t)C * N * sizeof(int32_t));
    }
    if (n_out)
        *n_out = count;
    return count > cap ? ORC_TRUNCATED : ORC_OK;
}

void orc_potentials(const orc_sim *s, int32_t *out)
{
    memcpy(out, s->potential, (size_t)s->net.num_cores * s->net.num_neurons * sizeof(int32_t));
}

void orc_counters(const orc_sim *s, int64_t *out)
{
    memcpy(out, s->counters, sizeof(s->counters));
}

/* Packets per mesh link since the start: out[c][d], d = +x, -x, +y, -y. */
void orc_links(const orc_sim *s, int64_t *out)
{
    memcpy(out, s->links, (size_t)s->net.num_cores * ORC_NLINKS * sizeof(int64_t));
}

int64_t orc_tick(const orc_sim *s)
{
    return s->tick;
}

int32_t orc_num_counters(void)
{
    return ORC_NCOUNTERS;
}
