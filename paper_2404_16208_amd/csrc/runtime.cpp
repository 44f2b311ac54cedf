// runtime.cpp -- host side of the C ABI declared in include/ranc.h.
//
// Validation of the network description, the workspace layout, host-side
// packing of the description into the device layouts of ranc_internal.h
// (crossbar columns, per-type masks, MFMA weight planes, the inverted routing
// table), the tick loop that queues the per-tick kernels (per launch or as a
// captured HIP graph), batches of several networks, the launch-shape
// autotuner, and readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ranc.h"
#include "ranc_internal.h"

using namespace ranc;

namespace {

thread_local std::string g_err;

ranc_status fail(ranc_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

ranc_status hip_fail(hipError_t e, const char *what)
{
    return fail(RANC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

enum Region {
    R_COLBITS, R_TYPEMASK, R_WTS, R_LEAK, R_THR, R_RST, R_VINIT, R_COREMASK, R_OUTMASK, R_OUTWORD,
    R_ININDEX, R_RTDCNT, R_RTGOFF, R_RTENT, R_DEGB, R_OUTIDX, R_PLANES, R_RTXPTR, R_RTXENT, R_HZERO,
    R_FLOOR, R_LINMASK, R_ECSRPTR, R_ECSRENT, R_LINKREC, R_OUTCOL, R_OUTPOS, R_LINKPTR, R_LINKENT,
    R_PARAMS_END,  // everything before this is uploaded once at load
    R_V = R_PARAMS_END, R_RING, R_SPK, R_HIST, R_RASTER, R_CNT, R_CRING, R_TICK, R_BATCH, R_EXT, R_LINKD,
    R_RSYNC,
    // MFMA path: the compact B source, uploaded at load as well; kept past
    // the state regions so that their placement does not depend on it
    R_BSRC, R_NREG
};

struct Plan {
    int C, A, N, G, W, NW, D, Q, S, S64, RT, Wout, Nout, Cin, path, two, spw;
    int bsrc;            // MFMA path B source: -1 by mfma_compact_b, 0 the planes, 1 the compact crossbar
    int grid_w, grid_h;  // mesh size
    int slices;          // MFMA and sparse: neuron slices per core (one workgroup each)
    int cnt_rows;        // counter rows per core
    long long E;         // routed (CORE) neurons
    long long ell_words; // u32 words of the wave-interleaved routing table
    long long ecsr_entries; // sparse path: row entries, each slice's rows padded to sparse_row_align()
    size_t off[R_NREG], size[R_NREG], params_bytes, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Batch tables (several networks advanced by one launch per tick) live in the
// workspace of the batch's first network: up to BATCH_MAX entries for the
// MFMA path, then up to BATCH_MAX for the plain path, then two queue counters.
constexpr int BATCH_MAX = 128;
constexpr size_t BATCH_TABLE_BYTES = 2 * BATCH_MAX * sizeof(BatchEntry) + 256;

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

ranc_status validate(const ranc_net_desc *d, int32_t S, int32_t RT, int32_t path)
{
    if (!d)
        return fail(RANC_EINVAL, "desc is NULL");
    if (d->abi_version != RANC_ABI_VERSION)
        return fail(RANC_EINVAL, "abi_version %u != %u", d->abi_version, RANC_ABI_VERSION);
    if (S < 1)
        return fail(RANC_EINVAL, "num_samples must be >= 1 (got %d)", S);
    if (S > 65535)
        return fail(RANC_EUNSUPPORTED, "num_samples must be <= 65535 (got %d)", S);
    if (RT < 1)
        return fail(RANC_EINVAL, "max_ticks_per_call must be >= 1 (got %d)", RT);
    if (path < RANC_PATH_AUTO || path > RANC_PATH_SPARSE)
        return fail(RANC_EINVAL, "unknown path %d", path);
    if (d->num_cores < 1)
        return fail(RANC_EINVAL, "num_cores must be >= 1");
    if (d->grid_w < 1 || d->grid_h < 1 || (long long)d->grid_w * d->grid_h != d->num_cores)
        return fail(RANC_EINVAL, "grid %dx%d does not hold %d cores", d->grid_w, d->grid_h, d->num_cores);
    if (!pow2_in(d->num_axons, 64, 512))
        return fail(RANC_EUNSUPPORTED, "num_axons must be 64, 128, 256 or 512 (got %d)", d->num_axons);
    if (!pow2_in(d->num_neurons, 64, 512))
        return fail(RANC_EUNSUPPORTED, "num_neurons must be 64, 128, 256 or 512 (got %d)", d->num_neurons);
    if (!pow2_in(d->num_types, 1, 8))
        return fail(RANC_EUNSUPPORTED, "num_types must be 1, 2, 4 or 8 (got %d)", d->num_types);
    if (d->weight_bits < 2 || d->weight_bits > 9)
        return fail(RANC_ERANGE, "weight_bits must be in [2, 9] (got %d)", d->weight_bits);
    if (d->potential_bits < 2 || d->potential_bits > 32)
        return fail(RANC_ERANGE, "potential_bits must be in [2, 32] (got %d)", d->potential_bits);
    if (d->max_delay < 1 || d->max_delay > 15)
        return fail(RANC_ERANGE, "max_delay must be in [1, 15] (got %d)", d->max_delay);
    if ((long long)d->num_cores * d->num_neurons > RT_MAX_NEURONS)
        return fail(RANC_EUNSUPPORTED, "num_cores * num_neurons must be <= 2^23");
    if (!d->crossbar || !d->axon_type || !d->weight || !d->leak || !d->threshold || !d->reset ||
        !d->v_init || !d->dest_kind || !d->dest_dx || !d->dest_dy || !d->dest_axon || !d->dest_delay)
        return fail(RANC_EINVAL, "a parameter array pointer is NULL");
    if (d->num_input_cores < 0 || d->num_input_cores > d->num_cores)
        return fail(RANC_EINVAL, "num_input_cores out of range (%d)", d->num_input_cores);
    if (d->num_input_cores > 0 && !d->input_cores)
        return fail(RANC_EINVAL, "input_cores is NULL");
    const int C = d->num_cores, A = d->num_axons, N = d->num_neurons, G = d->num_types;
    for (size_t i = 0; i < (size_t)C * A; ++i)
        if (d->axon_type[i] >= G)
            return fail(RANC_ERANGE, "axon_type[%zu] = %u is not < num_types", i, d->axon_type[i]);
    const int wlo = -(1 << (d->weight_bits - 1)), whi = (1 << (d->weight_bits - 1)) - 1;
    for (size_t i = 0; i < (size_t)C * N * G; ++i)
        if (d->weight[i] < wlo || d->weight[i] > whi)
            return fail(RANC_ERANGE, "weight[%zu] = %d outside %d-bit range", i, d->weight[i], d->weight_bits);
    const int leak_bits = d->leak_bits ? d->leak_bits : 32, reset_bits = d->reset_bits ? d->reset_bits : 32;
    if (leak_bits < 2 || leak_bits > 32)
        return fail(RANC_ERANGE, "leak_bits must be 0 or in [2, 32] (got %d)", d->leak_bits);
    if (reset_bits < 2 || reset_bits > 32)
        return fail(RANC_ERANGE, "reset_bits must be 0 or in [2, 32] (got %d)", d->reset_bits);
    const long long vlo = -(1LL << (d->potential_bits - 1)), vhi = (1LL << (d->potential_bits - 1)) - 1;
    const long long llo = -(1LL << (leak_bits - 1)), lhi = (1LL << (leak_bits - 1)) - 1;
    const long long rlo = std::max(vlo, -(1LL << (reset_bits - 1))), rhi = std::min(vhi, (1LL << (reset_bits - 1)) - 1);
    for (size_t i = 0; i < (size_t)C * N; ++i) {
        if (d->reset[i] < rlo || d->reset[i] > rhi)
            return fail(RANC_ERANGE, "reset[%zu] = %d outside the potential range and the %d-bit reset range", i,
                        d->reset[i], reset_bits);
        if (d->v_init[i] < vlo || d->v_init[i] > vhi)
            return fail(RANC_ERANGE, "v_init[%zu] = %d outside the potential range", i, d->v_init[i]);
        if (d->leak[i] < llo || d->leak[i] > lhi)
            return fail(RANC_ERANGE, "leak[%zu] = %d outside the %d-bit leak range", i, d->leak[i], leak_bits);
        if (d->leak[i] < -(1 << 30) || d->leak[i] > (1 << 30))
            return fail(RANC_ERANGE, "leak[%zu] = %d outside [-2^30, 2^30]", i, d->leak[i]);
        if (d->floor && (d->floor[i] < vlo || d->floor[i] > vhi))
            return fail(RANC_ERANGE, "floor[%zu] = %d outside the potential range", i, d->floor[i]);
        if (d->reset_mode && d->reset_mode[i] > RANC_RESET_LINEAR)
            return fail(RANC_EINVAL, "reset_mode[%zu] = %u unknown", i, d->reset_mode[i]);
        const uint8_t k = d->dest_kind[i];
        if (k > RANC_DEST_OUT)
            return fail(RANC_EINVAL, "dest_kind[%zu] = %u unknown", i, k);
        if (k == RANC_DEST_CORE) {
            const int c = (int)(i / N);
            const long long x = c % d->grid_w + (long long)d->dest_dx[i];
            const long long y = c / d->grid_w + (long long)d->dest_dy[i];
            if (x < 0 || x >= d->grid_w || y < 0 || y >= d->grid_h)
                return fail(RANC_ERANGE, "neuron %zu: destination (%+d, %+d) leaves the %dx%d mesh", i,
                            d->dest_dx[i], d->dest_dy[i], d->grid_w, d->grid_h);
            if (d->dest_axon[i] >= A)
                return fail(RANC_ERANGE, "neuron %zu: dest_axon %u >= num_axons", i, d->dest_axon[i]);
            if (d->dest_delay[i] < 1 || d->dest_delay[i] > d->max_delay)
                return fail(RANC_ERANGE, "neuron %zu: dest_delay %u outside [1, %d]", i, d->dest_delay[i],
                            d->max_delay);
        }
    }
    std::vector<char> seen(C, 0);
    for (int i = 0; i < d->num_input_cores; ++i) {
        const int c = d->input_cores[i];
        if (c < 0 || c >= C)
            return fail(RANC_ERANGE, "input_cores[%d] = %d out of range", i, c);
        if (seen[c])
            return fail(RANC_EINVAL, "input core %d listed twice", c);
        seen[c] = 1;
    }
    return RANC_OK;
}

// Whether the network needs the extended potential update: potentials
// narrower than 32 bits (clamp), a floor above the potential range's lowest
// value, or linear-reset neurons.
bool neuron_model_ext(const ranc_net_desc *d)
{
    if (d->potential_bits < 32)
        return true;
    const size_t CN = (size_t)d->num_cores * d->num_neurons;
    const int32_t vmin = (int32_t)(-(1LL << (d->potential_bits - 1)));
    for (size_t i = 0; i < CN; ++i)
        if ((d->floor && d->floor[i] > vmin) || (d->reset_mode && d->reset_mode[i] == RANC_RESET_LINEAR))
            return true;
    return false;
}

ranc_status make_plan(const ranc_net_desc *d, int32_t S, int32_t RT, int32_t path, Plan &p)
{
    ranc_status st = validate(d, S, RT, path);
    if (st != RANC_OK)
        return st;
    p.C = d->num_cores;
    p.A = d->num_axons;
    p.N = d->num_neurons;
    p.G = d->num_types;
    p.W = p.A / 32;
    p.NW = p.N / 32;
    p.D = d->max_delay;
    p.Q = p.D + 1;
    p.S = S;
    p.S64 = (S + 63) / 64 * 64;
    p.RT = RT;
    p.Cin = d->num_input_cores;
    p.grid_w = d->grid_w;
    p.grid_h = d->grid_h;
    p.two = d->weight_bits > 8;
    if (path == RANC_PATH_AUTO)
        path = (S >= 64 && mfma_shape_supported(p.A, p.N, p.two)) ? RANC_PATH_MFMA : RANC_PATH_PLAIN;
    if (path == RANC_PATH_MFMA && !mfma_shape_supported(p.A, p.N, p.two))
        return fail(RANC_EUNSUPPORTED, "MFMA path does not support A=%d N=%d with %d-bit weights", p.A, p.N,
                    d->weight_bits);
    if (path == RANC_PATH_SPARSE && !sparse_shape_supported(p.A, p.N, p.G))
        return fail(RANC_EUNSUPPORTED, "sparse path does not support N=%d with G=%d", p.N, p.G);
    p.path = path;
    p.slices = path == RANC_PATH_MFMA ? mfma_slices(p.A, p.N, p.two)
             : path == RANC_PATH_SPARSE ? p.N / sparse_slice_width(p.N) : 1;
    p.cnt_rows = path == RANC_PATH_PLAIN ? p.N / 64 : p.slices;
    // Samples per workgroup (sample-tiled paths), in 64-sample tiles: aim for
    // >= 2048 workgroups, but keep >= 4 tiles per workgroup where the batch
    // has them (the software pipeline runs over a workgroup's tiles). On the
    // 512-core net at 1024 samples: 256 -> 232.8 us per tick, 512 -> 235.5,
    // 128 -> 263.2.
    {
        const int tiles = (S + 63) / 64;
        const int per_chunk = p.C * p.slices;   // workgroups per sample chunk
        int chunks = (2048 + per_chunk - 1) / per_chunk;
        chunks = std::max(1, std::min(chunks, std::max(1, tiles / 4)));
        const int tiles_per = (tiles + chunks - 1) / chunks;
        const int cap = path == RANC_PATH_SPARSE ? sparse_max_samples_per_wg() : mfma_max_samples_per_wg();
        p.spw = std::min(64 * tiles_per, std::min(cap, 512));
        if (const char *e = getenv("RANC_MFMA_SPW")) {
            const int v = atoi(e);
            if (v > 0 && v % 64 == 0 && v <= cap)
                p.spw = v;
        }
    }
    p.bsrc = -1;
    if (const char *e = getenv("RANC_MFMA_BSRC"))
        p.bsrc = strcmp(e, "planes") == 0 ? 0 : strcmp(e, "compact") == 0 ? 1 : -1;
    long long E = 0, wout = 0, nout = 0;
    for (size_t i = 0; i < (size_t)p.C * p.N; ++i) {
        E += d->dest_kind[i] == RANC_DEST_CORE;
        nout += d->dest_kind[i] == RANC_DEST_OUT;
    }
    {
        // wave-interleaved table: every group of 64 destination words is padded
        // to its longest list
        const size_t CW = (size_t)p.C * p.W;
        std::vector<uint32_t> cnt(CW, 0);
        for (size_t i = 0; i < (size_t)p.C * p.N; ++i)
            if (d->dest_kind[i] == RANC_DEST_CORE) {
                const int c = (int)(i / p.N);
                const int dc = (c % d->grid_w + d->dest_dx[i]) + (c / d->grid_w + d->dest_dy[i]) * d->grid_w;
                ++cnt[(size_t)dc * p.W + d->dest_axon[i] / 32];
            }
        long long words = 0;
        for (size_t g = 0; g < (CW + 63) / 64; ++g) {
            uint32_t mx = 0;
            for (size_t k = g * 64; k < std::min(CW, g * 64 + 64); ++k)
                mx = std::max(mx, cnt[k]);
            words += 64LL * mx;
        }
        p.ell_words = words;
    }
    for (int c = 0; c < p.C; ++c)
        for (int w = 0; w < p.NW; ++w) {
            bool any = false;
            for (int b = 0; b < 32; ++b)
                any |= d->dest_kind[(size_t)c * p.N + 32 * w + b] == RANC_DEST_OUT;
            wout += any;
        }
    p.ecsr_entries = 0;
    if (path == RANC_PATH_SPARSE) {
        // connections per neuron slice, each slice's rows padded
        const int NW = p.N / 32, SW = sparse_slice_width(p.N) / 32, al = sparse_row_align();
        for (int c = 0; c < p.C; ++c)
            for (int sl = 0; sl < p.slices; ++sl) {
                long long k = 0;
                for (int a = 0; a < p.A; ++a)
                    for (int w = sl * SW; w < (sl + 1) * SW; ++w)
                        k += __builtin_popcount(d->crossbar[((size_t)c * p.A + a) * NW + w]);
                p.ecsr_entries += (k + al - 1) / al * al;
            }
    }
    p.E = E;
    p.Wout = (int)wout;
    p.Nout = (int)nout;
    const size_t C = p.C, A = p.A, N = p.N, G = p.G, W = p.W, NW = p.NW;
    const bool mf = p.path == RANC_PATH_MFMA;
    const bool sp = p.path == RANC_PATH_SPARSE;
    const bool tiled = mf || sp;   // sample-tiled paths: spike history, neuron-major raster
    p.size[R_COLBITS] = tiled ? 0 : C * W * N * 4;
    // MFMA path: crossbar column words, then the per-type plane bytes of
    // every neuron, then the axon types (the compact source its kernels build
    // B tiles from; see pack_bsrc)
    p.size[R_BSRC] = mf ? C * W * N * 4 + C * (p.two ? 2 : 1) * 2 * N * 4 + C * A : 0;
    p.size[R_TYPEMASK] = C * G * W * 4;
    p.size[R_WTS] = C * G * N * 4;
    p.size[R_LEAK] = p.size[R_THR] = p.size[R_RST] = p.size[R_VINIT] = p.size[R_FLOOR] = C * N * 4;
    p.size[R_LINMASK] = C * NW * 4;
    p.size[R_ECSRPTR] = sp ? C * p.slices * (A + 1) * 4 : 0;
    p.size[R_ECSRENT] = sp ? std::max<size_t>((size_t)p.ecsr_entries, 8) * 2 : 0;
    p.size[R_COREMASK] = p.size[R_OUTMASK] = p.size[R_OUTWORD] = C * NW * 4;
    p.size[R_ININDEX] = C * 4;
    p.size[R_RTDCNT] = tiled ? 0 : (C * W + 63) / 64 * 64 * route_dmax(p.D) * 2;
    p.size[R_RTGOFF] = tiled ? 0 : (C * W + 63) / 64 * 4;
    p.size[R_RTENT] = tiled ? 0 : std::max<size_t>((size_t)p.ell_words, 1) * 4;
    p.size[R_RTXPTR] = tiled ? (C * A + 1) * 4 : 0;
    p.size[R_RTXENT] = tiled ? std::max<size_t>((size_t)E, 1) * 4 : 0;
    const size_t HG = (size_t)p.S64 / 64;
    p.size[R_HZERO] = tiled ? HG * 8 : 0;
    p.size[R_DEGB] = mf ? C * p.slices * 2 * A : 0;
    p.size[R_OUTIDX] = tiled ? C * N * 4 : 0;
    // int8 weight planes: the B source when a core's samples take several
    // workgroups, of the persistent batch kernel and of the state-resident
    // kernel (otherwise B is built from R_BSRC)
    p.size[R_PLANES] = mf ? C * A * N * (p.two ? 2 : 1) : 0;
    p.size[R_V] = C * (tiled ? (size_t)p.S64 : (size_t)S) * N * 4;
    // plain path: the scheduler ring; sparse path: the scheduler row of the
    // tick being integrated, [C][S64][W], written by the delivery kernel
    p.size[R_RING] = mf ? 0 : sp ? C * (size_t)p.S64 * W * 4 : (size_t)p.Q * S * C * W * 4;
    p.size[R_SPK] = tiled ? 0 : (size_t)S * C * NW * 4;
    p.size[R_HIST] = tiled ? (size_t)p.Q * C * N * HG * 8 : 0;
    p.size[R_RASTER] = tiled ? (size_t)RT * p.Nout * HG * 8 : (size_t)RT * S * p.Wout * 4;
    p.size[R_CNT] = C * p.cnt_rows * S * CNT_N * 8;   // plain: one row per 64 neurons, MFMA and sparse: per slice
    p.size[R_CRING] = (size_t)RT * C * p.cnt_rows * S * 8;   // one packed word per row, sample and tick of a call
    p.size[R_TICK] = 16;
    p.size[R_BATCH] = BATCH_TABLE_BYTES;
    p.size[R_EXT] = (size_t)RT * S * p.Cin * W * 4;
    p.size[R_LINKREC] = C * N * 8;
    // sample-tiled paths: for every (direction, core) difference-array row,
    // the run starts (+1) and ends (-1) that land there, by source neuron
    p.size[R_LINKPTR] = tiled ? (size_t)(4 * C + 1) * 4 : 0;
    p.size[R_LINKENT] = tiled ? std::max<size_t>((size_t)4 * E, 1) * 4 : 0;
    p.size[R_OUTCOL] = tiled ? 0 : std::max<size_t>((size_t)p.Wout, 1) * 8;
    p.size[R_OUTPOS] = tiled ? 0 : std::max<size_t>((size_t)p.Nout, 1) * 4;
    p.size[R_LINKD] = (size_t)4 * C * p.S64 * 8;
    p.size[R_RSYNC] = mf ? 8 : 0;   // state-resident loop: arrival counter, give-up flag
    size_t off = 0;
    for (int r = 0; r < R_NREG; ++r) {
        if (r == R_PARAMS_END)
            p.params_bytes = off;
        p.off[r] = off;
        off += align256(p.size[r]);
    }
    p.total = off;
    return RANC_OK;
}

// Crossbar columns [C][A/32][N] (bit a % 32 of word a / 32 of neuron j: axon
// a connects to j), into zeroed words, visiting the set crossbar bits only.
static void pack_columns(const ranc_net_desc *d, const Plan &p, uint32_t *col)
{
    const int C = p.C, A = p.A, N = p.N, W = p.W, NW = p.NW;
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < A; ++a) {
            const uint32_t *row = d->crossbar + ((size_t)c * A + a) * NW;
            uint32_t *cw = col + ((size_t)c * W + a / 32) * N;
            const uint32_t bit = 1u << (a % 32);
            for (int w = 0; w < NW; ++w)
                for (uint32_t b = row[w]; b; b &= b - 1u)
                    cw[32 * w + __builtin_ctz(b)] |= bit;
        }
}

// Host-side packing of the MFMA path's compact B source (R_BSRC): column
// words [C][W][N] (bit a % 32 of word a / 32 of neuron j: axon a connects to
// j); then [C][planes][2][N] words, byte g % 4 of word g / 4 = the plane
// value of weight(j, g) (two planes: w >> 7, then w & 127; one: w); then the
// axon types [C][A], one byte each.
void pack_bsrc(const ranc_net_desc *d, const Plan &p, std::vector<uint8_t> &buf)
{
    buf.assign(p.size[R_BSRC], 0);
    const int C = p.C, A = p.A, N = p.N, G = p.G, W = p.W, PL = p.two ? 2 : 1;
    uint32_t *col = reinterpret_cast<uint32_t *>(buf.data());
    pack_columns(d, p, col);
    uint32_t *ws = col + (size_t)C * W * N;
    for (int c = 0; c < C; ++c)
        for (int j = 0; j < N; ++j)
            for (int g = 0; g < G; ++g) {
                const int w = d->weight[((size_t)c * N + j) * G + g];
                for (int pl = 0; pl < PL; ++pl) {
                    const uint32_t v = (uint32_t)(PL == 2 ? (pl == 0 ? w >> 7 : w & 127) : w) & 255u;
                    ws[(((size_t)c * PL + pl) * 2 + g / 4) * N + j] |= v << (8 * (g % 4));
                }
            }
    memcpy(reinterpret_cast<uint8_t *>(ws + (size_t)C * PL * 2 * N), d->axon_type, (size_t)C * A);
}

// Host-side packing of the parameter region (bytes [0, params_bytes)).
void pack_params(const ranc_net_desc *d, const Plan &p, std::vector<uint8_t> &buf, std::vector<int> &out_words)
{
    buf.assign(p.params_bytes, 0);
    auto at = [&](Region r) { return buf.data() + p.off[r]; };
    const int C = p.C, A = p.A, N = p.N, G = p.G, W = p.W, NW = p.NW;
    auto conn = [&](int c, int a, int j) -> int {
        return (d->crossbar[((size_t)c * A + a) * NW + j / 32] >> (j % 32)) & 1u;
    };
    if (p.size[R_COLBITS])
        pack_columns(d, p, (uint32_t *)at(R_COLBITS));
    uint32_t *tm = (uint32_t *)at(R_TYPEMASK);
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < A; ++a)
            tm[((size_t)c * G + d->axon_type[(size_t)c * A + a]) * W + a / 32] |= 1u << (a % 32);
    int32_t *wts = (int32_t *)at(R_WTS);
    for (int c = 0; c < C; ++c)
        for (int g = 0; g < G; ++g)
            for (int j = 0; j < N; ++j)
                wts[((size_t)c * G + g) * N + j] = d->weight[((size_t)c * N + j) * G + g];
    memcpy(at(R_LEAK), d->leak, (size_t)C * N * 4);
    memcpy(at(R_THR), d->threshold, (size_t)C * N * 4);
    memcpy(at(R_RST), d->reset, (size_t)C * N * 4);
    memcpy(at(R_VINIT), d->v_init, (size_t)C * N * 4);
    // floor: the lowest potential of the range where none is given (a no-op
    // after the clamp); linear-reset neurons as one bit per neuron
    int32_t *fl = (int32_t *)at(R_FLOOR);
    const int32_t vmin = (int32_t)(-(1LL << (d->potential_bits - 1)));
    for (size_t i = 0; i < (size_t)C * N; ++i)
        fl[i] = d->floor ? std::max(d->floor[i], vmin) : vmin;
    uint32_t *lin = (uint32_t *)at(R_LINMASK);
    if (d->reset_mode)
        for (size_t i = 0; i < (size_t)C * N; ++i)
            lin[i / 32] |= (uint32_t)(d->reset_mode[i] == RANC_RESET_LINEAR) << (i % 32);
    uint32_t *cmask = (uint32_t *)at(R_COREMASK), *omask = (uint32_t *)at(R_OUTMASK);
    int32_t *oword = (int32_t *)at(R_OUTWORD);
    out_words.clear();
    for (int c = 0; c < C; ++c)
        for (int w = 0; w < NW; ++w) {
            uint32_t cm = 0, om = 0;
            for (int b = 0; b < 32; ++b) {
                const uint8_t k = d->dest_kind[(size_t)c * N + 32 * w + b];
                cm |= (uint32_t)(k == RANC_DEST_CORE) << b;
                om |= (uint32_t)(k == RANC_DEST_OUT) << b;
            }
            cmask[(size_t)c * NW + w] = cm;
            omask[(size_t)c * NW + w] = om;
            oword[(size_t)c * NW + w] = om ? (int32_t)(out_words.size() / 2) : -1;
            if (om) {
                out_words.push_back(c);
                out_words.push_back(w);
            }
        }
    if (p.size[R_OUTCOL]) {
        // plain-path raster columns: neuron word and the output index of its
        // first output neuron (output neurons numbered in (core, neuron) order)
        int32_t *oc = (int32_t *)at(R_OUTCOL);
        int base = 0;
        for (size_t ow = 0; ow < out_words.size() / 2; ++ow) {
            const int c = out_words[2 * ow], w = out_words[2 * ow + 1];
            oc[2 * ow] = c * NW + w;
            oc[2 * ow + 1] = base;
            base += __builtin_popcount(omask[(size_t)c * NW + w]);
        }
        int32_t *op = (int32_t *)at(R_OUTPOS);
        int o = 0;
        for (size_t ow = 0; ow < out_words.size() / 2; ++ow) {
            const int c = out_words[2 * ow], w = out_words[2 * ow + 1];
            for (uint32_t m = omask[(size_t)c * NW + w]; m; m &= m - 1u)
                op[o++] = (int32_t)(ow << 5) | __builtin_ctz(m);
        }
    }
    int32_t *inidx = (int32_t *)at(R_ININDEX);
    for (int c = 0; c < C; ++c)
        inidx[c] = -1;
    for (int i = 0; i < p.Cin; ++i)
        inidx[d->input_cores[i]] = i;
    // Inverted routing table, one list per destination axon word, sorted by
    // delay, stored wave-interleaved (see ranc_internal.h).
    if (p.size[R_RTENT]) {
        const size_t CW = (size_t)C * W;
        std::vector<std::vector<uint32_t>> lists(CW);
        for (size_t i = 0; i < (size_t)C * N; ++i)
            if (d->dest_kind[i] == RANC_DEST_CORE) {
                const int c = (int)(i / N);
                const int dc = (c % d->grid_w + d->dest_dx[i]) + (c / d->grid_w + d->dest_dy[i]) * d->grid_w;
                const uint32_t ent = ((uint32_t)i << RT_SRC_SHIFT) |
                                     ((uint32_t)(d->dest_delay[i] - 1) << RT_DELAY_SHIFT) | (d->dest_axon[i] % 32u);
                lists[(size_t)dc * W + d->dest_axon[i] / 32].push_back(ent);
            }
        const int dmax = route_dmax(p.D);
        uint16_t *dcnt = (uint16_t *)at(R_RTDCNT);
        uint32_t *goff = (uint32_t *)at(R_RTGOFF), *ent = (uint32_t *)at(R_RTENT);
        size_t off = 0;
        for (size_t g = 0; g < (CW + 63) / 64; ++g) {
            size_t mx = 0;
            for (size_t k = g * 64; k < std::min(CW, g * 64 + 64); ++k) {
                auto &L = lists[k];
                std::stable_sort(L.begin(), L.end(), [](uint32_t a, uint32_t b) {
                    return ((a >> RT_DELAY_SHIFT) & 15u) < ((b >> RT_DELAY_SHIFT) & 15u);
                });
                for (uint32_t x : L)
                    ++dcnt[k * dmax + ((x >> RT_DELAY_SHIFT) & 15u)];
                mx = std::max(mx, L.size());
                for (size_t e = 0; e < L.size(); ++e)
                    ent[off + e * 64 + (k - g * 64)] = L[e];
            }
            goff[g] = (uint32_t)off;
            off += 64 * mx;
        }
    }
    // MFMA path: the inverted table keyed by destination axon (CSR).
    if (p.size[R_RTXPTR]) {
        uint32_t *ptr = (uint32_t *)at(R_RTXPTR), *ent = (uint32_t *)at(R_RTXENT);
        const size_t CA = (size_t)C * A;
        std::vector<uint32_t> fill(CA + 1, 0);
        auto dest_of = [&](size_t i) -> size_t {
            const int c = (int)(i / N);
            const int dc = (c % d->grid_w + d->dest_dx[i]) + (c / d->grid_w + d->dest_dy[i]) * d->grid_w;
            return (size_t)dc * A + d->dest_axon[i];
        };
        for (size_t i = 0; i < (size_t)C * N; ++i)
            if (d->dest_kind[i] == RANC_DEST_CORE)
                ++fill[dest_of(i) + 1];
        for (size_t k = 0; k < CA; ++k)
            fill[k + 1] += fill[k];
        memcpy(ptr, fill.data(), (CA + 1) * 4);
        for (size_t i = 0; i < (size_t)C * N; ++i)
            if (d->dest_kind[i] == RANC_DEST_CORE)
                ent[fill[dest_of(i)]++] = ((uint32_t)i << 4) | (uint32_t)(d->dest_delay[i] - 1);
    }
    if (p.size[R_ECSRPTR]) {
        // Sparse path: per (core, neuron slice) one row per axon, listing the
        // slice's connected neurons with their weight for the axon's type:
        // entry = neuron within the slice (7 bits) | weight (9 bits) << 7.
        // Row starts are absolute; each slice's rows start on a multiple of
        // sparse_row_align() entries (the padding entries are never read as
        // connections).
        uint32_t *ptr = (uint32_t *)at(R_ECSRPTR);
        uint16_t *ent = (uint16_t *)at(R_ECSRENT);
        const int NS = sparse_slice_width(N), al = sparse_row_align();
        uint32_t off = 0;
        for (int c = 0; c < C; ++c)
            for (int sl = 0; sl < p.slices; ++sl) {
                uint32_t *rp = ptr + ((size_t)c * p.slices + sl) * (A + 1);
                for (int a = 0; a < A; ++a) {
                    rp[a] = off;
                    const int g = d->axon_type[(size_t)c * A + a];
                    for (int jl = 0; jl < NS; ++jl) {
                        const int j = sl * NS + jl;
                        if (conn(c, a, j)) {
                            const int w = d->weight[((size_t)c * N + j) * G + g];
                            ent[off++] = (uint16_t)(jl | ((w & 511) << 7));
                        }
                    }
                }
                rp[A] = off;
                off = (off + al - 1) / al * al;
            }
    }
    if (p.size[R_DEGB]) {
        // connected neurons per axon within each neuron slice, as a low-byte
        // and a high-byte plane: [C][slices][2][A]
        uint8_t *db = at(R_DEGB);
        const int SL = p.slices, WS = NW / SL;
        for (int c = 0; c < C; ++c)
            for (int sl = 0; sl < SL; ++sl)
                for (int a = 0; a < A; ++a) {
                    int k = 0;
                    for (int w = sl * WS; w < (sl + 1) * WS; ++w)
                        k += __builtin_popcount(d->crossbar[((size_t)c * A + a) * NW + w]);
                    const size_t r = (size_t)c * SL + sl;
                    db[(r * 2 + 0) * A + a] = (uint8_t)(k & 255);
                    db[(r * 2 + 1) * A + a] = (uint8_t)(k >> 8);
                }
    }
    {
        // mesh path ends of each neuron's packets (x first, then y; see
        // kern_links.hip): no hop is -1, else 2 * end core + (negative step)
        int32_t *lr = (int32_t *)at(R_LINKREC);
        for (size_t i = 0; i < (size_t)C * N; ++i) {
            int32_t xc = -1, yc = -1;
            if (d->dest_kind[i] == RANC_DEST_CORE) {
                const int c = (int)(i / N), gw = d->grid_w;
                const int xs = c % gw, ys = c / gw, dx = d->dest_dx[i], dy = d->dest_dy[i];
                const int xd = xs + dx, yd = ys + dy;
                if (dx != 0)
                    xc = 2 * (ys * gw + xd) + (dx < 0);
                if (dy != 0)
                    yc = 2 * (yd * gw + xd) + (dy < 0);
            }
            lr[2 * i] = xc;
            lr[2 * i + 1] = yc;
        }
        if (p.size[R_LINKPTR]) {
            // rows of the difference arrays ([direction][core], direction
            // 0 +x, 1 -x, 2 +y, 3 -y) and the entries each packet adds to
            // them: +1 where a run of links starts, -1 where it ends; entry =
            // source neuron << 1 | (1 for -1), by source neuron within a row
            uint32_t *tp = (uint32_t *)at(R_LINKPTR);
            uint32_t *te = (uint32_t *)at(R_LINKENT);
            std::fill(tp, tp + 4 * (size_t)C + 1, 0u);
            auto visit = [&](auto &&emit) {
                for (size_t i = 0; i < (size_t)C * N; ++i) {
                    const int32_t xc = lr[2 * i], yc = lr[2 * i + 1];
                    const int c = (int)(i / N);
                    if (xc >= 0) {
                        emit((xc & 1) * C + c, i, 0u);
                        emit((xc & 1) * C + (xc >> 1), i, 1u);
                    }
                    if (yc >= 0) {
                        const int dir = 2 + (yc & 1);
                        emit(dir * C + (xc >= 0 ? xc >> 1 : c), i, 0u);
                        emit(dir * C + (yc >> 1), i, 1u);
                    }
                }
            };
            visit([&](int row, size_t, uint32_t) { ++tp[row + 1]; });
            for (size_t r = 0; r < 4 * (size_t)C; ++r)
                tp[r + 1] += tp[r];
            std::vector<uint32_t> fill(tp, tp + 4 * (size_t)C);
            visit([&](int row, size_t g, uint32_t neg) { te[fill[row]++] = (uint32_t)g << 1 | neg; });
        }
    }
    if (p.size[R_OUTIDX]) {
        int32_t *oi = (int32_t *)at(R_OUTIDX);
        int32_t next = 0;
        for (size_t i = 0; i < (size_t)C * N; ++i)
            oi[i] = d->dest_kind[i] == RANC_DEST_OUT ? next++ : -1;
    }
    if (p.size[R_PLANES]) {
        // B tiles: [C][N/32][A/32][planes][64 lanes][16 bytes]; lane l, byte b of
        // k-step k covers axon 32k + 16(l/32) + b and neuron 32nb + l%32.
        // Two planes: hi = w >> 7 (floor(w / 128)) first, then lo = w & 127.
        int8_t *pl = (int8_t *)at(R_PLANES);
        const int NB = N / 32, KS = A / 32, PL = p.two ? 2 : 1;
        for (int c = 0; c < C; ++c)
            for (int nb = 0; nb < NB; ++nb)
                for (int k = 0; k < KS; ++k)
                    for (int l = 0; l < 64; ++l)
                        for (int b = 0; b < 16; ++b) {
                            const int a = 32 * k + 16 * (l / 32) + b, j = 32 * nb + l % 32;
                            const int w = conn(c, a, j) ? d->weight[((size_t)c * N + j) * G +
                                                                    d->axon_type[(size_t)c * A + a]]
                                                        : 0;
                            const size_t base = ((((size_t)c * NB + nb) * KS + k) * PL) * 1024 + (size_t)l * 16 + b;
                            if (PL == 2) {
                                pl[base] = (int8_t)(w >> 7);
                                pl[base + 1024] = (int8_t)(w & 127);
                            } else {
                                pl[base] = (int8_t)w;
                            }
                        }
    }
}

}  // namespace

struct EventPair {
    hipEvent_t a, b;
};

struct Profiler {
    bool on = false;
    std::vector<EventPair> pool;          // created on demand, reused
    std::vector<std::pair<int, int>> used; // (pool index, kind 0=integrate 1=route 2=graph 3=resident)
    double ms[4] = {0, 0, 0, 0};           // kind 3: state-resident launches
    int64_t launches[4] = {0, 0, 0, 0};
};

// A captured tick loop: num_ticks ticks reading inputs at `base`. A handle
// keeps at most MAX_CAPTURED_LOOPS of them and drops the least recently
// replayed one to capture a new one (callers that cycle through many input
// buffers would otherwise hold one graph per address forever).
struct CapturedLoop {
    int num_ticks;
    const uint32_t *base;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t used;   // replay counter of the handle at the last replay
};
constexpr size_t MAX_CAPTURED_LOOPS = 16;

// A batch of networks run together, as last set up by ranc_run_ticks with
// this handle first; its tables are in this handle's workspace.
struct Batch {
    std::vector<ranc_net *> nets;
    std::vector<uint64_t> uids;   // identity of the networks (a freed handle's address may be reused)
    std::vector<const uint32_t *> bases;
    int num_ticks = 0;
    std::vector<BatchEntry> mf, pl;
    // MFMA shape classes (one launch each per tick), unless persistent
    struct Group { int first, num, units, code, ext, compact; MfmaGroupArgs args; };
    std::vector<Group> groups;
    // Phases: networks whose combined per-tick state fits the GPU's last-level
    // cache; all ticks of a phase run before the next phase starts. Groups
    // [g_first, g_first + g_num) and plain entries [pl_first, pl_first +
    // pl_num), numbered from 0 within the phase. One phase when persistent.
    struct Phase { int g_first, g_num, pl_first, pl_num, pl_units, rt_units; };
    std::vector<Phase> phases;
    std::vector<std::vector<int>> phase_links;   // per phase: networks (index in nets) counting mesh links
    std::vector<char> links;                     // links_on of each network when the batch was set up
    bool persistent = false;
    int mf_units = 0, pl_units = 0, rt_units = 0, mf_workgroups = 0;
    size_t rt_lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct ranc_net {
    Plan p;
    uint64_t uid = 0;   // unique per loaded handle
    Batch batch;
    std::vector<CapturedLoop> loops;
    uint64_t replays = 0;              // captured-loop replays (recency of the cached loops)
    uint64_t loops_dropped = 0;        // captured loops dropped to respect MAX_CAPTURED_LOOPS
    hipStream_t cap_stream = nullptr;  // private stream used only for capture
    // batches led by this handle: streams on which the shape classes' tick
    // chains run side by side, and the fork and join events
    static constexpr int BATCH_BRANCHES = 4;
    hipStream_t br_stream[BATCH_BRANCHES] = {};
    hipEvent_t br_fork = nullptr, br_join[BATCH_BRANCHES] = {};
    RouteCfg rcfg;
    Profiler prof;
    DevNet dn;
    uint8_t *ws;
    hipStream_t last_stream;
    int64_t tick;
    uint64_t version, raster_version;
    std::vector<int> out_words;        // (core, word) pairs of raster columns (plain path)
    std::vector<int> out_neurons;      // (core, neuron) of each output-bus neuron, in index order
    std::vector<uint32_t> raster_host; // mirror of the raster
    uint64_t v_version = 0;
    std::vector<int32_t> v_host;       // mirror of the potentials
    uint64_t cnt_version = 0;
    std::vector<unsigned long long> cnt_host; // mirror of the counters
    LinkArgs lk{nullptr, nullptr, nullptr, nullptr}; // mesh link path ends, rows and counts in the workspace
    const int2 *outcol = nullptr;      // plain path: raster columns (kern_raster.hip)
    const int32_t *opos = nullptr;     // plain path: raster position of each output neuron
    bool links_on = false;             // count packets per mesh link on every tick run
    uint64_t links_version = 0;
    std::vector<long long> links_host; // mirror of the link difference arrays
    int static_dev = -1;               // device whose library-held workspace this handle holds, or -1
    bool state_lost = false;           // a state-resident launch gave up: state undefined until reset
};

// MFMA path: whether this network's launches build their B tiles from the
// compact crossbar (RANC_MFMA_BSRC=planes|compact at load overrides the
// default choice, mfma_compact_b)
static int mfma_compact(const ranc_net *net)
{
    const Plan &p = net->p;
    return p.bsrc >= 0 ? p.bsrc : mfma_compact_b(net->dn, p.two, p.spw) ? 1 : 0;
}

static hipError_t prof_begin(ranc_net *net, int kind, hipStream_t s, int *slot)
{
    *slot = -1;
    if (!net->prof.on)
        return hipSuccess;
    Profiler &pr = net->prof;
    const size_t idx = pr.used.size();
    if (idx == pr.pool.size()) {
        EventPair e;
        hipError_t r = hipEventCreate(&e.a);
        if (r == hipSuccess)
            r = hipEventCreate(&e.b);
        if (r != hipSuccess)
            return r;
        pr.pool.push_back(e);
    }
    pr.used.push_back({(int)idx, kind});
    *slot = (int)idx;
    return hipEventRecord(pr.pool[idx].a, s);
}

static hipError_t prof_end(ranc_net *net, int slot, hipStream_t s)
{
    if (slot < 0)
        return hipSuccess;
    return hipEventRecord(net->prof.pool[slot].b, s);
}

// Fold recorded event pairs into the totals (the stream must be synchronized).
static hipError_t prof_collect(ranc_net *net)
{
    Profiler &pr = net->prof;
    for (auto &u : pr.used) {
        float ms = 0.f;
        hipError_t r = hipEventElapsedTime(&ms, pr.pool[u.first].a, pr.pool[u.first].b);
        if (r != hipSuccess)
            return r;
        pr.ms[u.second] += ms;
        pr.launches[u.second] += 1;
    }
    pr.used.clear();
    return hipSuccess;
}

// Queue num_ticks ticks on stream s: per tick the integration (and on the
// plain path the router), then the device tick advance. With `timed`, HIP
// event pairs are recorded around each launch while profiling is on.
static ranc_status queue_ticks(ranc_net *net, const uint32_t *base, int num_ticks, hipStream_t s, bool timed)
{
    const Plan &p = net->p;
    const size_t tick_words = (size_t)p.Cin * p.W;
    timed = timed && net->prof.on;
    for (int k = 0; k < num_ticks; ++k) {
        TickArgs ta;
        ta.k = k;
        ta.ext_t = base ? base + (size_t)k * tick_words : nullptr;
        ta.ext_sstride = (long long)num_ticks * tick_words;
        // A long timed run folds finished event pairs in batches.
        if (timed && net->prof.used.size() >= 4096) {
            hipError_t e = hipStreamSynchronize(s);
            if (e == hipSuccess)
                e = prof_collect(net);
            if (e != hipSuccess)
                return hip_fail(e, "collecting kernel timings");
        }
        int slot = -1;
        hipError_t e = timed ? prof_begin(net, 0, s, &slot) : hipSuccess;
        if (e == hipSuccess)
            e = p.path == RANC_PATH_MFMA     ? launch_integrate_mfma(net->dn, ta, p.two, p.spw, mfma_compact(net), s)
                : p.path == RANC_PATH_SPARSE ? launch_integrate_sparse(net->dn, ta, p.spw, s)
                                             : launch_integrate_plain(net->dn, ta, s);
        if (e == hipSuccess && timed)
            e = prof_end(net, slot, s);
        if (e != hipSuccess)
            return hip_fail(e, "launching integration");
        // The MFMA path delivers spikes inside the next tick's integration
        // (spike history gathered by destination); the plain path routes
        // into the scheduler ring here.
        if (p.path == RANC_PATH_PLAIN) {
            e = timed ? prof_begin(net, 1, s, &slot) : hipSuccess;
            if (e == hipSuccess)
                e = launch_route(net->dn, k, net->rcfg, s);
            if (e == hipSuccess && timed)
                e = prof_end(net, slot, s);
            if (e != hipSuccess)
                return hip_fail(e, "launching routing");
        }
        if (net->links_on) {
            e = launch_link_counts(net->dn, net->lk, k, s);
            if (e != hipSuccess)
                return hip_fail(e, "launching the mesh link count");
        }
    }
    hipError_t e = launch_fold_counts(net->dn, num_ticks, s);
    if (e == hipSuccess)
        e = launch_advance_tick(net->dn, num_ticks, s);
    if (e != hipSuccess)
        return hip_fail(e, "advancing the tick");
    return RANC_OK;
}

// Run num_ticks ticks as one captured graph: the tick loop is captured once
// per (num_ticks, input address) on a private stream and replayed on s.
// Every launch argument is position-in-call relative (the scheduler slot and
// raster row come from the device tick), so one graph serves every call.
static ranc_status run_captured(ranc_net *net, const uint32_t *base, int num_ticks, hipStream_t s)
{
    CapturedLoop *loop = nullptr;
    for (auto &g : net->loops)
        if (g.num_ticks == num_ticks && g.base == base)
            loop = &g;
    if (!loop) {
        hipError_t e = hipSuccess;
        if (!net->cap_stream)
            e = hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return hip_fail(e, "creating the capture stream");
        e = hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess)
            return hip_fail(e, "beginning capture");
        ranc_status st = queue_ticks(net, base, num_ticks, net->cap_stream, false);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(net->cap_stream, &graph);
        if (st != RANC_OK) {
            if (graph)
                hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess)
            return hip_fail(e, "ending capture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(graph);
            return hip_fail(e, "instantiating the tick loop");
        }
        if (net->loops.size() >= MAX_CAPTURED_LOOPS) {
            // drop the least recently used loop; its last replay may still be
            // queued, so wait for the handle's stream first
            e = hipStreamSynchronize(net->last_stream);
            if (e == hipSuccess && net->last_stream != s)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                hipGraphExecDestroy(exec);
                hipGraphDestroy(graph);
                return hip_fail(e, "synchronizing before dropping a captured tick loop");
            }
            auto old = std::min_element(net->loops.begin(), net->loops.end(),
                                        [](const CapturedLoop &x, const CapturedLoop &y) { return x.used < y.used; });
            hipGraphExecDestroy(old->exec);
            hipGraphDestroy(old->graph);
            net->loops.erase(old);
            ++net->loops_dropped;
        }
        net->loops.push_back({num_ticks, base, graph, exec, 0});
        loop = &net->loops.back();
    }
    loop->used = ++net->replays;
    int slot = -1;
    hipError_t e = prof_begin(net, 2, s, &slot);
    if (e == hipSuccess)
        e = hipGraphLaunch(loop->exec, s);
    if (e == hipSuccess)
        e = prof_end(net, slot, s);
    if (e != hipSuccess)
        return hip_fail(e, "launching the tick loop");
    return RANC_OK;
}

static int device_cu_count();

// Longest wait at a grid barrier of the state-resident loop, in microseconds
// (a normal wait takes a few). RANC_RESIDENT_WAIT_US overrides it (at most
// one hour).
static unsigned long long resident_wait_us()
{
    const char *e = getenv("RANC_RESIDENT_WAIT_US");
    if (e && *e) {
        char *end = nullptr;
        const unsigned long long v = strtoull(e, &end, 10);
        if (end && *end == '\0')
            return std::min(v, 3600000000ull);
    }
    return 2000000ull;
}

// Why the state-resident loop cannot run this handle (nullptr: it can), and
// its grid.
static const char *resident_blocker(const ranc_net *net, int num_ticks, int *grid)
{
    const Plan &p = net->p;
    if (p.path != RANC_PATH_MFMA)
        return "the state-resident loop runs MFMA-path handles only";
    if (p.N != 256 || p.slices != 1)
        return "the state-resident loop needs cores of 256 neurons";
    if (p.A > 256)
        return "the state-resident loop needs cores of at most 256 axons";
    if (!net->dn.planes)
        return "the state-resident loop needs the weight planes";
    if (net->links_on)
        return "mesh link counting needs the per-tick loop";
    const int per_cu = resident_blocks_per_cu(p.A, p.two, net->dn.model_ext);
    const int cus = device_cu_count();
    if (per_cu < 1 || cus < 1)
        return "the state-resident kernel cannot be resident on this device";
    const long long max_wg = (long long)per_cu * cus;
    const long long cpw = ((long long)p.C + max_wg - 1) / max_wg;
    if (cpw > resident_max_cores_per_wg())
        return "too many cores to keep resident on this device";
    *grid = (int)((p.C + cpw - 1) / cpw);
    // the arrival counter counts every workgroup at every barrier (one per
    // tick and 64-sample group) in 32 bits
    if ((unsigned long long)(p.S64 / 64) * (unsigned long long)num_ticks * (unsigned long long)*grid >= (1ull << 32))
        return "too many ticks x sample groups for one state-resident launch";
    return nullptr;
}

// All ticks of the call in one cooperative launch (kern_resident.hip), then
// the count fold and tick advance. The launch's give-up flag is read back
// before returning (the call synchronizes `s`).
static ranc_status run_resident(ranc_net *net, const uint32_t *base, int num_ticks, hipStream_t s)
{
    const Plan &p = net->p;
    int grid = 0;
    if (const char *why = resident_blocker(net, num_ticks, &grid))
        return fail(RANC_EUNSUPPORTED, "%s", why);
    int dev = 0, rate_khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess || rate_khz < 1)
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidValue, "reading the device wall-clock rate");
    ResidentArgs ra;
    ra.ext_base = base;
    ra.tick_words = (long long)p.Cin * p.W;
    ra.ext_sstride = (long long)num_ticks * ra.tick_words;
    ra.num_ticks = num_ticks;
    unsigned *sync = (unsigned *)(net->ws + p.off[R_RSYNC]);
    ResSync sy;
    sy.ctr = sync;
    sy.abort = sync + 1;
    sy.wait_ticks = resident_wait_us() * (unsigned long long)rate_khz / 1000ull;
    int slot = -1;
    e = prof_begin(net, 3, s, &slot);
    if (e == hipSuccess)
        e = launch_mfma_resident(net->dn, ra, sy, grid, p.two, s);
    if (e == hipSuccess)
        e = prof_end(net, slot, s);
    if (e != hipSuccess)
        return hip_fail(e, "launching the state-resident tick loop");
    e = launch_fold_counts(net->dn, num_ticks, s);
    if (e == hipSuccess)
        e = launch_advance_tick(net->dn, num_ticks, s);
    if (e != hipSuccess)
        return hip_fail(e, "advancing the tick");
    unsigned gave_up = 0;
    e = hipMemcpyAsync(&gave_up, sy.abort, sizeof(gave_up), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "reading the state-resident loop's give-up flag");
    if (gave_up) {
        net->state_lost = true;
        return fail(RANC_ETIMEOUT, "a grid barrier of the state-resident loop waited longer than %llu us; "
                                   "the state is undefined until ranc_reset_state",
                    resident_wait_us());
    }
    return RANC_OK;
}

// ---------------------------------------------------------------------------
// Batches: several networks (any shapes) advanced together, one launch per
// tick and path for all of them (plus one router launch for the plain path).

static int device_cu_count()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    return cus;
}

// Build the host tables of a batch: for the persistent MFMA launch one unit
// numbering sorted by decreasing work per unit (largest units handed out
// first); otherwise the MFMA entries by phase and shape class, each class
// split into launches of at most MFMA_GROUP_MAX networks whose descriptions
// travel as kernel arguments; plain entries by phase.
static ranc_status build_batch(ranc_net *const *nets, int num, const uint32_t *const *bases,
                               int num_ticks, bool persistent, Batch &b)
{
    b.persistent = persistent;
    b.groups.clear();
    b.phases.clear();
    // Phase of each network: first fit, largest state first, into phases of
    // at most `budget` bytes of state (a larger network forms its own phase).
    // Networks are independent, so running them phase after phase is exact.
    // Off unless RANC_BATCH_PHASE_MB is set: on the 64-variant sweep, phases
    // of 64 or 160 MB were 0.5-1% slower than one phase.
    size_t budget = 0;
    if (const char *env = getenv("RANC_BATCH_PHASE_MB"))
        budget = (size_t)std::max(0, atoi(env)) << 20;
    std::vector<int> phase_of(num, 0);
    if (!persistent && budget > 0) {
        std::vector<std::pair<size_t, int>> foot;
        for (int i = 0; i < num; ++i) {
            const Plan &p = nets[i]->p;
            foot.push_back({p.params_bytes + p.size[R_BSRC] + p.size[R_V] + p.size[R_HIST] + p.size[R_RING] +
                                p.size[R_SPK] + p.size[R_CNT],
                            i});
        }
        std::stable_sort(foot.begin(), foot.end(), [](const std::pair<size_t, int> &x,
                                                       const std::pair<size_t, int> &y) { return x.first > y.first; });
        std::vector<size_t> fill;
        for (const auto &f : foot) {
            size_t ph = 0;
            while (ph < fill.size() && fill[ph] + f.first > budget)
                ++ph;
            if (ph == fill.size())
                fill.push_back(0);
            fill[ph] += f.first;
            phase_of[f.second] = (int)ph;
        }
    }
    b.nets.assign(nets, nets + num);
    b.uids.clear();
    for (int i = 0; i < num; ++i)
        b.uids.push_back(nets[i]->uid);
    b.bases.assign(bases, bases + num);
    b.num_ticks = num_ticks;
    b.mf.clear();
    b.pl.clear();
    b.rt_lds = 0;
    for (int i = 0; i < num; ++i) {
        ranc_net *net = nets[i];
        const Plan &p = net->p;
        BatchEntry e;
        memset(&e, 0, sizeof e);
        e.n = net->dn;
        e.ext_base = bases[i];
        e.tick_words = (long long)p.Cin * p.W;
        e.ext_sstride = (long long)num_ticks * e.tick_words;
        e.spw = p.spw;
        e.compact = p.path == RANC_PATH_MFMA ? mfma_compact(net) : 0;
        e.phase = phase_of[i];
        if (p.path == RANC_PATH_SPARSE)
            return fail(RANC_EUNSUPPORTED, "nets[%d]: the sparse path runs one network per call", i);
        if (p.path == RANC_PATH_MFMA) {
            e.code = mfma_shape_code(p.A, mfma_width(p.A, p.N, p.two), p.two);
            e.units = p.C * p.slices * ((p.S + p.spw - 1) / p.spw);
            b.mf.push_back(e);
        } else {
            e.code = plain_shape_code(p.W, p.G);
            e.units = p.C * p.S * (p.N / 64);
            // batched routing reads the spike bitmaps from L2 (no LDS staging,
            // so the one launch keeps its occupancy for every network)
            RouteCfg rc = net->rcfg;
            rc.stage = 0;
            e.route_code = route_shape_code(rc, p.D);
            if (e.route_code < 0)
                return fail(RANC_EUNSUPPORTED, "nets[%d]: router shape (%d samples per block, max delay %d) "
                            "cannot run in a batch", i, net->rcfg.samples_per_block, p.D);
            e.route_split = net->rcfg.blocks_per_group;
            e.route_units = e.route_split * ((p.S + net->rcfg.samples_per_block - 1) / net->rcfg.samples_per_block);
            b.pl.push_back(e);
        }
    }
    if ((int)b.mf.size() > BATCH_MAX || (int)b.pl.size() > BATCH_MAX)
        return fail(RANC_EUNSUPPORTED, "a batch holds at most %d networks per path", BATCH_MAX);
    auto work = [](const BatchEntry &e) {
        return (double)e.spw * (e.n.N / e.n.slices) * (e.n.A + 64) * ((e.code & 1) ? 2 : 1);
    };
    auto ext = [](const BatchEntry &e) { return e.n.model_ext; };
    auto compact = [](const BatchEntry &e) { return e.compact; };
    long long mu = 0, pu = 0, ru = 0;
    if (persistent) {
        // one unit numbering, largest units first
        std::stable_sort(b.mf.begin(), b.mf.end(),
                         [&](const BatchEntry &x, const BatchEntry &y) { return work(x) > work(y); });
        for (auto &e : b.mf) {
            e.unit_begin = (int)mu;
            mu += e.units;
        }
    } else {
        // by phase, then shape class (each numbered from 0), largest units first within a class
        std::stable_sort(b.mf.begin(), b.mf.end(), [&](const BatchEntry &x, const BatchEntry &y) {
            if (x.phase != y.phase)
                return x.phase < y.phase;
            if (x.code != y.code)
                return x.code < y.code;
            if (ext(x) != ext(y))
                return ext(x) < ext(y);
            if (compact(x) != compact(y))
                return compact(x) < compact(y);
            return work(x) > work(y);
        });
        for (size_t i = 0; i < b.mf.size(); ++i) {
            BatchEntry &e = b.mf[i];
            if (b.groups.empty() || b.mf[b.groups.back().first].phase != e.phase ||
                b.groups.back().code != e.code || b.groups.back().ext != ext(e) ||
                b.groups.back().compact != compact(e) || b.groups.back().num == MFMA_GROUP_MAX) {
                b.groups.push_back(Batch::Group());
                Batch::Group &g = b.groups.back();
                memset(&g.args, 0, sizeof g.args);
                g.first = (int)i;
                g.num = g.units = 0;
                g.code = e.code;
                g.ext = ext(e);
                g.compact = compact(e);
            }
            Batch::Group &g = b.groups.back();
            if ((long long)g.units + e.units > INT32_MAX)
                return fail(RANC_EUNSUPPORTED, "batch has too many work units");
            e.unit_begin = g.units;
            MfmaGroupEntry &ge = g.args.e[g.num];
            ge.n = e.n;
            ge.ext_base = e.ext_base;
            ge.tick_words = e.tick_words;
            ge.ext_sstride = e.ext_sstride;
            ge.spw = e.spw;
            ge.unit_begin = e.unit_begin;
            g.units += e.units;
            g.num += 1;
            g.args.num = g.num;
            mu += e.units;
        }
    }
    // plain entries by phase, numbered from 0 within the phase
    std::stable_sort(b.pl.begin(), b.pl.end(),
                     [](const BatchEntry &x, const BatchEntry &y) { return x.phase < y.phase; });
    int nphases = 0;
    for (int i = 0; i < num; ++i)
        nphases = std::max(nphases, phase_of[i] + 1);
    b.phases.assign(nphases, Batch::Phase{0, 0, 0, 0, 0, 0});
    b.phase_links.assign(nphases, std::vector<int>());
    b.links.assign(num, 0);
    for (int i = 0; i < num; ++i) {
        b.links[i] = nets[i]->links_on ? 1 : 0;
        if (nets[i]->links_on)
            b.phase_links[phase_of[i]].push_back(i);
    }
    for (size_t g = b.groups.size(); g-- > 0;) {
        Batch::Phase &ph = b.phases[b.mf[b.groups[g].first].phase];
        ph.g_first = (int)g;
        ph.g_num += 1;
    }
    for (size_t i = b.pl.size(); i-- > 0;)
        b.phases[b.pl[i].phase].pl_first = (int)i;
    for (auto &e : b.pl) {
        Batch::Phase &ph = b.phases[e.phase];
        if ((long long)ph.pl_units + e.units > INT32_MAX || (long long)ph.rt_units + e.route_units > INT32_MAX)
            return fail(RANC_EUNSUPPORTED, "batch has too many work units");
        e.unit_begin = ph.pl_units;
        ph.pl_units += e.units;
        e.route_begin = ph.rt_units;
        ph.rt_units += e.route_units;
        ph.pl_num += 1;
        pu += e.units;
        ru += e.route_units;
    }
    if (mu > INT32_MAX || pu > INT32_MAX || ru > INT32_MAX)
        return fail(RANC_EUNSUPPORTED, "batch has too many work units");
    b.mf_units = (int)mu;
    b.pl_units = (int)pu;
    b.rt_units = (int)ru;
    b.mf_workgroups = (int)std::min<long long>(mu, device_cu_count());
    return RANC_OK;
}

static BatchEntry *batch_table(ranc_net *lead, int which)
{
    return (BatchEntry *)(lead->ws + lead->p.off[R_BATCH]) + (which ? BATCH_MAX : 0);
}

static unsigned *batch_queue(ranc_net *lead)
{
    return (unsigned *)(batch_table(lead, 0) + 2 * BATCH_MAX);
}

// Branch form of a batch's ticks: the networks of different shape classes do
// not depend on each other, so each class's launches for all ticks form one
// chain, and the chains (and the chain of the plain-path networks) run on the
// lead handle's branch streams side by side, forked from and joined back to
// `s` with events (under stream capture they become parallel branches of the
// graph). Used when nothing orders the classes within a tick: one phase, no
// persistent launch, no link counting, no per-launch timing.
static hipError_t queue_batch_branches(ranc_net *lead, const Batch &b, hipStream_t s)
{
    const BatchEntry *tpl = batch_table(lead, 1);
    const Batch::Phase &ph = b.phases[0];
    const int chains = ph.g_num + (ph.pl_num > 0 ? 1 : 0);
    const int nb = std::min(chains, (int)ranc_net::BATCH_BRANCHES);
    hipError_t e = hipSuccess;
    for (int i = 0; e == hipSuccess && i < nb; ++i) {
        if (!lead->br_stream[i])
            e = hipStreamCreateWithFlags(&lead->br_stream[i], hipStreamNonBlocking);
        if (e == hipSuccess && !lead->br_join[i])
            e = hipEventCreateWithFlags(&lead->br_join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess && !lead->br_fork)
        e = hipEventCreateWithFlags(&lead->br_fork, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventRecord(lead->br_fork, s);
    for (int i = 0; e == hipSuccess && i < nb; ++i)
        e = hipStreamWaitEvent(lead->br_stream[i], lead->br_fork, 0);
    for (int c = 0; e == hipSuccess && c < chains; ++c) {
        hipStream_t st = lead->br_stream[c % nb];
        if (c < ph.g_num) {
            const Batch::Group &g = b.groups[ph.g_first + c];
            for (int k = 0; e == hipSuccess && k < b.num_ticks; ++k)
                e = launch_integrate_mfma_group(g.args, g.units, k, g.code, g.ext, g.compact, st);
        } else {
            const BatchEntry *tp = tpl + ph.pl_first;
            for (int k = 0; e == hipSuccess && k < b.num_ticks; ++k) {
                e = launch_integrate_plain_batch(tp, ph.pl_num, ph.pl_units, k, st);
                if (e == hipSuccess)
                    e = launch_route_batch(tp, ph.pl_num, ph.rt_units, k, b.rt_lds, st);
            }
        }
    }
    for (int i = 0; e == hipSuccess && i < nb; ++i) {
        e = hipEventRecord(lead->br_join[i], lead->br_stream[i]);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, lead->br_join[i], 0);
    }
    return e;
}

static ranc_status queue_batch_ticks(ranc_net *lead, const Batch &b, hipStream_t s, bool timed)
{
    const BatchEntry *tmf = batch_table(lead, 0), *tpl = batch_table(lead, 1);
    unsigned *queue = batch_queue(lead);
    timed = timed && lead->prof.on;
    bool any_links = false;
    for (const auto &pl : b.phase_links)
        any_links = any_links || !pl.empty();
    const bool branches = !b.persistent && b.phases.size() == 1 && !any_links && !timed &&
                          b.phases[0].g_num + (b.phases[0].pl_num > 0 ? 1 : 0) > 1;
    if (branches) {
        hipError_t e = queue_batch_branches(lead, b, s);
        if (e != hipSuccess)
            return hip_fail(e, "launching batch integration (branches)");
    }
    for (const Batch::Phase &ph : b.phases)
    for (int k = 0; !branches && k < b.num_ticks; ++k) {
        int slot = -1;
        hipError_t e = hipSuccess;
        const bool mf = b.persistent ? !b.mf.empty() : ph.g_num > 0;
        if (mf) {
            e = timed ? prof_begin(lead, 0, s, &slot) : hipSuccess;
            if (e == hipSuccess && b.persistent)
                e = launch_integrate_mfma_batch(tmf, (int)b.mf.size(), b.mf_units, k, queue, b.mf_workgroups, s);
            for (int g = ph.g_first; e == hipSuccess && !b.persistent && g < ph.g_first + ph.g_num; ++g)
                e = launch_integrate_mfma_group(b.groups[g].args, b.groups[g].units, k, b.groups[g].code,
                                                b.groups[g].ext, b.groups[g].compact, s);
            if (e == hipSuccess && timed)
                e = prof_end(lead, slot, s);
            if (e != hipSuccess)
                return hip_fail(e, "launching batch integration (MFMA)");
        }
        if (ph.pl_num > 0) {
            const BatchEntry *tp = tpl + ph.pl_first;
            e = timed ? prof_begin(lead, 0, s, &slot) : hipSuccess;
            if (e == hipSuccess)
                e = launch_integrate_plain_batch(tp, ph.pl_num, ph.pl_units, k, s);
            if (e == hipSuccess && timed)
                e = prof_end(lead, slot, s);
            if (e == hipSuccess)
                e = timed ? prof_begin(lead, 1, s, &slot) : hipSuccess;
            if (e == hipSuccess)
                e = launch_route_batch(tp, ph.pl_num, ph.rt_units, k, b.rt_lds, s);
            if (e == hipSuccess && timed)
                e = prof_end(lead, slot, s);
            if (e != hipSuccess)
                return hip_fail(e, "launching batch integration (plain)");
        }
        for (int i : b.phase_links[&ph - b.phases.data()]) {
            e = launch_link_counts(b.nets[i]->dn, b.nets[i]->lk, k, s);
            if (e != hipSuccess)
                return hip_fail(e, "launching the mesh link count");
        }
    }
    hipError_t e = hipSuccess;
    for (size_t i = 0; e == hipSuccess && i < b.nets.size(); ++i)
        e = launch_fold_counts(b.nets[i]->dn, b.num_ticks, s);
    if (e == hipSuccess && !b.mf.empty())
        e = launch_advance_batch(tmf, (int)b.mf.size(), b.num_ticks, queue, s);
    if (e == hipSuccess && !b.pl.empty())
        e = launch_advance_batch(tpl, (int)b.pl.size(), b.num_ticks, queue, s);
    if (e != hipSuccess)
        return hip_fail(e, "advancing batch ticks");
    return RANC_OK;
}

// Run num_ticks ticks of several networks together. The batch set-up (tables
// in the first network's workspace, and the captured graph with
// RANC_RUN_GRAPH) is reused while the same networks, input addresses and
// tick count repeat.
static ranc_status run_batch(ranc_net *const *nets, int num, const uint32_t *const *bases, int num_ticks,
                             bool graph, bool persistent, hipStream_t s)
{
    ranc_net *lead = nets[0];
    Batch &b = lead->batch;
    bool same = b.num_ticks == num_ticks && b.persistent == persistent && (int)b.nets.size() == num &&
                std::equal(b.nets.begin(), b.nets.end(), nets) && std::equal(b.bases.begin(), b.bases.end(), bases);
    for (int i = 0; same && i < num; ++i)
        same = b.uids[i] == nets[i]->uid && b.links[i] == (nets[i]->links_on ? 1 : 0);
    if (!same) {
        if (b.exec)
            hipGraphExecDestroy(b.exec);
        if (b.graph)
            hipGraphDestroy(b.graph);
        b.exec = nullptr;
        b.graph = nullptr;
        b.num_ticks = 0;
        Batch nb;
        ranc_status st = build_batch(nets, num, bases, num_ticks, persistent, nb);
        if (st != RANC_OK)
            return st;
        // the previous tables may still be read by queued work
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess && !nb.mf.empty())
            e = hipMemcpy(batch_table(lead, 0), nb.mf.data(), nb.mf.size() * sizeof(BatchEntry), hipMemcpyHostToDevice);
        if (e == hipSuccess && !nb.pl.empty())
            e = hipMemcpy(batch_table(lead, 1), nb.pl.data(), nb.pl.size() * sizeof(BatchEntry), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            const unsigned zero[2] = {0u, 0u};
            e = hipMemcpy(batch_queue(lead), zero, sizeof zero, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess)
            return hip_fail(e, "uploading the batch table");
        b.nets = std::move(nb.nets);
        b.uids = std::move(nb.uids);
        b.bases = std::move(nb.bases);
        b.mf = std::move(nb.mf);
        b.pl = std::move(nb.pl);
        b.groups = std::move(nb.groups);
        b.phases = std::move(nb.phases);
        b.phase_links = std::move(nb.phase_links);
        b.links = std::move(nb.links);
        b.persistent = nb.persistent;
        b.mf_units = nb.mf_units;
        b.pl_units = nb.pl_units;
        b.rt_units = nb.rt_units;
        b.mf_workgroups = nb.mf_workgroups;
        b.rt_lds = nb.rt_lds;
        b.num_ticks = num_ticks;
    }
    if (!graph)
        return queue_batch_ticks(lead, b, s, true);
    if (!b.exec) {
        hipError_t e = hipSuccess;
        if (!lead->cap_stream)
            e = hipStreamCreateWithFlags(&lead->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipStreamBeginCapture(lead->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess)
            return hip_fail(e, "beginning batch capture");
        ranc_status st = queue_batch_ticks(lead, b, lead->cap_stream, false);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(lead->cap_stream, &g);
        if (st != RANC_OK) {
            if (g)
                hipGraphDestroy(g);
            return st;
        }
        if (e == hipSuccess)
            e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g)
                hipGraphDestroy(g);
            return hip_fail(e, "capturing the batch tick loop");
        }
        b.graph = g;
    }
    int slot = -1;
    hipError_t e = prof_begin(lead, 2, s, &slot);
    if (e == hipSuccess)
        e = hipGraphLaunch(b.exec, s);
    if (e == hipSuccess)
        e = prof_end(lead, slot, s);
    if (e != hipSuccess)
        return hip_fail(e, "launching the batch tick loop");
    return RANC_OK;
}

static void drop_graphs(ranc_net *net);

extern "C" {

const char *ranc_last_error(void) { return g_err.c_str(); }

ranc_status ranc_workspace_bytes(const ranc_net_desc *desc, int32_t num_samples, int32_t max_ticks_per_call,
                                 int32_t path, size_t *bytes)
{
    if (!bytes)
        return fail(RANC_EINVAL, "bytes is NULL");
    Plan p;
    ranc_status st = make_plan(desc, num_samples, max_ticks_per_call, path, p);
    if (st != RANC_OK)
        return st;
    *bytes = p.total;
    return RANC_OK;
}

ranc_status ranc_load_network(const ranc_net_desc *desc, int32_t num_samples, int32_t max_ticks_per_call,
                              int32_t path, void *workspace, size_t workspace_bytes, void *stream, ranc_net **out)
{
    if (!out)
        return fail(RANC_EINVAL, "out is NULL");
    *out = nullptr;
    Plan p;
    ranc_status st = make_plan(desc, num_samples, max_ticks_per_call, path, p);
    if (st != RANC_OK)
        return st;
    if (!workspace)
        return fail(RANC_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256)
        return fail(RANC_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < p.total)
        return fail(RANC_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, p.total);
    ranc_net *net = new (std::nothrow) ranc_net();
    if (!net)
        return fail(RANC_ENOMEM, "host allocation failed");
    static std::atomic<uint64_t> next_uid{1};
    net->p = p;
    net->uid = next_uid++;
    net->ws = (uint8_t *)workspace;
    auto reg = [&](Region r) -> uint8_t * { return net->ws + p.off[r]; };
    DevNet &n = net->dn;
    n.C = p.C; n.A = p.A; n.N = p.N; n.G = p.G; n.W = p.W; n.NW = p.NW; n.D = p.D; n.Q = p.Q;
    n.S = p.S; n.S64 = p.S64; n.RT = p.RT; n.Wout = p.Wout; n.Nout = p.Nout; n.Cin = p.Cin;
    n.cnt_rows = p.cnt_rows;
    n.slices = p.slices;
    n.vlayout = p.path == RANC_PATH_MFMA ? VLAYOUT_BRICK : p.path == RANC_PATH_SPARSE ? VLAYOUT_SPARSE : VLAYOUT_CSN;
    n.vmin = (int32_t)(-(1LL << (desc->potential_bits - 1)));
    n.vmax = (int32_t)((1LL << (desc->potential_bits - 1)) - 1);
    n.model_ext = neuron_model_ext(desc) ? 1 : 0;
    n.floor = (const int32_t *)reg(R_FLOOR);
    n.linmask = (const uint32_t *)reg(R_LINMASK);
    // the plain path's column words, or the MFMA path's compact B source
    // (which starts with the same words)
    n.colbits = p.size[R_BSRC] ? (const uint32_t *)reg(R_BSRC)
                : p.size[R_COLBITS] ? (const uint32_t *)reg(R_COLBITS) : nullptr;
    n.typemask = (const uint32_t *)reg(R_TYPEMASK);
    n.wts = (const int32_t *)reg(R_WTS);
    n.leak = (const int32_t *)reg(R_LEAK);
    n.thr = (const int32_t *)reg(R_THR);
    n.rst = (const int32_t *)reg(R_RST);
    n.vinit = (const int32_t *)reg(R_VINIT);
    n.coremask = (const uint32_t *)reg(R_COREMASK);
    n.outmask = (const uint32_t *)reg(R_OUTMASK);
    n.outword = (const int32_t *)reg(R_OUTWORD);
    n.in_index = (const int32_t *)reg(R_ININDEX);
    n.rt_dcnt = (const uint16_t *)reg(R_RTDCNT);
    n.rt_goff = (const uint32_t *)reg(R_RTGOFF);
    n.rt_ent = (const uint32_t *)reg(R_RTENT);
    n.degb = (const uint32_t *)reg(R_DEGB);
    n.outidx = (const int32_t *)reg(R_OUTIDX);
    n.planes = p.size[R_PLANES] ? (const uint4 *)reg(R_PLANES) : nullptr;
    n.V = (int32_t *)reg(R_V);
    n.ring = (uint32_t *)reg(R_RING);
    n.spk = (uint32_t *)reg(R_SPK);
    n.hist = (uint64_t *)reg(R_HIST);
    n.rtx_ptr = (const uint32_t *)reg(R_RTXPTR);
    n.rtx_ent = (const uint32_t *)reg(R_RTXENT);
    n.hist_zero = (const uint64_t *)reg(R_HZERO);
    n.ecsr_ptr = (const uint32_t *)reg(R_ECSRPTR);
    n.ecsr_ent = (const uint16_t *)reg(R_ECSRENT);
    n.raster = (uint32_t *)reg(R_RASTER);
    n.cnt = (unsigned long long *)reg(R_CNT);
    n.cring = (unsigned long long *)reg(R_CRING);
    n.tick = (int *)reg(R_TICK);
    net->lk.rec = (const int2 *)reg(R_LINKREC);
    net->lk.rows = p.size[R_LINKPTR] ? (const uint32_t *)reg(R_LINKPTR) : nullptr;
    net->lk.ents = p.size[R_LINKPTR] ? (const uint32_t *)reg(R_LINKENT) : nullptr;
    net->outcol = p.size[R_OUTCOL] ? (const int2 *)reg(R_OUTCOL) : nullptr;
    net->opos = p.size[R_OUTPOS] ? (const int32_t *)reg(R_OUTPOS) : nullptr;
    net->lk.d = (long long *)reg(R_LINKD);
    std::vector<uint8_t> host;
    pack_params(desc, p, host, net->out_words);
    for (size_t i = 0; i < (size_t)p.C * p.N; ++i)
        if (desc->dest_kind[i] == RANC_DEST_OUT) {
            net->out_neurons.push_back((int)(i / p.N));
            net->out_neurons.push_back((int)(i % p.N));
        }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(net->ws, host.data(), p.params_bytes, hipMemcpyHostToDevice, s);
    std::vector<uint8_t> bsrc;
    if (e == hipSuccess && p.size[R_BSRC]) {
        pack_bsrc(desc, p, bsrc);
        e = hipMemcpyAsync(reg(R_BSRC), bsrc.data(), bsrc.size(), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess)
        e = launch_reset_state(n, net->lk, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete net;
        return hip_fail(e, "uploading the network");
    }
    net->rcfg = route_default_cfg(n);
    if (const char *e = getenv("RANC_ROUTE_SB")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8)
            net->rcfg.samples_per_block = v;
    }
    if (const char *e = getenv("RANC_ROUTE_SPLIT")) {
        const int v = atoi(e);
        if (v >= 1)
            net->rcfg.blocks_per_group = v;
    }
    if (const char *e = getenv("RANC_ROUTE_STAGE"))
        net->rcfg.stage = atoi(e) != 0;
    if ((size_t)n.C * n.NW * 4 * net->rcfg.samples_per_block > 128 * 1024)
        net->rcfg.stage = 0;
    net->rcfg.lanes = route_auto_lanes(n, net->rcfg);
    net->last_stream = s;
    net->tick = 0;
    net->version = 1;
    net->raster_version = 0;
    *out = net;
    return RANC_OK;
}

ranc_status ranc_load_network_static(const ranc_net_desc *desc, int32_t num_samples, int32_t max_ticks_per_call,
                                     int32_t path, void *stream, ranc_net **out)
{
    if (!out)
        return fail(RANC_EINVAL, "out is NULL");
    *out = nullptr;
    Plan p;
    ranc_status st = make_plan(desc, num_samples, max_ticks_per_call, path, p);
    if (st != RANC_OK)
        return st;
    if (p.total > RANC_STATIC_WORKSPACE_BYTES)
        return fail(RANC_ENOMEM, "the network needs %zu bytes of workspace; the library-held workspace has %zu",
                    p.total, (size_t)RANC_STATIC_WORKSPACE_BYTES);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "querying the current device");
    if (dev < 0 || dev >= STATIC_WS_MAX_DEVICES)
        return fail(RANC_EUNSUPPORTED, "device %d: the library-held workspace exists for devices 0..%d", dev,
                    STATIC_WS_MAX_DEVICES - 1);
    void *ws = nullptr;
    bool held = false;
    e = static_ws_claim(dev, &ws, &held);
    if (e != hipSuccess)
        return hip_fail(e, "looking up the library-held workspace");
    if (held)
        return fail(RANC_ESTATE, "the library-held workspace of device %d is used by a handle not yet freed", dev);
    st = ranc_load_network(desc, num_samples, max_ticks_per_call, path, ws, RANC_STATIC_WORKSPACE_BYTES, stream,
                           out);
    if (st != RANC_OK) {
        static_ws_release(dev);
        return st;
    }
    (*out)->static_dev = dev;
    return RANC_OK;
}

ranc_status ranc_run_ticks(ranc_net *const *nets, int32_t num_nets, const uint32_t *const *inputs, uint32_t flags,
                           int32_t num_ticks, void *stream)
{
    if (!nets || num_nets < 1)
        return fail(RANC_EINVAL, "nets is NULL or num_nets < 1");
    for (int i = 0; i < num_nets; ++i) {
        if (!nets[i])
            return fail(RANC_EINVAL, "nets[%d] is NULL", i);
        if (num_ticks < 1 || num_ticks > nets[i]->p.RT)
            return fail(RANC_EINVAL, "num_ticks %d outside [1, max_ticks_per_call=%d]", num_ticks, nets[i]->p.RT);
    }
    if (flags & ~(RANC_INPUTS_ON_DEVICE | RANC_RUN_GRAPH | RANC_BATCH_PERSISTENT | RANC_RUN_RESIDENT))
        return fail(RANC_EINVAL, "unknown flags 0x%x", flags);
    for (int i = 0; i < num_nets; ++i)
        if (nets[i]->state_lost)
            return fail(RANC_ESTATE, "nets[%d]: a state-resident run gave up; reset the state first", i);
    if (flags & RANC_RUN_RESIDENT) {
        if (num_nets != 1)
            return fail(RANC_EUNSUPPORTED, "RANC_RUN_RESIDENT runs one network per call");
        int grid = 0;
        if (const char *why = resident_blocker(nets[0], num_ticks, &grid))
            return fail(RANC_EUNSUPPORTED, "%s", why);
    }
    for (int i = 0; i < num_nets; ++i)
        for (int j = 0; j < i; ++j)
            if (nets[i] == nets[j])
                return fail(RANC_EINVAL, "nets[%d] and nets[%d] are the same network", j, i);
    hipStream_t s = (hipStream_t)stream;
    std::vector<const uint32_t *> bases(num_nets, nullptr);
    for (int i = 0; i < num_nets; ++i) {
        ranc_net *net = nets[i];
        const Plan &p = net->p;
        const uint32_t *base = inputs ? inputs[i] : nullptr;
        const size_t tick_words = (size_t)p.Cin * p.W;
        if (base && p.Cin > 0 && !(flags & RANC_INPUTS_ON_DEVICE)) {
            uint32_t *stage = (uint32_t *)(net->ws + p.off[R_EXT]);
            hipError_t e = hipMemcpyAsync(stage, base, (size_t)p.S * num_ticks * tick_words * 4,
                                          hipMemcpyHostToDevice, s);
            if (e != hipSuccess)
                return hip_fail(e, "staging inputs");
            base = stage;
        }
        if (p.Cin == 0)
            base = nullptr;
        bases[i] = base;
    }
    if (num_nets > 1) {
        ranc_status st = run_batch(nets, num_nets, bases.data(), num_ticks, (flags & RANC_RUN_GRAPH) != 0,
                                   (flags & RANC_BATCH_PERSISTENT) != 0, s);
        if (st != RANC_OK)
            return st;
    } else {
        ranc_status st = (flags & RANC_RUN_RESIDENT) ? run_resident(nets[0], bases[0], num_ticks, s)
                         : (flags & RANC_RUN_GRAPH)  ? run_captured(nets[0], bases[0], num_ticks, s)
                                                     : queue_ticks(nets[0], bases[0], num_ticks, s, true);
        if (st == RANC_ETIMEOUT) {   // the ticks ran partially: the call counts as run
            nets[0]->tick += num_ticks;
            nets[0]->last_stream = s;
            ++nets[0]->version;
        }
        if (st != RANC_OK)
            return st;
    }
    for (int i = 0; i < num_nets; ++i) {
        nets[i]->tick += num_ticks;
        nets[i]->last_stream = s;
        ++nets[i]->version;
    }
    return RANC_OK;
}

static ranc_status sync_net(ranc_net *net)
{
    hipError_t e = hipStreamSynchronize(net->last_stream);
    if (e != hipSuccess)
        return hip_fail(e, "synchronizing");
    return RANC_OK;
}

// Whole-buffer host mirrors, refreshed once per state version: reading many
// samples costs one device-to-host copy.
static ranc_status refresh_mirror(ranc_net *net, const void *src, size_t bytes, void *dst, uint64_t &version,
                                  const char *what)
{
    if (version == net->version)
        return RANC_OK;
    ranc_status st = sync_net(net);
    if (st != RANC_OK)
        return st;
    hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(e, what);
    version = net->version;
    return RANC_OK;
}

ranc_status ranc_read_spikes(ranc_net *net, int32_t sample, int64_t tick_begin, int64_t tick_end, ranc_spike *out,
                             int64_t capacity, int64_t *count)
{
    if (!net || !count)
        return fail(RANC_EINVAL, "net or count is NULL");
    const Plan &p = net->p;
    if (sample < 0 || sample >= p.S)
        return fail(RANC_EINVAL, "sample %d out of range", sample);
    const int64_t lo = std::max<int64_t>(0, net->tick - p.RT);
    if (tick_begin < lo || tick_end > net->tick || tick_begin > tick_end)
        return fail(RANC_ESTATE, "ticks [%lld, %lld) outside the retained window [%lld, %lld)",
                    (long long)tick_begin, (long long)tick_end, (long long)lo, (long long)net->tick);
    const bool mf = p.path != RANC_PATH_PLAIN;   // sample-tiled paths: neuron-major raster
    const size_t HG = (size_t)p.S64 / 64;
    net->raster_host.resize(mf ? (size_t)p.RT * p.Nout * HG * 2 : (size_t)p.RT * p.S * p.Wout);
    ranc_status st = refresh_mirror(net, net->dn.raster, net->raster_host.size() * 4, net->raster_host.data(),
                                    net->raster_version, "reading the raster");
    if (st != RANC_OK)
        return st;
    int64_t k = 0;
    auto emit = [&](int64_t t, int core, int neuron) {
        if (out && k < capacity) {
            out[k].tick = t;
            out[k].core = core;
            out[k].neuron = neuron;
        }
        ++k;
    };
    if (mf) {
        // neuron-major words of 64 samples; on the MFMA path the bit of a
        // sample inverts the spike-word order sigma(b) = 8((b%16)/4) + 4(b/16)
        // + b%4, on the sparse path it is the sample's index in its tile
        const int i = sample % 32;
        const int bit = p.path == RANC_PATH_SPARSE ? sample % 64
                                                   : 32 * ((sample % 64) / 32) + 16 * ((i % 8) / 4) + 4 * (i / 8) + i % 4;
        const uint64_t *r64 = reinterpret_cast<const uint64_t *>(net->raster_host.data());
        for (int64_t t = tick_begin; t < tick_end; ++t) {
            const uint64_t *row = r64 + (size_t)(t % p.RT) * p.Nout * HG + sample / 64;
            // 64 output neurons at a time: gather their bits into one mask
            // without branches, then emit the set bits in order
            for (int o0 = 0; o0 < p.Nout; o0 += 64) {
                const int n = std::min(64, p.Nout - o0);
                uint64_t m = 0;
                for (int j = 0; j < n; ++j)
                    m |= ((row[(size_t)(o0 + j) * HG] >> bit) & 1u) << j;
                while (m) {
                    const int o = o0 + __builtin_ctzll(m);
                    m &= m - 1;
                    emit(t, net->out_neurons[2 * o], net->out_neurons[2 * o + 1]);
                }
            }
        }
    } else {
        for (int64_t t = tick_begin; t < tick_end; ++t) {
            const uint32_t *row = net->raster_host.data() + ((size_t)(t % p.RT) * p.S + sample) * p.Wout;
            for (int ow = 0; ow < p.Wout; ++ow) {
                uint32_t w = row[ow];
                while (w) {
                    const int b = __builtin_ctz(w);
                    w &= w - 1;
                    emit(t, net->out_words[2 * ow], net->out_words[2 * ow + 1] * 32 + b);
                }
            }
        }
    }
    *count = k;
    if (k > capacity)
        return fail(RANC_ETRUNC, "%lld spikes do not fit capacity %lld", (long long)k, (long long)capacity);
    return RANC_OK;
}

ranc_status ranc_raster_bytes(const ranc_net *net, int64_t num_ticks, uint32_t layout, size_t *bytes)
{
    if (!net || !bytes)
        return fail(RANC_EINVAL, "net or bytes is NULL");
    if (num_ticks < 0)
        return fail(RANC_EINVAL, "num_ticks %lld < 0", (long long)num_ticks);
    const Plan &p = net->p;
    if (layout == RANC_RASTER_BY_NEURON)
        *bytes = (size_t)num_ticks * p.Nout * (p.S64 / 64) * 8;
    else if (layout == RANC_RASTER_BY_SAMPLE)
        *bytes = (size_t)num_ticks * p.S * ((p.Nout + 31) / 32) * 4;
    else
        return fail(RANC_EINVAL, "unknown raster layout %u", layout);
    return RANC_OK;
}

ranc_status ranc_copy_raster(ranc_net *net, int64_t tick_begin, int64_t tick_end, uint32_t layout, void *dst,
                             size_t dst_bytes, void *stream)
{
    if (!net || !dst)
        return fail(RANC_EINVAL, "net or dst is NULL");
    if (layout != RANC_RASTER_BY_NEURON && layout != RANC_RASTER_BY_SAMPLE)
        return fail(RANC_EINVAL, "unknown raster layout %u", layout);
    const Plan &p = net->p;
    const int64_t lo = std::max<int64_t>(0, net->tick - p.RT);
    if (tick_begin < lo || tick_end > net->tick || tick_begin >= tick_end)
        return fail(RANC_ESTATE, "ticks [%lld, %lld) empty or outside the retained window [%lld, %lld)",
                    (long long)tick_begin, (long long)tick_end, (long long)lo, (long long)net->tick);
    size_t need = 0;
    ranc_raster_bytes(net, tick_end - tick_begin, layout, &need);
    if (dst_bytes < need)
        return fail(RANC_ENOMEM, "dst has %zu bytes, needs %zu", dst_bytes, need);
    hipError_t e = launch_pack_raster(net->dn, net->outcol, net->opos, layout == RANC_RASTER_BY_SAMPLE, tick_begin,
                                      (int)(tick_end - tick_begin), dst, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "packing the output raster");
    return RANC_OK;
}

ranc_status ranc_output_neurons(const ranc_net *net, int32_t *out, int64_t capacity, int64_t *count)
{
    if (!net || !count)
        return fail(RANC_EINVAL, "net or count is NULL");
    const int64_t n = (int64_t)net->out_neurons.size() / 2;
    *count = n;
    if (capacity < n)
        return fail(RANC_ETRUNC, "%lld output neurons do not fit capacity %lld", (long long)n, (long long)capacity);
    if (n && !out)
        return fail(RANC_EINVAL, "out is NULL");
    memcpy(out, net->out_neurons.data(), (size_t)n * 2 * sizeof(int32_t));
    return RANC_OK;
}

ranc_status ranc_read_potentials(ranc_net *net, int32_t sample, int32_t *out)
{
    if (!net || !out)
        return fail(RANC_EINVAL, "net or out is NULL");
    const Plan &p = net->p;
    if (sample < 0 || sample >= p.S)
        return fail(RANC_EINVAL, "sample %d out of range", sample);
    const bool brick = net->dn.vlayout == VLAYOUT_BRICK;
    const size_t SV = net->dn.vlayout == VLAYOUT_CSN ? (size_t)p.S : (size_t)p.S64;
    net->v_host.resize((size_t)p.C * SV * p.N);
    ranc_status st = refresh_mirror(net, net->dn.V, net->v_host.size() * 4, net->v_host.data(), net->v_version,
                                    "reading potentials");
    if (st != RANC_OK)
        return st;
    if (net->dn.vlayout == VLAYOUT_SPARSE) {   // [C][N][S64]
        for (size_t cj = 0; cj < (size_t)p.C * p.N; ++cj)
            out[cj] = net->v_host[cj * SV + sample];
        return RANC_OK;
    }
    if (!brick) {
        for (int c = 0; c < p.C; ++c)
            memcpy(out + (size_t)c * p.N, net->v_host.data() + ((size_t)c * SV + sample) * p.N, (size_t)p.N * 4);
        return RANC_OK;
    }
    // brick (c, nb, g): element (q, lane l, e) = sample 32g + 8q + 4(l/32) + e, neuron 32nb + l%32
    const int NB = p.N / 32;
    const size_t groups = (size_t)p.S64 / 32;
    const int g = sample / 32, i = sample % 32, q = i / 8, hh = (i % 8) / 4, e = i % 4;
    for (int c = 0; c < p.C; ++c)
        for (int nb = 0; nb < NB; ++nb)
            for (int jj = 0; jj < 32; ++jj)
                out[(size_t)c * p.N + nb * 32 + jj] =
                    net->v_host[(((((size_t)c * NB + nb) * groups + g) * 4 + q) * 64 + 32 * hh + jj) * 4 + e];
    return RANC_OK;
}

ranc_status ranc_read_counters(ranc_net *net, int32_t sample, ranc_counters *out)
{
    if (!net || !out)
        return fail(RANC_EINVAL, "net or out is NULL");
    const Plan &p = net->p;
    if (sample < 0 || sample >= p.S)
        return fail(RANC_EINVAL, "sample %d out of range", sample);
    const int rows = p.C * net->dn.cnt_rows;   // counter rows: per core, 64-neuron block (plain) or slice (MFMA)
    net->cnt_host.resize((size_t)rows * p.S * CNT_N);
    ranc_status st = refresh_mirror(net, net->dn.cnt, net->cnt_host.size() * 8, net->cnt_host.data(),
                                    net->cnt_version, "reading counters");
    if (st != RANC_OK)
        return st;
    unsigned long long sum[CNT_N] = {0, 0, 0, 0, 0};
    for (int c = 0; c < rows; ++c)
        for (int k = 0; k < CNT_N; ++k)
            sum[k] += net->cnt_host[((size_t)c * p.S + sample) * CNT_N + k];
    out->emitted = sum[CNT_EMITTED];
    out->routed = sum[CNT_ROUTED];
    out->delivered = sum[CNT_DELIVERED];
    out->out = sum[CNT_OUT];
    out->events = sum[CNT_EVENTS];
    return RANC_OK;
}

ranc_status ranc_link_counts_enable(ranc_net *net, int32_t enable)
{
    if (!net)
        return fail(RANC_EINVAL, "net is NULL");
    if (enable != 0 && enable != 1)
        return fail(RANC_EINVAL, "enable must be 0 or 1");
    if (net->links_on != (enable == 1)) {
        drop_graphs(net);
        net->links_on = enable == 1;
    }
    return RANC_OK;
}

ranc_status ranc_read_links(ranc_net *net, int32_t sample, int64_t *out)
{
    if (!net || !out)
        return fail(RANC_EINVAL, "net or out is NULL");
    const Plan &p = net->p;
    if (sample < 0 || sample >= p.S)
        return fail(RANC_EINVAL, "sample %d out of range", sample);
    net->links_host.resize((size_t)4 * p.C * p.S64);
    ranc_status st = refresh_mirror(net, net->lk.d, net->links_host.size() * 8, net->links_host.data(),
                                    net->links_version, "reading mesh link counts");
    if (st != RANC_OK)
        return st;
    // difference arrays [dir][core][S64] -> counts: prefix sums along each
    // mesh row (+x ascending x, -x descending), column (+y, -y)
    const int gw = p.grid_w, gh = p.grid_h;
    auto dv = [&](int dir, int core) { return net->links_host[((size_t)dir * p.C + core) * p.S64 + sample]; };
    for (int y = 0; y < gh; ++y) {
        long long up = 0, down = 0;
        for (int x = 0; x < gw; ++x) {
            up += dv(RANC_LINK_XPLUS, y * gw + x);
            out[(size_t)(y * gw + x) * 4 + RANC_LINK_XPLUS] = up;
            const int xr = gw - 1 - x;
            down += dv(RANC_LINK_XMINUS, y * gw + xr);
            out[(size_t)(y * gw + xr) * 4 + RANC_LINK_XMINUS] = down;
        }
    }
    for (int x = 0; x < gw; ++x) {
        long long up = 0, down = 0;
        for (int y = 0; y < gh; ++y) {
            up += dv(RANC_LINK_YPLUS, y * gw + x);
            out[(size_t)(y * gw + x) * 4 + RANC_LINK_YPLUS] = up;
            const int yr = gh - 1 - y;
            down += dv(RANC_LINK_YMINUS, yr * gw + x);
            out[(size_t)(yr * gw + x) * 4 + RANC_LINK_YMINUS] = down;
        }
    }
    return RANC_OK;
}

ranc_status ranc_current_tick(const ranc_net *net, int64_t *tick)
{
    if (!net || !tick)
        return fail(RANC_EINVAL, "net or tick is NULL");
    *tick = net->tick;
    return RANC_OK;
}

ranc_status ranc_get_path(const ranc_net *net, int32_t *path)
{
    if (!net || !path)
        return fail(RANC_EINVAL, "net or path is NULL");
    *path = net->p.path;
    return RANC_OK;
}

ranc_status ranc_profile_enable(ranc_net *net, int32_t enable)
{
    if (!net)
        return fail(RANC_EINVAL, "net is NULL");
    if (enable) {
        ranc_status st = sync_net(net);
        if (st != RANC_OK)
            return st;
        net->prof.used.clear();
        for (int k = 0; k < 4; ++k) {
            net->prof.ms[k] = 0;
            net->prof.launches[k] = 0;
        }
    }
    net->prof.on = enable != 0;
    return RANC_OK;
}

ranc_status ranc_profile_read(ranc_net *net, ranc_profile *out)
{
    if (!net || !out)
        return fail(RANC_EINVAL, "net or out is NULL");
    ranc_status st = sync_net(net);
    if (st != RANC_OK)
        return st;
    hipError_t e = prof_collect(net);
    if (e != hipSuccess)
        return hip_fail(e, "reading kernel timings");
    out->integrate_ms = net->prof.ms[0];
    out->route_ms = net->prof.ms[1];
    out->integrate_launches = net->prof.launches[0];
    out->route_launches = net->prof.launches[1];
    out->graph_ms = net->prof.ms[2];
    out->graph_launches = net->prof.launches[2];
    out->graphs_held = (int64_t)net->loops.size();
    out->graphs_dropped = (int64_t)net->loops_dropped;
    out->resident_ms = net->prof.ms[3];
    out->resident_launches = net->prof.launches[3];
    return RANC_OK;
}

ranc_status ranc_reset_state(ranc_net *net, void *stream)
{
    if (!net)
        return fail(RANC_EINVAL, "net is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_reset_state(net->dn, net->lk, s);
    if (e != hipSuccess)
        return hip_fail(e, "resetting state");
    net->tick = 0;
    net->last_stream = s;
    ++net->version;
    net->state_lost = false;
    return RANC_OK;
}

// Launch-shape autotuner: time every candidate shape of the handle's path on
// num_ticks ticks of the given inputs and keep the fastest.
static void drop_graphs(ranc_net *net)
{
    for (auto &g : net->loops) {
        hipGraphExecDestroy(g.exec);
        hipGraphDestroy(g.graph);
    }
    net->loops.clear();
    if (net->batch.exec)
        hipGraphExecDestroy(net->batch.exec);
    if (net->batch.graph)
        hipGraphDestroy(net->batch.graph);
    net->batch = Batch();
}

ranc_status ranc_autotune(ranc_net *net, const uint32_t *inputs, uint32_t flags, int32_t num_ticks, void *stream,
                          ranc_tune *out)
{
    if (!net || !out)
        return fail(RANC_EINVAL, "net or out is NULL");
    if (num_ticks < 1 || num_ticks > net->p.RT)
        return fail(RANC_EINVAL, "num_ticks %d outside [1, max_ticks_per_call=%d]", num_ticks, net->p.RT);
    if (flags & ~RANC_INPUTS_ON_DEVICE)
        return fail(RANC_EINVAL, "unknown flags 0x%x", flags);
    hipStream_t s = (hipStream_t)stream;
    Plan &p = net->p;
    struct Cand {
        int spw;
        RouteCfg rc;
    };
    std::vector<Cand> cands;
    if (p.path != RANC_PATH_PLAIN) {
        const int tiles = (p.S + 63) / 64;
        int last_chunks = -1;
        const int cap = p.path == RANC_PATH_SPARSE ? sparse_max_samples_per_wg() : mfma_max_samples_per_wg();
        for (int spw = 64; spw <= cap; spw *= 2) {
            const int chunks = (tiles * 64 + spw - 1) / spw;
            if (chunks == last_chunks)
                break;
            last_chunks = chunks;
            cands.push_back({spw, net->rcfg});
        }
    } else {
        const RouteCfg def = route_default_cfg(net->dn);
        const int dmax = route_dmax(p.D);
        for (int sb = 1; sb <= 8; sb *= 2) {
            if (sb * dmax > 32 || (sb > 1 && sb > p.S))
                continue;
            const size_t bitmap = (size_t)p.C * p.NW * 4 * sb;
            const int groups = (p.S + sb - 1) / sb;
            const int max_split = std::max(1, (p.C * p.W + 255) / 256);
            int base = std::max(1, std::min(max_split, (2048 + groups - 1) / groups));
            for (int f = 0; f < 3; ++f) {
                const int split = f == 0 ? std::max(1, base / 2) : f == 1 ? base : std::min(max_split, base * 2);
                if (f > 0 && split == (f == 1 ? std::max(1, base / 2) : base))
                    continue;
                for (int stage = 0; stage <= 1; ++stage) {
                    if (stage && bitmap > 128 * 1024)
                        continue;
                    if ((p.S + sb - 1) / sb > 65535)
                        continue;
                    RouteCfg rc;
                    rc.samples_per_block = sb;
                    rc.blocks_per_group = split;
                    rc.stage = stage;
                    rc.lanes = 1;
                    cands.push_back({p.spw, rc});
                }
            }
        }
        if (p.S <= 65535) {
            // the lane-split router (one sample per block row; the fields
            // above do not apply to it), once
            RouteCfg rc = def;
            rc.lanes = route_split_lanes();
            cands.push_back({p.spw, rc});
        }
        if (cands.empty())
            cands.push_back({p.spw, def});
    }
    const uint32_t *base = inputs;
    if (base && p.Cin > 0 && !(flags & RANC_INPUTS_ON_DEVICE)) {
        uint32_t *stage = (uint32_t *)(net->ws + p.off[R_EXT]);
        hipError_t e = hipMemcpyAsync(stage, base, (size_t)p.S * num_ticks * p.Cin * p.W * 4,
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return hip_fail(e, "staging inputs");
        base = stage;
    }
    if (p.Cin == 0)
        base = nullptr;
    drop_graphs(net);
    const bool prof_on = net->prof.on;
    net->prof.on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    double best = -1.0;
    Cand best_c = cands[0];
    ranc_status st = RANC_OK;
    for (const Cand &c : cands) {
        if (e != hipSuccess || st != RANC_OK)
            break;
        p.spw = c.spw;
        net->rcfg = c.rc;
        // one untimed pass, then a timed pass, each from the initial state
        e = launch_reset_state(net->dn, net->lk, s);
        if (e == hipSuccess && (st = queue_ticks(net, base, num_ticks, s, false)) == RANC_OK)
            e = launch_reset_state(net->dn, net->lk, s);
        if (e == hipSuccess && st == RANC_OK)
            e = hipEventRecord(e0, s);
        if (e == hipSuccess && st == RANC_OK && (st = queue_ticks(net, base, num_ticks, s, false)) == RANC_OK)
            e = hipEventRecord(e1, s);
        if (e == hipSuccess && st == RANC_OK)
            e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess && st == RANC_OK)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && st == RANC_OK && (best < 0 || ms < best)) {
            best = ms;
            best_c = c;
        }
    }
    if (e0)
        hipEventDestroy(e0);
    if (e1)
        hipEventDestroy(e1);
    p.spw = best_c.spw;
    net->rcfg = best_c.rc;
    net->prof.on = prof_on;
    if (st != RANC_OK)
        return st;
    if (e == hipSuccess)
        e = launch_reset_state(net->dn, net->lk, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "autotuning");
    net->tick = 0;
    net->last_stream = s;
    ++net->version;
    const bool tiled = p.path != RANC_PATH_PLAIN;
    out->samples_per_wg = tiled ? p.spw : 0;
    out->route_samples_per_block = tiled ? 0 : net->rcfg.samples_per_block;
    out->route_split = tiled ? 0 : net->rcfg.blocks_per_group;
    out->route_stage = tiled ? 0 : net->rcfg.stage;
    out->ms_per_tick = best / num_ticks;
    out->candidates = (int32_t)cands.size();
    out->route_lanes_per_word = tiled ? 0 : net->rcfg.lanes;
    return RANC_OK;
}

ranc_status ranc_set_launch_shape(ranc_net *net, const ranc_tune *shape)
{
    if (!net || !shape)
        return fail(RANC_EINVAL, "net or shape is NULL");
    const Plan &p = net->p;
    if (p.path != RANC_PATH_PLAIN) {
        const int v = shape->samples_per_wg;
        const int cap = p.path == RANC_PATH_SPARSE ? sparse_max_samples_per_wg() : mfma_max_samples_per_wg();
        if (v <= 0 || v % 64 || v > cap)
            return fail(RANC_EINVAL, "samples_per_wg %d must be a multiple of 64 in [64, %d]", v, cap);
        drop_graphs(net);
        net->p.spw = v;
        return RANC_OK;
    }
    RouteCfg rc;
    rc.samples_per_block = shape->route_samples_per_block;
    rc.blocks_per_group = shape->route_split;
    rc.stage = shape->route_stage != 0;
    const int sb = rc.samples_per_block;
    if ((sb != 1 && sb != 2 && sb != 4 && sb != 8) || sb * route_dmax(p.D) > 32)
        return fail(RANC_EINVAL, "route_samples_per_block %d unsupported with max delay %d", sb, p.D);
    if (rc.blocks_per_group < 1)
        return fail(RANC_EINVAL, "route_split must be >= 1");
    if (rc.stage && (size_t)p.C * p.NW * 4 * sb > 128 * 1024)
        return fail(RANC_EINVAL, "staged spike bitmaps of %d samples exceed the router's LDS", sb);
    if ((p.S + sb - 1) / sb > 65535)
        return fail(RANC_EINVAL, "too many sample groups for the router grid");
    const int lanes = shape->route_lanes_per_word;
    if (lanes != 0 && lanes != 1 && lanes != route_split_lanes())
        return fail(RANC_EINVAL, "route_lanes_per_word %d must be 0 (automatic), 1 or %d", lanes,
                    route_split_lanes());
    rc.lanes = lanes ? lanes : route_auto_lanes(net->dn, rc);
    if (rc.lanes != 1 && p.S > 65535)
        return fail(RANC_EINVAL, "the lane-split router takes at most 65535 samples");
    drop_graphs(net);
    net->rcfg = rc;
    return RANC_OK;
}

ranc_status ranc_get_launch_shape(const ranc_net *net, ranc_tune *out)
{
    if (!net || !out)
        return fail(RANC_EINVAL, "net or out is NULL");
    const bool mf = net->p.path != RANC_PATH_PLAIN;
    out->samples_per_wg = mf ? net->p.spw : 0;
    out->route_samples_per_block = mf ? 0 : net->rcfg.samples_per_block;
    out->route_split = mf ? 0 : net->rcfg.blocks_per_group;
    out->route_stage = mf ? 0 : net->rcfg.stage;
    out->ms_per_tick = 0.0;
    out->candidates = 0;
    out->route_lanes_per_word = mf ? 0 : net->rcfg.lanes;
    return RANC_OK;
}

void ranc_free(ranc_net *net)
{
    if (!net)
        return;
    hipStreamSynchronize(net->last_stream);
    drop_graphs(net);
    if (net->cap_stream)
        hipStreamDestroy(net->cap_stream);
    for (int i = 0; i < ranc_net::BATCH_BRANCHES; ++i) {
        if (net->br_stream[i])
            hipStreamDestroy(net->br_stream[i]);
        if (net->br_join[i])
            hipEventDestroy(net->br_join[i]);
    }
    if (net->br_fork)
        hipEventDestroy(net->br_fork);
    for (auto &e : net->prof.pool) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    if (net->static_dev >= 0)
        static_ws_release(net->static_dev);
    delete net;
}

}  // extern "C"
