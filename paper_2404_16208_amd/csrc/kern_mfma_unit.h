// kern_mfma_unit.h -- the MFMA path's work unit (one workgroup's share of
// a tick: delivery, integration on int8 MFMA, leak/threshold/reset, and the
// scheduler write; described in kern_mfma.hip) and its kernel templates,
// shared by kern_mfma.hip, which instantiates them with the B tiles read
// from the int8 weight planes, and kern_mfma_cb.hip, which instantiates them
// with the B tiles built from the compact crossbar. The two forms live in
// separate translation units: instantiated side by side in one, the plane
// form's code came out slightly different (an add folded differently,
// registers renumbered) and its tick on the 512-core net at 1024 samples ran
// 0.9% slower.
#pragma once
#include "kern_common.h"
#include "kern_bits.h"
#include "ranc_internal.h"

namespace ranc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

static constexpr int MFMA_TS = 64;        // samples per tile
static constexpr int MFMA_SPW_MAX = 512;  // samples per workgroup (LDS counters)

// s_waitcnt immediates (gfx9 encoding: vmcnt in [3:0] and [15:14], expcnt in
// [6:4], lgkmcnt in [11:8]): wait for all vector-memory operations / all LDS
// operations of this wave.
static constexpr int WAIT_VMCNT0 = 0x0F70;
static constexpr int WAIT_LGKMCNT0 = 0xC07F;

typedef __attribute__((address_space(3))) void lds_void;

// cache-policy bits of a global-to-LDS load: non-temporal
static constexpr int CPOL_NT = 2;


template <bool WIDE> struct RawWord { typedef uint32_t type; };
template <> struct RawWord<true> { typedef uint64_t type; };

// Compact B source (DevNet::colbits on this path): the crossbar as
// column words [C][W][N] (bit a % 32 of word a / 32 of neuron j: axon a
// connects to j), then each neuron's plane values by axon type, [C][planes]
// [2][N] words (byte g % 4 of word g / 4: the plane's value of the neuron's
// weight for type g), then the axon types, [C][A] bytes.
__device__ inline const uint32_t *mfma_bsrc_wsel(const DevNet &n)
{
    return n.colbits + (size_t)n.C * n.W * n.N;
}
__device__ inline const uint8_t *mfma_bsrc_types(const DevNet &n, int planes)
{
    return reinterpret_cast<const uint8_t *>(mfma_bsrc_wsel(n) + (size_t)n.C * planes * 2 * n.N);
}

// LDS of one workgroup, by shape.
template <int A_, int N_> struct MfmaLds {
    static constexpr int STW = N_ / 128;   // 32-sample sub-tiles per wave per tile
    static constexpr int ROWB = A_ + 16;   // padded LDS row of the int8 tile (bytes)
    static constexpr int XW = A_ / 32 + 1; // padded axon words per sample
    typedef int8_t ATile[MFMA_TS * ROWB];  // int8 axon spikes of a tile (x2, double buffer)
    typedef v4i VTile[STW][4][64];         // next tile's potentials (one per wave)
    typedef uint32_t XTile[MFMA_TS][XW];   // delivered axon words of a tile (x2)
    // this tick's history words of the workgroup's neurons, collected over HB
    // tiles and written to memory in 64-byte runs per neuron (two batches in
    // flight when two wavefronts share a neuron's words)
    static constexpr int HB = A_ == 512 ? 4 : 8;
    static constexpr int HBS = STW == 1 ? 2 * HB : HB;
    typedef uint64_t HBuf[N_][HBS];
    // plane split (A = 512 with two weight planes): the partial sums one
    // wavefront hands to its partner, [wave][accumulator element][lane]
    typedef int32_t Xch[8][16][64];
};

// One unit of work: workgroup `bid` of the tick's grid (core bid % C, then
// neuron slice and sample chunk), on 512 threads. N_ is the slice width: a
// core of 512 neurons runs as two slices of 256, each with its own B tiles,
// degree counts and counter row, sharing the axon inputs of the core; a core
// of 64 neurons runs as a slice of 128 whose upper two 32-neuron blocks are
// dead (their wavefronts keep their gather and expansion roles and the
// barriers, and skip all neuron work and memory traffic).
// Plane split (A = 512 with two weight planes, 128-neuron slices): the B
// tiles of both planes would take 128 VGPRs per lane, so the two wavefronts
// of a 32-neuron block hold one plane each (wave stg: plane stg, hi first),
// each multiplies both 32-sample groups of the tile with its plane, and they
// swap the partial sums of one group through LDS (`xch`): wave stg finishes
// group stg with in = lo + 128 * hi. The LDS arrays come from the calling
// kernel, so several shapes can share one kernel's LDS.
// EXT: the extended potential update (lif_update): potentials narrower than
// 32 bits are clamped to [vmin, vmax] after the saturating 32-bit add (with
// 32-bit potentials the add alone is exact), and the floor and linear-reset
// options apply; without them the epilogue is the add, compare and select.
// HBUF: history words are collected in `hbuf` and written in runs of HB
// words per neuron; otherwise each tile's word is stored at once.
// CB: the B tiles are built from the compact crossbar (mfma_bsrc_*), else
// read from the int8 weight planes.
template <int A_, int N_, bool TWO, bool EXT, bool HBUF, bool CB>
__device__ __forceinline__ void integrate_mfma_unit(const DevNet &n, const TickArgs &ta, int spw, int bid,
                                                    typename MfmaLds<A_, N_>::ATile *a_lds,
                                                    typename MfmaLds<A_, N_>::VTile *v_lds,
                                                    typename MfmaLds<A_, N_>::XTile *x_lds,
                                                    typename MfmaLds<A_, N_>::HBuf *hbuf,
                                                    typename MfmaLds<A_, N_>::Xch *xch,
                                                    unsigned (*s_cnt)[MFMA_SPW_MAX])
{
    typedef MfmaLds<A_, N_> L;
    constexpr int NB = N_ / 32;          // 32-neuron blocks (4 or 8)
    constexpr int KS = A_ / 32;          // 32-axon k-steps
    constexpr bool PSPLIT = TWO && A_ == 512;   // one plane per wavefront
    static_assert(!PSPLIT || N_ == 128, "the plane split pairs the two wavefronts of a block");
    constexpr int PLY = TWO ? 2 : 1;     // B planes in the layout
    constexpr int PL = PSPLIT ? 1 : PLY; // B planes held by a wavefront
    constexpr int STW = NB / 4;          // 32-sample sub-tiles per wave per tile
    constexpr int W_ = A_ / 32;          // axon words
    constexpr int ROWB = A_ + 16;        // padded LDS row of the int8 tile (bytes)
    constexpr int WPW = (W_ + 7) / 8;    // axon words expanded per wave
    constexpr int APW = A_ / 64;         // 64-axon blocks of the gather
    constexpr int GPW = APW == 8 ? 2 : 1;  // 32-sample groups gathered per wave
    typedef typename RawWord<GPW == 2>::type RawT;
    static_assert(NB == 4 || NB == 8, "N must be 128 or 256");

    // s_cnt, per sample of the chunk: [0] emitted | routed << 10 | out << 20
    // (each <= N per tick), [1] events | delivered << 18 (<= 512*256, <= 512)

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // unit v = slice + slices * chunk of core c, XCD-grouped (core_unit_of)
    int c, v;
    core_unit_of(bid, n.C, n.slices * ((n.S + spw - 1) / spw), c, v);
    const int slice = v % n.slices;
    const int chunk = v / n.slices;
    const int s_begin = chunk * spw;
    const int s_end = min(n.S, s_begin + spw);
    const int h = lane >> 5, jj = lane & 31;
    const int sig = sigma32(jj);
    const int nb = wave % NB;
    const int stg = wave / NB;
    // wave-uniform; only 128-wide workgroups (64-neuron cores) have dead blocks
    const bool live = N_ == 256 || slice * NB + nb < n.NW;
    const int nbu = live ? nb : 0;         // block whose addresses a dead wave computes (never used)
    const int neuron = nbu * 32 + jj;      // within the slice
    const int nbc = slice * NB + nbu;      // 32-neuron block within the core

    for (int i = threadIdx.x; i < 2 * MFMA_SPW_MAX; i += blockDim.x)
        (&s_cnt[0][0])[i] = 0u;

    // B tiles of this wave's neuron block, resident for the whole chunk. With
    // one sample chunk per core (a sweep of 64-sample networks) every
    // workgroup reads its core's B source once per tick, and the int8 planes
    // (A*N bytes per plane and core) were a third of the tick's bytes; there
    // they are built from the compact crossbar instead (A*N/8 bytes of
    // column words per core): byte b of k-step k is the plane value of
    // weight(neuron, type(axon)) where the axon connects, else 0, v_perm_b32
    // picking byte `type` of the neuron's 8 per-type plane bytes, or zero for
    // selector 0x0C. With several chunks per core the planes are read from
    // L2 by the core's other workgroups, and loading them is 0.5% faster
    // (1024 samples).
    v4i breg[KS][PL];
    if constexpr (CB) {
        const int jc = nbc * 32 + jj;   // neuron within the core
        const uint32_t *colw = n.colbits + (size_t)c * W_ * n.N + jc;
        const uint32_t *wsel = mfma_bsrc_wsel(n) + (size_t)c * PLY * 2 * n.N + jc;
        const uint4 *ts = reinterpret_cast<const uint4 *>(mfma_bsrc_types(n, PLY) + (size_t)c * A_) + h;
        uint32_t wl[PL], wh[PL];
#pragma unroll
        for (int p = 0; p < PL; ++p) {
            const int pp = PSPLIT ? stg : p;
            wl[p] = wsel[(size_t)(2 * pp) * n.N];       // types 0..3
            wh[p] = wsel[(size_t)(2 * pp + 1) * n.N];   // types 4..7
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const uint32_t bits = colw[(size_t)k * n.N] >> (16 * h);   // axons 32k + 16h + [0, 16)
            const uint4 t4 = ts[2 * k];
            const uint32_t tq[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // bit i of the nibble (axon 32k + 16h + 4q + i connects) to
                // bit 2 of byte i (one 24-bit multiply: the four shifted
                // copies do not overlap), then byte i of the index = i, or
                // 4 + i where the axon connects
                const uint32_t spread = ((bits >> (4 * q)) & 15u) * 0x00810204u;
                const uint32_t idx = (spread & 0x04040404u) | 0x03020100u;
                // byte i: the axon's type (byte i of tq), or 0x0C where it does not connect
                const uint32_t sel = __builtin_amdgcn_perm(tq[q], 0x0C0C0C0Cu, idx);
#pragma unroll
                for (int p = 0; p < PL; ++p)
                    breg[k][p][q] = (int)__builtin_amdgcn_perm(wh[p], wl[p], sel);
            }
        }
    } else {
        const v4i *planes = reinterpret_cast<const v4i *>(n.planes);
#pragma unroll
        for (int k = 0; k < KS; ++k)
#pragma unroll
            for (int p = 0; p < PL; ++p)
                breg[k][p] = planes[((((size_t)c * n.NW + nbc) * KS + k) * PLY + (PSPLIT ? stg : p)) * 64 + lane];
    }
    const size_t cj = (size_t)c * n.N + slice * N_ + neuron;
    const int32_t lk = n.leak[cj], th = n.thr[cj], rs = n.rst[cj];
    const int32_t vmin = n.vmin, vmax = n.vmax;
    int32_t fl = vmin;
    bool lin = false;
    if constexpr (EXT) {
        fl = n.floor[cj];
        lin = (n.linmask[cj >> 5] >> (cj & 31)) & 1u;
    }
    const int oi = n.outidx[cj];
    const uint32_t cm32 = n.coremask[(size_t)c * n.NW + nbc];
    const uint32_t om32 = n.outmask[(size_t)c * n.NW + nbc];

    // Connected-neuron counts (neurons of the slice) of this wave's expansion
    // words, low and high bytes, 4 axons per word, for the dot4 event count.
    const size_t dg = (size_t)c * n.slices + slice;
    uint32_t degl[WPW][8], degh[WPW][8];
    bool any_hi = false;
#pragma unroll
    for (int k = 0; k < WPW; ++k) {
        const int wi = wave + 8 * k;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            degl[k][q] = wi < W_ ? n.degb[(dg * 2 + 0) * (A_ / 4) + wi * 8 + q] : 0u;
            degh[k][q] = wi < W_ ? n.degb[(dg * 2 + 1) * (A_ / 4) + wi * 8 + q] : 0u;
            any_hi |= degh[k][q] != 0u;
        }
    }

    const int ci = n.in_index[c];
    const uint32_t *ext_c = (ta.ext_t != nullptr && ci >= 0) ? ta.ext_t + (size_t)ci * W_ : nullptr;
    const int q_now = tick_slot(n, ta.k), r_row = tick_row(n, ta.k);
    const size_t G32 = (size_t)n.S64 / 32;   // 32-sample groups
    const size_t HG = (size_t)n.S64 / 64;    // 64-sample history words per neuron
    const size_t vbase = ((size_t)c * n.NW + nbc) * G32 * 256 + lane;
    const v4i *vb_in = reinterpret_cast<const v4i *>(n.V) + vbase;
    v4i *vb_out = reinterpret_cast<v4i *>(n.V) + vbase;
    const size_t CN = (size_t)n.C * n.N;
    uint64_t *hist_out = n.hist + ((size_t)q_now * CN + cj) * HG;
    uint64_t *rast_out =
        oi >= 0 ? reinterpret_cast<uint64_t *>(n.raster) + ((size_t)r_row * n.Nout + oi) * HG : nullptr;

    // ---- history gather: wave w collects, for axon block w % APW, the
    // history bits of group w / APW of each tile (both groups when A = 512).
    const bool gatherer = wave < 2 * APW;   // wave-uniform
    const int axb = wave % APW;
    const int grp = GPW == 2 ? 0 : wave / APW;
    const int ga = axb * 64 + lane;
    uint32_t e_beg = 0, e_end = 0;
    if (gatherer) {
        e_beg = n.rtx_ptr[(size_t)c * A_ + ga];
        e_end = n.rtx_ptr[(size_t)c * A_ + ga + 1];
    }
    // The first FMAX sources of the axon stay in registers as history rows of
    // (slot of their delay, source neuron); unused ones point at a zero row.
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
    const bool multi = __ballot(e_end - e_beg > 1) != 0;         // wave-uniform
    const bool long_lists = __ballot(e_end - e_beg > FMAX) != 0;  // wave-uniform
    auto raw_word = [&](const uint64_t *row, int tile) -> RawT {
        if constexpr (GPW == 2)
            return row[tile];
        else
            return reinterpret_cast<const uint32_t *>(row + tile)[grp];
    };
    // Each source's word goes straight into a register that carries it to its
    // use one iteration later (no arithmetic on it before then, so the loads
    // stay in flight); sources past the first FMAX (rare) are ORed in at once.
    // Tiles past the chunk load an in-range word that is never used.
    auto load_mask = [&](int s0, RawT (&raw)[FMAX]) {
        const int tile = (s0 < s_end ? s0 : s_begin) / MFMA_TS;
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
    // Lane (h, j) holds, for axon 64*axb + 32h + j, the bits of a 32-sample
    // group; after the transpose lane (h, i) holds the axon word 2*axb + h of
    // the sample of bit i.
    auto transpose_store = [&](RawT m, int buf) {
#pragma unroll
        for (int g = 0; g < GPW; ++g) {
            const uint32_t t = transpose32((uint32_t)(m >> (32 * g)), lane);
            x_lds[buf][32 * (GPW == 2 ? g : grp) + sig][2 * axb + h] = t;
        }
    };
    // external input words of sample s0 + lane (clamped into the chunk; lanes
    // past its end are masked where the words are used)
    uint32_t xe[WPW];
#pragma unroll
    for (int k = 0; k < WPW; ++k)
        xe[k] = 0u;
    auto load_ext = [&](int s0) {
        if (!ext_c)
            return;
        const int s = min(s0 + lane, s_end - 1);
#pragma unroll
        for (int k = 0; k < WPW; ++k) {
            const int wi = wave + 8 * k;
            if (wi < W_)
                xe[k] = ext_c[(size_t)s * ta.ext_sstride + wi];
        }
    };
    // Potentials of a tile go from HBM straight into this wave's LDS region,
    // one tile ahead of their use, as non-temporal (streaming) loads: they are
    // used once per tick, and keeping them out of L2 leaves it to the history
    // words and B sources that other workgroups read again.
    auto prefetch_v = [&](int s0) {
        if (!live)
            return;
#pragma unroll
        for (int t = 0; t < STW; ++t) {
            const int g = (s0 >> 5) + stg * STW + t;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                __builtin_amdgcn_global_load_lds((const void *)(vb_in + ((size_t)g * 4 + q) * 64),
                                                 (lds_void *)&v_lds[wave][t][q][0], 16, 0, CPOL_NT);
        }
        compiler_fence();   // issue now, not later in the iteration
    };

    // results of the previous tile, written at the top of the next iteration
    v4i vnew[STW][4];
    uint32_t hword[STW];   // lanes h = 0: the neuron's 32-sample spike word
    unsigned pcnt[STW];    // lanes h = 0: packed spike counts of sample sigma(jj)
    unsigned pdlev = 0;    // events | delivered << 18 of sample ps0 + lane
    int ps0 = -1;
    auto flush = [&]() {
        if (ps0 < 0)
            return;
#pragma unroll
        for (int t = 0; t < STW; ++t) {
            const int sg = (ps0 >> 5) + stg * STW + t;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (live)
                    __builtin_nontemporal_store(vnew[t][q], vb_out + ((size_t)sg * 4 + q) * 64);
        }
        if (h == 0 && live) {
            if constexpr (HBUF) {
                const int hslot = ((ps0 - s_begin) / MFMA_TS) % L::HBS;
                if constexpr (STW == 2)
                    (*hbuf)[neuron][hslot] = (uint64_t)hword[0] | ((uint64_t)hword[STW - 1] << 32);
                else
                    reinterpret_cast<uint32_t *>(&(*hbuf)[neuron][hslot])[stg] = hword[0];
            } else {
                const int tile = ps0 / MFMA_TS;
                if constexpr (STW == 2) {
                    const uint64_t w64 = (uint64_t)hword[0] | ((uint64_t)hword[STW - 1] << 32);
                    hist_out[tile] = w64;
                    if (rast_out)
                        rast_out[tile] = w64;
                } else {
                    reinterpret_cast<uint32_t *>(hist_out + tile)[stg] = hword[0];
                    if (rast_out)
                        reinterpret_cast<uint32_t *>(rast_out + tile)[stg] = hword[0];
                }
            }
#pragma unroll
            for (int t = 0; t < STW; ++t) {
                const int s = ps0 + 32 * (stg * STW + t) + sig;
                if (s < s_end && pcnt[t])
                    atomicAdd(&s_cnt[0][s - s_begin], pcnt[t]);
            }
        }
        const int s = ps0 + lane;
        if (s < s_end && pdlev)
            atomicAdd(&s_cnt[1][s - s_begin], pdlev);
    };

    // history (and raster) words of chunk tiles [t0, t0 + nt) from LDS to
    // memory: lanes jj and jj + 32 write the first and second half of the
    // run of neuron 32nb + jj
    auto write_hist = [&](int t0, int nt) {
        if (!HBUF || !live || (STW == 1 && stg != 0))
            return;   // wave-uniform: wave stg 0 writes the neuron's words
        const int tile0 = s_begin / MFMA_TS + t0;
#pragma unroll
        for (int k = h * (L::HB / 2); k < (h + 1) * (L::HB / 2); ++k) {
            if (k < nt) {
                const uint64_t w = (*hbuf)[neuron][(t0 + k) % L::HBS];
                hist_out[tile0 + k] = w;
                if (rast_out)
                    rast_out[tile0 + k] = w;
            }
        }
    };

    prefetch_v(s_begin);
    RawT mraw[FMAX] = {};
    if (gatherer) {
        load_mask(s_begin, mraw);
        transpose_store(mask_of(mraw), 0);
        load_mask(s_begin + MFMA_TS, mraw);
    }
    load_ext(s_begin);
    lds_barrier();

    int it = 0;
    for (int s0 = s_begin; s0 < s_end; s0 += MFMA_TS, ++it) {
        int8_t *A = a_lds[it & 1];
        const bool more = s0 + MFMA_TS < s_end;
        // 0. everything issued in the previous iteration has completed: write
        //    out the previous tile, move this tile's potentials to VGPRs and
        //    start the next tile's potential transfer
        __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
        flush();
        v4i vold[STW][4];
#pragma unroll
        for (int t = 0; t < STW; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                vold[t][q] = v_lds[wave][t][q][lane];
        __builtin_amdgcn_s_waitcnt(WAIT_LGKMCNT0);
        if (more)
            prefetch_v(s0 + MFMA_TS);

        // 1. expansion, one lane per sample: delivered | external spikes of
        //    this wave's axon words to int8, delivered and event counts
        {
            const bool svalid = s0 + lane < s_end;
            unsigned pdl = 0u, pev = 0u, pevh = 0u;
#pragma unroll
            for (int k = 0; k < WPW; ++k) {
                const int wi = wave + 8 * k;
                if (wi < W_) {
                    const uint32_t xd = x_lds[it & 1][lane][wi];
                    const uint32_t x = xd | (svalid ? xe[k] : 0u);
                    pdl += (unsigned)__popc(xd);
                    uint32_t d[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        // nibble b3b2b1b0 -> bytes: bit i moves to bit 8i, no carries
                        d[q] = (((x >> (4 * q)) & 0xFu) * 0x00204081u) & 0x01010101u;
                        pev = __builtin_amdgcn_udot4(d[q], degl[k][q], pev, false);
                        if (any_hi)
                            pevh = __builtin_amdgcn_udot4(d[q], degh[k][q], pevh, false);
                    }
                    v4i *dst = reinterpret_cast<v4i *>(&A[lane * ROWB + 32 * wi]);
                    dst[0] = v4i{(int)d[0], (int)d[1], (int)d[2], (int)d[3]};
                    dst[1] = v4i{(int)d[4], (int)d[5], (int)d[6], (int)d[7]};
                }
            }
            pdlev = (pev + (pevh << 8)) | (pdl << 18);
        }
        ps0 = s0;
        // 2. delivered spikes of the next tile into LDS, then the loads for
        //    the tiles after (history bits two tiles ahead, input one ahead)
        if (more) {
            if (gatherer) {
                transpose_store(mask_of(mraw), (it + 1) & 1);
                load_mask(s0 + 2 * MFMA_TS, mraw);
            }
            load_ext(s0 + MFMA_TS);
        }
        lds_barrier();
        // the history words of the last HB tiles are complete in LDS
        if (it > 0 && it % L::HB == 0)
            write_hist(it - L::HB, L::HB);

        // 3. products and potential update (dead blocks skip it: their
        //    results are never stored)
        if constexpr (PSPLIT) {
            // epilogue of sub-tile t (32-sample group st of the tile at s0) from the
            // input plus leak of each accumulator element: saturating add, clamp,
            // threshold, reset; the neuron's spike word and the per-sample counts
            auto finish = [&](int t, int st, int s0, const v16i &in) {
                const int sg = (s0 >> 5) + st;   // 32-sample group
                // spike bits r of this lane, built from r = 15 down by doubling
                uint32_t hb = 0;
#pragma unroll
                for (int r = 15; r >= 0; --r) {
                    int32_t u = __builtin_elementwise_add_sat(vold[t][r >> 2][r & 3], in[r]);
                    if constexpr (EXT)
                        u = min(max(u, vmin), vmax);
                    const bool fire = u >= th;
                    if constexpr (EXT)
                        vnew[t][r >> 2][r & 3] = fire ? lif_reset(u, th, rs, vmax, lin) : max(u, fl);
                    else
                        vnew[t][r >> 2][r & 3] = fire ? rs : u;
                    hb = hb + hb + (uint32_t)fire;
                }
                // samples past the end never fire (their potentials are never read)
                if (sg * 32 + 32 > s_end) {   // wave-uniform
                    uint32_t vm = 0;
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        vm |= (uint32_t)(sg * 32 + 8 * (r >> 2) + 4 * h + (r & 3) < s_end) << r;
                    hb &= vm;
                }
                // the neuron's spike word: bits r from lane jj, bits 16 + r from lane jj + 32
                const uint32_t hw = hb | ((uint32_t)__shfl_xor((int)hb, 32, 64) << 16);
                hword[t] = hw;
                // per-sample spike words of the wave's 32 neurons, and their counts
                const uint32_t sw = transpose32(hw, lane);
                pcnt[t] = (unsigned)__popc(sw) | ((unsigned)__popc(sw & cm32) << 10) |
                          ((unsigned)__popc(sw & om32) << 20);
            };

            v16i accg[2];
            if (live) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    accg[0][r] = stg == 1 ? lk : 0;   // the lo plane carries the leak
                    accg[1][r] = stg == 1 ? lk : 0;
                }
                const int8_t *arow = &A[jj * ROWB + 16 * h];
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const v4i a0 = *reinterpret_cast<const v4i *>(arow + 32 * k);
                    const v4i a1 = *reinterpret_cast<const v4i *>(arow + 32 * ROWB + 32 * k);
                    accg[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, breg[k][0], accg[0], 0, 0, 0);
                    accg[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, breg[k][0], accg[1], 0, 0, 0);
                }
                // hand over the group the partner finishes
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    (*xch)[wave][r][lane] = stg == 0 ? accg[1][r] : accg[0][r];
            }
            lds_barrier();
            if (live) {
                v16i in;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t own = stg == 0 ? accg[0][r] : accg[1][r];
                    const int32_t other = (*xch)[wave ^ 4][r][lane];
                    in[r] = stg == 0 ? other + own * 128 : own + other * 128;
                }
                finish(0, stg, s0, in);
            }
        } else if (live) {
#pragma unroll
            for (int t = 0; t < STW; ++t) {
                const int st = stg * STW + t;
                const int sg = (s0 >> 5) + st;   // 32-sample group
                v16i acc_lo, acc_hi;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc_lo[r] = lk;
                    acc_hi[r] = 0;
                }
                const int8_t *arow = &A[(st * 32 + jj) * ROWB + 16 * h];
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const v4i a = *reinterpret_cast<const v4i *>(arow + 32 * k);
                    if constexpr (TWO) {
                        acc_hi = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, breg[k][0], acc_hi, 0, 0, 0);
                        acc_lo = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, breg[k][1], acc_lo, 0, 0, 0);
                    } else {
                        acc_lo = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, breg[k][0], acc_lo, 0, 0, 0);
                    }
                }
                // spike bits r of this lane, built from r = 15 down by doubling
                uint32_t hb = 0;
#pragma unroll
                for (int r = 15; r >= 0; --r) {
                    const int32_t in_leak = TWO ? acc_lo[r] + acc_hi[r] * 128 : acc_lo[r];
                    int32_t u = __builtin_elementwise_add_sat(vold[t][r >> 2][r & 3], in_leak);
                    if constexpr (EXT)
                        u = min(max(u, vmin), vmax);
                    const bool fire = u >= th;
                    if constexpr (EXT)
                        vnew[t][r >> 2][r & 3] = fire ? lif_reset(u, th, rs, vmax, lin) : max(u, fl);
                    else
                        vnew[t][r >> 2][r & 3] = fire ? rs : u;
                    hb = hb + hb + (uint32_t)fire;
                }
                // samples past the end never fire (their potentials are never read)
                if (sg * 32 + 32 > s_end) {   // wave-uniform
                    uint32_t vm = 0;
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        vm |= (uint32_t)(sg * 32 + 8 * (r >> 2) + 4 * h + (r & 3) < s_end) << r;
                    hb &= vm;
                }
                // the neuron's spike word: bits r from lane jj, bits 16 + r from lane jj + 32
                const uint32_t hw = hb | ((uint32_t)__shfl_xor((int)hb, 32, 64) << 16);
                hword[t] = hw;
                // per-sample spike words of the wave's 32 neurons, and their counts
                const uint32_t sw = transpose32(hw, lane);
                pcnt[t] = (unsigned)__popc(sw) | ((unsigned)__popc(sw & cm32) << 10) |
                          ((unsigned)__popc(sw & om32) << 20);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
    flush();
    lds_barrier();
    write_hist(it - 1 - (it - 1) % L::HB, (it - 1) % L::HB + 1);
    unsigned long long *cw_out =
        n.cring + ((size_t)r_row * n.C * n.cnt_rows + (size_t)c * n.cnt_rows + slice) * n.S + s_begin;
    for (int i = threadIdx.x; i < s_end - s_begin; i += blockDim.x) {
        const unsigned sp = s_cnt[0][i], ev = s_cnt[1][i];
        // the core's delivered spikes are counted once, by slice 0
        cw_out[i] = pack_counts(sp & 1023u, (sp >> 10) & 1023u, sp >> 20, slice == 0 ? ev >> 18 : 0u,
                                ev & ((1u << 18) - 1u));
    }
}

// Occupancy request (amdgpu_waves_per_eu(4): at most 128 VGPRs, so two
// 8-wavefront workgroups per CU): the compiler meets it for the 128-neuron
// slices with at most 128 axons (a few spilled VGPRs), whose LDS also fits
// twice per CU, and keeps the larger shapes as they are (one workgroup per
// CU). On the 64-variant sweep at 64 samples (one tile per workgroup, so no
// pipelining across tiles) the overlap of two workgroups gains 1.6%.
template <int A_, int N_, bool TWO, bool EXT, bool CB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_integrate_mfma(DevNet n, TickArgs ta,
                                                                                               int spw)
{
    typedef MfmaLds<A_, N_> L;
    __shared__ __attribute__((aligned(16))) typename L::ATile a_lds[2];
    __shared__ __attribute__((aligned(16))) typename L::VTile v_lds[8];
    __shared__ typename L::XTile x_lds[2];
    __shared__ typename L::HBuf hbuf[1];
    __shared__ int32_t xch_raw[TWO && A_ == 512 ? sizeof(typename L::Xch) / 4 : 1];
    __shared__ unsigned s_cnt[2][MFMA_SPW_MAX];
    integrate_mfma_unit<A_, N_, TWO, EXT, true, CB>(n, ta, spw, blockIdx.x, a_lds, v_lds, x_lds, hbuf,
                                                  reinterpret_cast<typename L::Xch *>(xch_raw), s_cnt);
}

// ---------------------------------------------------------------------------
// Several networks of one shape class (A, slice width, planes, potential update) in one
// launch: workgroup u runs unit u - e.unit_begin of the entry e whose unit
// range holds u. The entries come as kernel arguments and the LDS is exactly
// the shape's, as in the single-network kernel.
template <int A_, int N_, bool TWO, bool EXT, bool CB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_integrate_mfma_group(MfmaGroupArgs g,
                                                                                                     int k)
{
    typedef MfmaLds<A_, N_> L;
    __shared__ __attribute__((aligned(16))) typename L::ATile a_lds[2];
    __shared__ __attribute__((aligned(16))) typename L::VTile v_lds[8];
    __shared__ typename L::XTile x_lds[2];
    __shared__ typename L::HBuf hbuf[1];
    __shared__ int32_t xch_raw[TWO && A_ == 512 ? sizeof(typename L::Xch) / 4 : 1];
    __shared__ unsigned s_cnt[2][MFMA_SPW_MAX];
    const int u = blockIdx.x;
    int idx = 0;   // the last entry whose first unit is <= u (independent scalar loads)
    for (int i = 1; i < MFMA_GROUP_MAX; ++i)
        if (i < g.num && g.e[i].unit_begin <= u)
            idx = i;
    const MfmaGroupEntry &e = g.e[idx];
    TickArgs ta;
    ta.k = k;
    ta.ext_t = e.ext_base ? e.ext_base + (size_t)k * e.tick_words : nullptr;
    ta.ext_sstride = e.ext_sstride;
    integrate_mfma_unit<A_, N_, TWO, EXT, true, CB>(e.n, ta, e.spw, u - e.unit_begin, a_lds, v_lds, x_lds, hbuf,
                                                  reinterpret_cast<typename L::Xch *>(xch_raw), s_cnt);
}

// Launch of the kernels above for one B-source form (CB), by shape. Each
// form is instantiated in its own translation unit (see the file comment).
template <int A_, int N_, bool TWO, bool CB>
static void launch_group_k(const MfmaGroupArgs &g, int total, int k, int ext, hipStream_t st)
{
    if (ext)
        hipLaunchKernelGGL((k_integrate_mfma_group<A_, N_, TWO, true, CB>), dim3(total), dim3(512), 0, st, g, k);
    else
        hipLaunchKernelGGL((k_integrate_mfma_group<A_, N_, TWO, false, CB>), dim3(total), dim3(512), 0, st, g, k);
}

template <bool CB>
static hipError_t launch_group_code(const MfmaGroupArgs &g, int total, int k, int code, int ext, hipStream_t st)
{
    switch (code) {
    case 0: launch_group_k<64, 128, false, CB>(g, total, k, ext, st); break;
    case 1: launch_group_k<64, 128, true, CB>(g, total, k, ext, st); break;
    case 2: launch_group_k<64, 256, false, CB>(g, total, k, ext, st); break;
    case 3: launch_group_k<64, 256, true, CB>(g, total, k, ext, st); break;
    case 4: launch_group_k<128, 128, false, CB>(g, total, k, ext, st); break;
    case 5: launch_group_k<128, 128, true, CB>(g, total, k, ext, st); break;
    case 6: launch_group_k<128, 256, false, CB>(g, total, k, ext, st); break;
    case 7: launch_group_k<128, 256, true, CB>(g, total, k, ext, st); break;
    case 8: launch_group_k<256, 128, false, CB>(g, total, k, ext, st); break;
    case 9: launch_group_k<256, 128, true, CB>(g, total, k, ext, st); break;
    case 10: launch_group_k<256, 256, false, CB>(g, total, k, ext, st); break;
    case 11: launch_group_k<256, 256, true, CB>(g, total, k, ext, st); break;
    case 12: launch_group_k<512, 128, false, CB>(g, total, k, ext, st); break;
    case 13: launch_group_k<512, 128, true, CB>(g, total, k, ext, st); break;
    case 14: launch_group_k<512, 256, false, CB>(g, total, k, ext, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int A_, int N_, bool TWO, bool CB>
static void launch_mfma_k(const DevNet &n, const TickArgs &a, int spw, hipStream_t st)
{
    const int chunks = (n.S + spw - 1) / spw;
    const dim3 grid(n.C * n.slices * chunks), block(512);
    if (!n.model_ext)
        hipLaunchKernelGGL((k_integrate_mfma<A_, N_, TWO, false, CB>), grid, block, 0, st, n, a, spw);
    else
        hipLaunchKernelGGL((k_integrate_mfma<A_, N_, TWO, true, CB>), grid, block, 0, st, n, a, spw);
}

template <int A_, int N_, bool CB>
static hipError_t launch_mfma_an(const DevNet &n, const TickArgs &a, int two, int spw, hipStream_t st)
{
    if constexpr (A_ <= 256) {
        if (two)
            launch_mfma_k<A_, N_, true, CB>(n, a, spw, st);
        else
            launch_mfma_k<A_, N_, false, CB>(n, a, spw, st);
    } else {
        if (!two)
            launch_mfma_k<A_, N_, false, CB>(n, a, spw, st);
        else if constexpr (N_ == 128)
            launch_mfma_k<A_, 128, true, CB>(n, a, spw, st);   // plane split
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// n, two and spw already validated (launch_integrate_mfma)
template <bool CB>
static hipError_t launch_mfma_shape(const DevNet &n, const TickArgs &a, int two, int spw, hipStream_t st)
{
    const int w = mfma_width(n.A, n.N, two);
    switch (n.A * 2 + (w == 256 ? 1 : 0)) {
    case 128: return launch_mfma_an<64, 128, CB>(n, a, two, spw, st);
    case 129: return launch_mfma_an<64, 256, CB>(n, a, two, spw, st);
    case 256: return launch_mfma_an<128, 128, CB>(n, a, two, spw, st);
    case 257: return launch_mfma_an<128, 256, CB>(n, a, two, spw, st);
    case 512: return launch_mfma_an<256, 128, CB>(n, a, two, spw, st);
    case 513: return launch_mfma_an<256, 256, CB>(n, a, two, spw, st);
    case 1024: return launch_mfma_an<512, 128, CB>(n, a, two, spw, st);
    case 1025: return launch_mfma_an<512, 256, CB>(n, a, two, spw, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ranc
