// kern_resident.hip -- every tick of a call on the batched MFMA path in one
// persistent, cooperatively launched grid that keeps the potentials on chip.
//
// The per-tick kernel (kern_mfma.hip) reads and writes every potential once
// per tick; on a batch of many samples that read-modify-write stream is what
// bounds it. Here each workgroup owns up to two cores for the whole launch
// (cores wg and wg + grid), and each of its 8 wavefronts the 32-neuron block
// `wave` of both, with both blocks' B tiles held in VGPRs. The samples go in
// groups of 64: the workgroup loads its cores' potentials of the group into
// LDS, runs every tick of the call on them, and writes them back, so the
// potentials cross HBM once per call instead of once per tick.
//
// A core's axons can take spikes from any core, so spikes still travel
// through the sample-sliced spike history in HBM: at tick t each workgroup
// gathers its axons' source words written at t - d (d >= 1), and after each
// tick the whole grid synchronizes, which makes every history word of tick t
// visible before any workgroup gathers for tick t + 1, and keeps a history
// slot from being overwritten while its old contents are still due (a slot is
// rewritten Q = D + 1 ticks later, after its last reader at delay <= D).
// The sample groups are independent (each reads and writes only its own
// 64-sample history and raster words and counter entries).
//
// Tick semantics, data layouts, the MFMA formulation (int8 products, hi/lo
// planes for 9-bit weights, the leak as the accumulator's start), the
// history bit order and the per-sample counters are those of
// k_integrate_mfma; results are identical to running it tick by tick.
//
// Grid synchronization: an arrival counter and a give-up flag in the
// workspace, both zeroed before the launch. Each wave waits for its own
// stores, the workgroup meets at a barrier, and one thread releases
// (agent-scope fence: the stores reach memory visible to all XCDs), adds one
// to the counter, waits until the counter reaches (barriers passed) x (grid
// size), and acquires (agent-scope fence: stale cached lines are dropped).
// Every wait is bounded: a thread that has waited longer than `wait_ticks`
// of the constant-rate wall clock, or that sees the flag set, sets the flag
// and the workgroup leaves the kernel; so every workgroup exits, and the host
// reads the flag after the launch and reports the call as failed. The grid
// is launched cooperatively (all workgroups resident at once) and sized from
// the occupancy the runtime reports.
#include "kern_common.h"
#include "kern_bits.h"
#include "ranc_internal.h"

namespace ranc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

static constexpr int RS_TS = 64;    // samples per group
static constexpr int RS_CPW = 2;    // cores per workgroup, at most
static constexpr int RS_NB = 8;     // 32-neuron blocks per core (256 neurons)
static constexpr int RS_WAVES = 4;  // wavefronts per workgroup (one per SIMD: 512 registers each)
static constexpr int RS_WAIT_VMCNT0 = 0x0F70;   // s_waitcnt vmcnt(0) (gfx9 encoding)
static constexpr int RS_CPOL_NT = 2;            // cache policy of a global-to-LDS load: non-temporal

typedef __attribute__((address_space(3))) void lds_void;

template <int A_> struct ResLds {
    static constexpr int ROWB = A_ + 16;   // padded row of the int8 tile (bytes)
    static constexpr int XW = A_ / 32 + 1; // padded axon words per sample
    v4i v[RS_CPW][RS_NB][2][4][64];        // potentials: [core][block][32-sample half][quad][lane]
    int8_t a[RS_TS * ROWB];                // int8 axon spikes of one core's group
    uint32_t x[RS_CPW][RS_TS][XW];         // delivered axon words per sample
    uint32_t deg[RS_CPW][2][A_ / 4];       // connected-neuron counts, low / high byte planes
    unsigned cnt[RS_CPW][2][RS_TS];        // per-sample packed counts of the tick
    int ok;
};

// Grid-wide barrier number `b` (1, 2, ...) with a bounded wait; false when
// this or another workgroup gave up.
__device__ __forceinline__ bool grid_barrier(const ResSync &sy, unsigned b, int *ok_lds)
{
    __builtin_amdgcn_s_waitcnt(RS_WAIT_VMCNT0);   // this wave's global stores are done
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(sy.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = b * gridDim.x;
        const unsigned long long t0 = wall_clock64();
        int ok = 1;
        while (__hip_atomic_load(sy.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(sy.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                wall_clock64() - t0 > sy.wait_ticks) {
                __hip_atomic_store(sy.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

template <int A_, bool TWO, bool EXT>
__global__ __launch_bounds__(64 * RS_WAVES) void k_mfma_resident(DevNet n, ResidentArgs ra, ResSync sy)
{
    constexpr int KS = A_ / 32;                  // 32-axon k-steps
    constexpr int W_ = A_ / 32;                  // axon words
    constexpr int PL = TWO ? 2 : 1;              // weight planes
    constexpr int APW = A_ / 64;                 // 64-axon blocks of the gather
    constexpr int GT = 2 * APW;                  // gather tasks per core: (axon block, 32-sample half)
    constexpr int GPW = (GT + RS_WAVES - 1) / RS_WAVES;   // gather tasks per wave
    constexpr int XPW = (W_ + RS_WAVES - 1) / RS_WAVES;   // axon words expanded per wave
    constexpr int BPW = RS_NB / RS_WAVES;        // 32-neuron blocks per wave and core
    constexpr int FMAX = 4;                      // sources per axon gathered without a loop
    typedef ResLds<A_> L;
    constexpr int ROWB = L::ROWB;
    __shared__ L lds;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, jj = lane & 31;
    const int sig = sigma32(jj);
    const int grid = gridDim.x;
    const size_t CN = (size_t)n.C * n.N;
    const size_t G32 = (size_t)n.S64 / 32;
    const size_t HG = (size_t)n.S64 / 64;
    const int tick_q = n.tick[0], tick_r = n.tick[1];

    int core[RS_CPW];
    bool has[RS_CPW];
#pragma unroll
    for (int j = 0; j < RS_CPW; ++j) {
        core[j] = blockIdx.x + j * grid;
        has[j] = core[j] < n.C;   // workgroup-uniform
    }

    // B tiles of the wave's blocks (wave + RS_WAVES * b) of both cores,
    // resident for the launch
    v4i breg[RS_CPW][BPW][KS][PL];
    const v4i *planes = reinterpret_cast<const v4i *>(n.planes);
#pragma unroll
    for (int j = 0; j < RS_CPW; ++j)
#pragma unroll
        for (int b = 0; b < BPW; ++b)
#pragma unroll
            for (int k = 0; k < KS; ++k)
#pragma unroll
                for (int p = 0; p < PL; ++p)
                    breg[j][b][k][p] =
                        has[j] ? planes[((((size_t)core[j] * n.NW + wave + RS_WAVES * b) * KS + k) * PL + p) * 64 + lane]
                               : v4i{0, 0, 0, 0};
    // the lane's neurons 32 * (wave + RS_WAVES * b) + jj of each core
    int32_t lk[RS_CPW][BPW], th[RS_CPW][BPW], rs[RS_CPW][BPW], fl[RS_CPW][BPW];
    bool lin[RS_CPW][BPW];
    int oi[RS_CPW][BPW];
    uint32_t cm32[RS_CPW][BPW], om32[RS_CPW][BPW];
    int ci[RS_CPW];
#pragma unroll
    for (int j = 0; j < RS_CPW; ++j) {
        const int c = has[j] ? core[j] : 0;
        ci[j] = n.in_index[c];
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int nb = wave + RS_WAVES * b;
            const size_t cj = (size_t)c * n.N + nb * 32 + jj;
            lk[j][b] = n.leak[cj];
            th[j][b] = n.thr[cj];
            rs[j][b] = n.rst[cj];
            fl[j][b] = n.vmin;
            lin[j][b] = false;
            if constexpr (EXT) {
                fl[j][b] = n.floor[cj];
                lin[j][b] = (n.linmask[cj >> 5] >> (cj & 31)) & 1u;
            }
            oi[j][b] = n.outidx[cj];
            cm32[j][b] = n.coremask[(size_t)c * n.NW + nb];
            om32[j][b] = n.outmask[(size_t)c * n.NW + nb];
        }
    }
    // connected-neuron counts to LDS; per-sample counts start at zero
    for (int i = threadIdx.x; i < RS_CPW * 2 * (A_ / 4); i += blockDim.x) {
        const int j = i / (2 * (A_ / 4)), r = i % (2 * (A_ / 4));
        const int c = blockIdx.x + j * grid;
        (&lds.deg[j][0][0])[r] = c < n.C ? n.degb[(size_t)c * 2 * (A_ / 4) + r] : 0u;
    }
    for (int i = threadIdx.x; i < RS_CPW * 2 * RS_TS; i += blockDim.x)
        (&lds.cnt[0][0][0])[i] = 0u;

    // gather task t = wave + RS_WAVES * u collects, for axon block t % APW, the
    // 32-sample half t / APW of each group; each lane keeps its axon's entry
    // range and first entry (source neuron << 4 | delay - 1)
    uint32_t e_beg[RS_CPW][GPW], e_end[RS_CPW][GPW], ent0[RS_CPW][GPW];
#pragma unroll
    for (int j = 0; j < RS_CPW; ++j)
#pragma unroll
        for (int u = 0; u < GPW; ++u) {
            const int t = wave + RS_WAVES * u;
            e_beg[j][u] = e_end[j][u] = 0u;
            if (t < GT && has[j]) {
                const size_t ax = (size_t)core[j] * A_ + (t % APW) * 64 + lane;
                e_beg[j][u] = n.rtx_ptr[ax];
                e_end[j][u] = n.rtx_ptr[ax + 1];
            }
            ent0[j][u] = e_beg[j][u] < e_end[j][u] ? n.rtx_ent[e_beg[j][u]] : 0u;
        }
    __syncthreads();

    unsigned barriers = 0;
    const int groups = n.S64 / RS_TS;
    for (int g = 0; g < groups; ++g) {
        // this group's potentials of the wave's blocks from HBM straight into
        // LDS (no VGPRs on the way), complete before the first tick uses them
#pragma unroll
        for (int j = 0; j < RS_CPW; ++j) {
            if (!has[j])
                continue;
#pragma unroll
            for (int b = 0; b < BPW; ++b) {
                const int nb = wave + RS_WAVES * b;
                const v4i *vb = reinterpret_cast<const v4i *>(n.V) + ((size_t)core[j] * n.NW + nb) * G32 * 256 + lane;
#pragma unroll
                for (int st = 0; st < 2; ++st)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        __builtin_amdgcn_global_load_lds((const void *)(vb + ((size_t)(2 * g + st) * 4 + q) * 64),
                                                         (lds_void *)&lds.v[j][nb][st][q][0], 16, 0, RS_CPOL_NT);
            }
        }
        __builtin_amdgcn_s_waitcnt(RS_WAIT_VMCNT0);
        const int s_end = min(n.S - g * RS_TS, RS_TS);   // valid samples in this group

        for (int k = 0; k < ra.num_ticks; ++k) {
            const int q_now = (tick_q + k) % n.Q;
            const int r_row = (tick_r + k) % n.RT;
            // 1. delivered axon words of both cores: OR of the sources' history
            //    words of this group at their delays, transposed to per-sample words
#pragma unroll
            for (int j = 0; j < RS_CPW; ++j) {
#pragma unroll
                for (int u = 0; u < GPW; ++u) {
                    const int t = wave + RS_WAVES * u;
                    if (!has[j] || t >= GT)
                        continue;   // wave-uniform
                    const int axb = t % APW, grp = t / APW;
                    // sources past the first are rare: their entries are read here
                    uint32_t en[FMAX];
                    en[0] = ent0[j][u];
#pragma unroll
                    for (int f = 1; f < FMAX; ++f)
                        en[f] = e_beg[j][u] + f < e_end[j][u] ? n.rtx_ent[e_beg[j][u] + f] : 0u;
                    uint32_t m = 0u;
#pragma unroll
                    for (int f = 0; f < FMAX; ++f) {
                        if (e_beg[j][u] + f < e_end[j][u]) {
                            int slot = q_now - (int)(en[f] & 15u) - 1;
                            if (slot < 0)
                                slot += n.Q;
                            m |= reinterpret_cast<const uint32_t *>(n.hist + ((size_t)slot * CN + (en[f] >> 4)) * HG + g)[grp];
                        }
                    }
                    for (uint32_t e = e_beg[j][u] + FMAX; e < e_end[j][u]; ++e) {
                        const uint32_t ee = n.rtx_ent[e];
                        int slot = q_now - (int)(ee & 15u) - 1;
                        if (slot < 0)
                            slot += n.Q;
                        m |= reinterpret_cast<const uint32_t *>(n.hist + ((size_t)slot * CN + (ee >> 4)) * HG + g)[grp];
                    }
                    lds.x[j][32 * grp + sig][2 * axb + h] = transpose32(m, lane);
                }
            }
            lds_barrier();

#pragma unroll
            for (int j = 0; j < RS_CPW; ++j) {
                if (!has[j])
                    continue;   // workgroup-uniform
                // 2. expansion, one lane per sample: delivered | external spikes
                //    of the wave's axon words to int8, delivered and event counts
                {
                    const bool svalid = lane < s_end;
                    unsigned pdlev = 0u;
#pragma unroll
                    for (int u = 0; u < XPW; ++u) {
                        const int wi = wave + RS_WAVES * u;
                        if (wi >= W_)
                            continue;   // wave-uniform
                        const uint32_t xd = lds.x[j][lane][wi];
                        uint32_t xe = 0u;
                        if (ra.ext_base && ci[j] >= 0 && svalid)
                            xe = ra.ext_base[(size_t)k * ra.tick_words + (size_t)ci[j] * W_ + wi +
                                             (size_t)(g * RS_TS + lane) * ra.ext_sstride];
                        const uint32_t x = xd | xe;
                        unsigned pev = 0u, pevh = 0u;
                        uint32_t d[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            // nibble b3b2b1b0 -> bytes: bit i moves to bit 8i, no carries
                            d[q] = (((x >> (4 * q)) & 0xFu) * 0x00204081u) & 0x01010101u;
                            pev = __builtin_amdgcn_udot4(d[q], lds.deg[j][0][wi * 8 + q], pev, false);
                            pevh = __builtin_amdgcn_udot4(d[q], lds.deg[j][1][wi * 8 + q], pevh, false);
                        }
                        v4i *dst = reinterpret_cast<v4i *>(&lds.a[lane * ROWB + 32 * wi]);
                        dst[0] = v4i{(int)d[0], (int)d[1], (int)d[2], (int)d[3]};
                        dst[1] = v4i{(int)d[4], (int)d[5], (int)d[6], (int)d[7]};
                        pdlev += (pev + (pevh << 8)) | ((unsigned)__popc(xd) << 18);
                    }
                    if (svalid && pdlev)
                        atomicAdd(&lds.cnt[j][1][lane], pdlev);
                }
                lds_barrier();

                // 3. products and potential update of the wave's blocks, per
                //    32-sample half
#pragma unroll
                for (int b = 0; b < BPW; ++b) {
                    const int nb = wave + RS_WAVES * b;
                    uint64_t w64 = 0;   // the neuron's 64-sample spike word
#pragma unroll 1
                    for (int st = 0; st < 2; ++st) {
                        // one accumulator: with two planes the high plane's products
                        // go first, are scaled by 128, and the leak and the low
                        // plane's products are added on top (exact in int32)
                        v16i acc;
                        const int8_t *arow = &lds.a[(st * 32 + jj) * ROWB + 16 * h];
                        if constexpr (TWO) {
#pragma unroll
                            for (int r = 0; r < 16; ++r)
                                acc[r] = 0;
#pragma unroll
                            for (int kk = 0; kk < KS; ++kk) {
                                const v4i a = *reinterpret_cast<const v4i *>(arow + 32 * kk);
                                acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, breg[j][b][kk][0], acc, 0, 0, 0);
                            }
#pragma unroll
                            for (int r = 0; r < 16; ++r)
                                acc[r] = acc[r] * 128 + lk[j][b];
                        } else {
#pragma unroll
                            for (int r = 0; r < 16; ++r)
                                acc[r] = lk[j][b];
                        }
#pragma unroll
                        for (int kk = 0; kk < KS; ++kk) {
                            const v4i a = *reinterpret_cast<const v4i *>(arow + 32 * kk);
                            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, breg[j][b][kk][PL - 1], acc, 0, 0, 0);
                        }
                        uint32_t hb = 0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            v4i vo = lds.v[j][nb][st][q][lane];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int r = 4 * q + e;
                                int32_t u = __builtin_elementwise_add_sat(vo[e], acc[r]);
                                if constexpr (EXT)
                                    u = min(max(u, n.vmin), n.vmax);
                                const bool fire = u >= th[j][b];
                                if constexpr (EXT)
                                    vo[e] = fire ? lif_reset(u, th[j][b], rs[j][b], n.vmax, lin[j][b]) : max(u, fl[j][b]);
                                else
                                    vo[e] = fire ? rs[j][b] : u;
                                hb |= (uint32_t)fire << r;
                            }
                            lds.v[j][nb][st][q][lane] = vo;
                        }
                        // samples past the end never fire
                        if (st * 32 + 32 > s_end) {   // wave-uniform
                            uint32_t vm = 0;
#pragma unroll
                            for (int r = 0; r < 16; ++r)
                                vm |= (uint32_t)(st * 32 + 8 * (r >> 2) + 4 * h + (r & 3) < s_end) << r;
                            hb &= vm;
                        }
                        // the neuron's spike word: bits r from lane jj, bits 16 + r from lane jj + 32
                        const uint32_t hw = hb | ((uint32_t)__shfl_xor((int)hb, 32, 64) << 16);
                        w64 |= (uint64_t)hw << (32 * st);
                        // per-sample spike words of the block's 32 neurons, and their counts
                        const uint32_t sw = transpose32(hw, lane);
                        const unsigned pc = (unsigned)__popc(sw) | ((unsigned)__popc(sw & cm32[j][b]) << 10) |
                                            ((unsigned)__popc(sw & om32[j][b]) << 20);
                        const int s = st * 32 + sig;
                        if (h == 0 && s < s_end && pc)
                            atomicAdd(&lds.cnt[j][0][s], pc);
                    }
                    if (h == 0) {
                        const size_t cj = (size_t)core[j] * n.N + nb * 32 + jj;
                        n.hist[((size_t)q_now * CN + cj) * HG + g] = w64;
                        if (oi[j][b] >= 0)
                            reinterpret_cast<uint64_t *>(n.raster)[((size_t)r_row * n.Nout + oi[j][b]) * HG + g] = w64;
                    }
                }
                lds_barrier();   // the int8 tile is free for the next core
            }
            // 4. this tick's per-sample counts of the group
            for (int i = threadIdx.x; i < RS_CPW * RS_TS; i += blockDim.x) {
                const int j = i / RS_TS, sl = i % RS_TS;
                const int c = blockIdx.x + j * grid;
                if (c < n.C && sl < s_end) {
                    const unsigned sp = lds.cnt[j][0][sl], ev = lds.cnt[j][1][sl];
                    n.cring[((size_t)r_row * n.C * n.cnt_rows + (size_t)c * n.cnt_rows) * n.S + g * RS_TS + sl] =
                        pack_counts(sp & 1023u, (sp >> 10) & 1023u, sp >> 20, ev >> 18, ev & ((1u << 18) - 1u));
                }
                lds.cnt[j][0][sl] = 0u;
                lds.cnt[j][1][sl] = 0u;
            }
            // 5. every workgroup's history words of this tick are visible
            if (!grid_barrier(sy, ++barriers, &lds.ok))
                return;
        }
        // the group's potentials back to HBM, one 16-byte store per lane at a
        // time (once per group: no registers held for it)
#pragma unroll 1
        for (int i = 0; i < RS_CPW * BPW * 8; ++i) {
            const int j = i / (BPW * 8), b = (i / 8) % BPW, st = (i >> 2) & 1, q = i & 3;
            const int c = blockIdx.x + j * grid;
            const int nb = wave + RS_WAVES * b;
            if (c < n.C) {
                v4i *vb = reinterpret_cast<v4i *>(n.V) + ((size_t)c * n.NW + nb) * G32 * 256 + lane;
                __builtin_nontemporal_store(lds.v[j][nb][st][q][lane], vb + ((size_t)(2 * g + st) * 4 + q) * 64);
            }
        }
    }
}

__global__ void k_resident_arm(ResSync sy)
{
    if (threadIdx.x == 0) {
        sy.ctr[0] = 0u;
        sy.abort[0] = 0u;
    }
}

template <int A_, bool TWO, bool EXT>
static hipError_t launch_res(const DevNet &n, const ResidentArgs &ra, const ResSync &sy, int grid, hipStream_t st)
{
    DevNet nn = n;
    ResidentArgs a = ra;
    ResSync s = sy;
    void *args[] = {&nn, &a, &s};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_mfma_resident<A_, TWO, EXT>), dim3(grid),
                                      dim3(64 * RS_WAVES), args, 0, st);
}

template <int A_, bool TWO, bool EXT>
static int res_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(&k_mfma_resident<A_, TWO, EXT>),
                                                     64 * RS_WAVES, 0) != hipSuccess)
        return 0;
    return nb;
}

int resident_blocks_per_cu(int A, int two, int ext)
{
    switch ((A == 64 ? 0 : A == 128 ? 1 : A == 256 ? 2 : 3) * 4 + (two ? 2 : 0) + (ext ? 1 : 0)) {
    case 0: return res_occupancy<64, false, false>();
    case 1: return res_occupancy<64, false, true>();
    case 2: return res_occupancy<64, true, false>();
    case 3: return res_occupancy<64, true, true>();
    case 4: return res_occupancy<128, false, false>();
    case 5: return res_occupancy<128, false, true>();
    case 6: return res_occupancy<128, true, false>();
    case 7: return res_occupancy<128, true, true>();
    case 8: return res_occupancy<256, false, false>();
    case 9: return res_occupancy<256, false, true>();
    case 10: return res_occupancy<256, true, false>();
    case 11: return res_occupancy<256, true, true>();
    default: return 0;
    }
}

int resident_max_cores_per_wg() { return RS_CPW; }

hipError_t launch_mfma_resident(const DevNet &n, const ResidentArgs &ra, const ResSync &sy, int grid, int two,
                                hipStream_t st)
{
    if (n.N != 256 || n.slices != 1 || grid < 1 || (long long)grid * RS_CPW < n.C || n.S64 % RS_TS != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_resident_arm, dim3(1), dim3(64), 0, st, sy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const bool ext = n.model_ext != 0;
    switch ((n.A == 64 ? 0 : n.A == 128 ? 1 : n.A == 256 ? 2 : 3) * 4 + (two ? 2 : 0) + (ext ? 1 : 0)) {
    case 0: return launch_res<64, false, false>(n, ra, sy, grid, st);
    case 1: return launch_res<64, false, true>(n, ra, sy, grid, st);
    case 2: return launch_res<64, true, false>(n, ra, sy, grid, st);
    case 3: return launch_res<64, true, true>(n, ra, sy, grid, st);
    case 4: return launch_res<128, false, false>(n, ra, sy, grid, st);
    case 5: return launch_res<128, false, true>(n, ra, sy, grid, st);
    case 6: return launch_res<128, true, false>(n, ra, sy, grid, st);
    case 7: return launch_res<128, true, true>(n, ra, sy, grid, st);
    case 8: return launch_res<256, false, false>(n, ra, sy, grid, st);
    case 9: return launch_res<256, false, true>(n, ra, sy, grid, st);
    case 10: return launch_res<256, true, false>(n, ra, sy, grid, st);
    case 11: return launch_res<256, true, true>(n, ra, sy, grid, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ranc
