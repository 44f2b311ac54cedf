// kern_mfma.hip -- one tick of the batched path on int8 MFMA: delivery of the
// spikes scheduled for this tick, integration, leak/threshold/reset, and the
// scheduler write of this tick's spikes.
//
// Integration. With many samples, the integration of one core (GPU-RANC
// Sec. II: sum over spiking connected axons of the neuron's weight for the
// axon's type) is the dense product X[samples x A] * B[A x N] with X the 0/1
// axon spikes and B[a][n] = crossbar(a, n) * weight(n, type(a)). It runs on
// V_MFMA_I32_16X16X64_I8 with int32 accumulation, which is exact:
//   - weights of up to 8 bits are int8 as they are (one B plane);
//   - 9-bit weights w in [-256, 255] are split as w = 128*hi + lo with
//     lo = w & 127 in [0, 127] and hi = w >> 7 in [-2, 1]. The hi term is
//     formed as (-128 * x) * (-hi): the spike byte shifted left by 7 is the
//     int8 value -128, and -hi lies in [-1, 2], so both planes accumulate into
//     the same int32 register and no rescaling pass is needed.
//   |sum| <= 512 * 256 < 2^31, so int32 never overflows.
//
// Scheduler. A spike fired at tick t by neuron g with destination
// (core, axon, delay d) must reach that axon at tick t + d (Sec. III-D/E;
// several spikes to one (core, axon, tick) merge into one bit). On this path
// the scheduler holds the last Q = D + 1 ticks of every neuron's spikes,
// sample-sliced (one u16 = 16 samples of one neuron), and delivery is done by
// the destination: at tick t the workgroup of a core ORs, for each of its
// axons, the history bits of its sources at tick t - d. Every scheduler word
// has exactly one writer (the firing neuron's workgroup, at tick t, slot
// t % Q) and no atomics are used. A 64-lane ballot turns the per-axon sample
// bits back into per-sample axon words.
//
// Mapping: one workgroup of 16 wavefronts per (core, chunk of samples); the
// core's B tiles stay in VGPRs for the whole chunk (A*N*planes/4096 VGPRs per
// lane). Samples are taken 64 at a time in a software pipeline:
//   - history bits of tile i+2 are loaded and those of tile i+1 transposed
//     into LDS while tile i runs, so no load latency sits on the critical path;
//   - the axon spikes of tile i (delivered OR external input) are expanded to
//     an int8 [64 x A] tile in LDS, double-buffered so one barrier per tile
//     suffices; delivered spikes and synaptic events (sum over spiking axons
//     of their connected-neuron counts) are reduced per sample in the same pass;
//   - each wavefront loads its potentials as one 16-byte vector per lane (V is
//     stored in "bricks" matching the MFMA result layout, so a wave's load is
//     a contiguous 1 KiB), multiplies its 16-sample sub-tiles against its
//     16-neuron block and applies leak / threshold / reset in the epilogue,
//     which also writes this tick's spikes to the history, the output raster
//     and per-sample counters (accumulated in LDS, written once per chunk).
//
// MFMA operand convention used for both A and B: in k-step k, lane l holds 16
// bytes for row/column l % 16 and axons 64k + 16*(l/16) + [0, 16). The sum
// over k does not depend on which hardware k each byte stands for as long as
// A and B agree. Result: lane l, element r is row 4*(l/16) + r, column l % 16.
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

typedef int v4i __attribute__((ext_vector_type(4)));

static constexpr int MFMA_TS = 64;        // samples per LDS tile
static constexpr int MFMA_SPW_MAX = 1024; // samples per workgroup (LDS counters)

int mfma_max_samples_per_wg() { return MFMA_SPW_MAX; }

template <int A_, int N_, bool TWO>
__global__ __launch_bounds__(1024) void k_integrate_mfma(DevNet n, TickArgs ta, int spw)
{
    constexpr int NB = N_ / 16;                     // 16-neuron blocks (<= 16)
    constexpr int KS = A_ / 64;                     // 64-axon k-steps
    constexpr int PL = TWO ? 2 : 1;                 // B planes
    constexpr int WPB = 16 / NB;                    // waves sharing a neuron block
    constexpr int STW = 4 / WPB;                    // 16-sample sub-tiles per wave per tile
    constexpr int W_ = A_ / 32;
    constexpr int NW_ = N_ / 32;
    constexpr int ROWB = A_ + 16;                   // padded LDS row (bytes)
    constexpr int QD = A_ / 4;                      // axon dwords per sample row
    constexpr int QPL = (QD + 63) / 64;             // axon dwords per lane in the expansion
    constexpr unsigned EV_BITS = 18;                // events per (sample, core) <= 512*256 < 2^18
    constexpr int APW = A_ / 64;                    // 64-axon blocks
    constexpr int PARTS = 16 / APW;                 // sample parts in the history gather
    constexpr int SPT = MFMA_TS / PARTS;            // samples per gathering lane (4..32)

    __shared__ __attribute__((aligned(16))) int8_t a_lds[2][MFMA_TS * ROWB];
    __shared__ uint32_t x_lds[2][MFMA_TS][W_];      // delivered axon spikes of a tile
    __shared__ unsigned s_cnt[5][MFMA_SPW_MAX];     // emitted, routed, out, delivered, events

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x % n.C;
    const int chunk = blockIdx.x / n.C;
    const int s_begin = chunk * spw;
    const int s_end = min(n.S, s_begin + spw);
    const int s_end16 = min(n.S16, s_begin + spw);
    const int g4 = lane >> 4, jj = lane & 15;
    const int nb = wave % NB;
    const int stg = wave / NB;

    for (int i = threadIdx.x; i < 5 * MFMA_SPW_MAX; i += blockDim.x)
        (&s_cnt[0][0])[i] = 0u;

    // B tiles of this wave's neuron block, resident for the whole chunk.
    v4i breg[KS][PL];
    const v4i *planes = reinterpret_cast<const v4i *>(n.planes);
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
        for (int p = 0; p < PL; ++p)
            breg[k][p] = planes[((((size_t)c * NB + nb) * KS + k) * PL + p) * 64 + lane];
    const size_t cj = (size_t)c * N_ + nb * 16 + jj;
    const int32_t lk = n.leak[cj], th = n.thr[cj], rs = n.rst[cj];
    const size_t mword = (size_t)c * NW_ + (nb >> 1);
    const int hsh = 16 * (nb & 1);
    const uint32_t cm16 = (n.coremask[mword] >> hsh) & 0xFFFFu;
    const uint32_t om16 = (n.outmask[mword] >> hsh) & 0xFFFFu;
    const int ow = n.outword[mword];

    // Connected-neuron counts of the axons this lane expands.
    int degv[QPL][4];
#pragma unroll
    for (int qi = 0; qi < QPL; ++qi) {
        const int q = lane + 64 * qi;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            degv[qi][b] = q < QD ? n.deg[(size_t)c * A_ + 4 * q + b] : 0;
    }

    const int ci = n.in_index[c];
    const uint32_t *ext_c = (ta.ext_t != nullptr && ci >= 0) ? ta.ext_t + (size_t)ci * W_ : nullptr;
    const size_t groups = (size_t)n.S16 / 16;
    const v4i *vb_in = reinterpret_cast<const v4i *>(n.V) + (((size_t)c * NB + nb) * groups) * 64 + lane;
    v4i *vb_out = reinterpret_cast<v4i *>(n.V) + (((size_t)c * NB + nb) * groups) * 64 + lane;
    const size_t CN = (size_t)n.C * N_;
    uint16_t *hist_out = n.hist + ((size_t)ta.q_now * CN + (size_t)c * N_ + nb * 16 + jj) * groups;

    // History gather: this lane collects axon ga of the core for SPT samples.
    const int ga = (wave % APW) * 64 + lane;
    const int part = wave / APW;
    const uint32_t e_beg = n.rtx_ptr[(size_t)c * A_ + ga], e_end = n.rtx_ptr[(size_t)c * A_ + ga + 1];
    auto load_mask = [&](int s0) -> uint32_t {
        const int sp = s0 + part * SPT;
        uint32_t m = 0;
        if (sp < s_end) {
            for (uint32_t e = e_beg; e < e_end; ++e) {
                const uint32_t ent = n.rtx_ent[e];
                int slot = ta.q_now - (int)(ent & 15u) - 1;
                if (slot < 0)
                    slot += n.Q;
                const uint16_t *h = n.hist + ((size_t)slot * CN + (ent >> 4)) * groups + (sp >> 4);
                if (SPT < 16) {
                    m |= ((uint32_t)h[0] >> (sp & 15)) & ((1u << SPT) - 1u);
                } else if (SPT == 16) {
                    m |= (uint32_t)h[0];
                } else {
                    m |= (uint32_t)h[0] | (sp + 16 < s_end ? (uint32_t)h[1] << 16 : 0u);
                }
            }
        }
        return m;
    };
    // Transpose: bit i of lane l's mask -> bit l of the axon word of sample i.
    auto transpose = [&](uint32_t m, int buf) {
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const unsigned long long b = __ballot((m >> i) & 1u);
            if (lane == 0) {
                x_lds[buf][part * SPT + i][2 * (wave % APW)] = (uint32_t)b;
                x_lds[buf][part * SPT + i][2 * (wave % APW) + 1] = (uint32_t)(b >> 32);
            }
        }
    };
    // external input words of the 4 samples this wave expands
    uint32_t xe[4][QPL];
    auto load_ext = [&](int s0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int s = s0 + wave + 16 * m;
#pragma unroll
            for (int qi = 0; qi < QPL; ++qi) {
                const int q = lane + 64 * qi;
                xe[m][qi] = (q < QD && s < s_end && ext_c) ? ext_c[(size_t)s * ta.ext_sstride + (q >> 3)] : 0u;
            }
        }
    };

    transpose(load_mask(s_begin), 0);
    uint32_t mnext = load_mask(s_begin + MFMA_TS);
    load_ext(s_begin);
    __syncthreads();

    int it = 0;
    for (int s0 = s_begin; s0 < s_end; s0 += MFMA_TS, ++it) {
        int8_t *A = a_lds[it & 1];
        // 1. expand delivered | external spikes to int8, count delivered spikes
        //    and synaptic events
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int i = wave + 16 * m;
            unsigned pk = 0;
#pragma unroll
            for (int qi = 0; qi < QPL; ++qi) {
                const int q = lane + 64 * qi;
                if (q < QD) {
                    const uint32_t xd = x_lds[it & 1][i][q >> 3];
                    const uint32_t x = xd | xe[m][qi];
                    const uint32_t nib = (x >> (4 * (q & 7))) & 0xFu;
                    // nibble b3b2b1b0 -> bytes 0/1: bit i moves to bit 8i, no carries
                    *reinterpret_cast<uint32_t *>(&A[i * ROWB + 4 * q]) = (nib * 0x00204081u) & 0x01010101u;
                    pk += (nib & 1u) * degv[qi][0] + ((nib >> 1) & 1u) * degv[qi][1] +
                          ((nib >> 2) & 1u) * degv[qi][2] + ((nib >> 3) & 1u) * degv[qi][3];
                    if ((q & 7) == 0)
                        pk += (unsigned)__popc(xd) << EV_BITS;
                }
            }
            pk = wave_sum(pk);
            const int s = s0 + i;
            if (lane == 0 && s < s_end) {
                s_cnt[3][s - s_begin] += pk >> EV_BITS;
                s_cnt[4][s - s_begin] += pk & ((1u << EV_BITS) - 1u);
            }
        }
        // 2. potentials of this tile; delivered spikes of the next tile into
        //    LDS; history loads of the tile after; next tile's external input
        v4i vold[STW];
#pragma unroll
        for (int t = 0; t < STW; ++t) {
            const int sb = s0 + (stg * STW + t) * 16;
            vold[t] = sb < s_end16 ? __builtin_nontemporal_load(vb_in + (size_t)(sb >> 4) * 64) : v4i{0, 0, 0, 0};
        }
        if (s0 + MFMA_TS < s_end) {
            transpose(mnext, (it + 1) & 1);
            mnext = load_mask(s0 + 2 * MFMA_TS);
            load_ext(s0 + MFMA_TS);
        }
        __syncthreads();

        // 3. products and potential update
#pragma unroll
        for (int t = 0; t < STW; ++t) {
            const int st = stg * STW + t;
            const int sb = s0 + st * 16;
            if (sb >= s_end16)
                continue;
            v4i acc = {0, 0, 0, 0};
            const int8_t *arow = &A[(st * 16 + jj) * ROWB + 16 * g4];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const v4i a = *reinterpret_cast<const v4i *>(arow + 64 * k);
                if (TWO) {
                    const v4i ah = a << 7;
                    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah, breg[k][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, breg[k][1], acc, 0, 0, 0);
                } else {
                    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, breg[k][0], acc, 0, 0, 0);
                }
            }
            v4i vnew;
            unsigned long long bal[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = sb + 4 * g4 + r;
                int32_t vn;
                const bool fire = lif_update(vold[t][r], acc[r], lk, th, rs, n.vmin, n.vmax, vn) && s < s_end;
                vnew[r] = vn;
                bal[r] = __ballot(fire);
            }
            __builtin_nontemporal_store(vnew, vb_out + (size_t)(sb >> 4) * 64);
            // this tick's spikes of neuron 16nb + jj for the 16 samples of the
            // sub-tile, sample-sliced, into history slot t % Q
            uint32_t m16 = 0;
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t half = (uint32_t)(bal[r] >> (16 * g)) & 0xFFFFu;
                    m16 |= ((half >> jj) & 1u) << (4 * g + r);
                }
            if (g4 == 0)
                hist_out[sb >> 4] = (uint16_t)m16;
            if (jj < 4) {
                const int i = st * 16 + 4 * g4 + jj;
                const int s = s0 + i;
                if (s < s_end) {
                    const unsigned long long bs = jj == 0 ? bal[0] : jj == 1 ? bal[1] : jj == 2 ? bal[2] : bal[3];
                    const uint32_t hw = (uint32_t)(bs >> (16 * g4)) & 0xFFFFu;
                    if (hw) {
                        atomicAdd(&s_cnt[0][s - s_begin], (unsigned)__popc(hw));
                        atomicAdd(&s_cnt[1][s - s_begin], (unsigned)__popc(hw & cm16));
                        atomicAdd(&s_cnt[2][s - s_begin], (unsigned)__popc(hw & om16));
                    }
                    if (ow >= 0)
                        reinterpret_cast<uint16_t *>(n.raster)[(((size_t)ta.r_row * n.S + s) * n.Wout + ow) * 2 +
                                                               (nb & 1)] = (uint16_t)(hw & om16);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s_end - s_begin; i += blockDim.x) {
        unsigned long long *cp = n.cnt + ((size_t)c * n.S + s_begin + i) * CNT_N;
        cp[CNT_EMITTED] += s_cnt[0][i];
        cp[CNT_ROUTED] += s_cnt[1][i];
        cp[CNT_OUT] += s_cnt[2][i];
        cp[CNT_DELIVERED] += s_cnt[3][i];
        cp[CNT_EVENTS] += s_cnt[4][i];
    }
}

bool mfma_shape_supported(int A, int N, int two_planes)
{
    const bool ok_a = A == 64 || A == 128 || A == 256 || A == 512;
    const bool ok_n = N == 64 || N == 128 || N == 256 || N == 512;
    // B tiles must fit in 32 VGPRs per lane (A * N * planes / 4096) with one
    // neuron block per wavefront; larger cores would spill. 512-axon cores
    // with two planes also spill (wider expansion state).
    return ok_a && ok_n && N <= 256 && (long)A * N * (two_planes ? 2 : 1) <= (1L << 17) &&
           !(A == 512 && two_planes);
}

template <int A_, int N_>
static hipError_t launch_mfma_an(const DevNet &n, const TickArgs &a, int two, int spw, hipStream_t st)
{
    const int chunks = (n.S + spw - 1) / spw;
    const dim3 grid(n.C * chunks), block(1024);
    if constexpr ((long)A_ * N_ * 2 <= (1L << 17) && A_ < 512) {
        if (two)
            hipLaunchKernelGGL((k_integrate_mfma<A_, N_, true>), grid, block, 0, st, n, a, spw);
        else
            hipLaunchKernelGGL((k_integrate_mfma<A_, N_, false>), grid, block, 0, st, n, a, spw);
    } else if constexpr ((long)A_ * N_ <= (1L << 17)) {
        if (two)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_integrate_mfma<A_, N_, false>), grid, block, 0, st, n, a, spw);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int A_>
static hipError_t launch_mfma_a(const DevNet &n, const TickArgs &a, int two, int spw, hipStream_t st)
{
    switch (n.N) {
    case 64: return launch_mfma_an<A_, 64>(n, a, two, spw, st);
    case 128: return launch_mfma_an<A_, 128>(n, a, two, spw, st);
    case 256: return launch_mfma_an<A_, 256>(n, a, two, spw, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_integrate_mfma(const DevNet &n, const TickArgs &a, int two_planes, int samples_per_wg,
                                 hipStream_t st)
{
    if (!mfma_shape_supported(n.A, n.N, two_planes) || samples_per_wg <= 0 || samples_per_wg % MFMA_TS ||
        samples_per_wg > MFMA_SPW_MAX || n.vlayout != VLAYOUT_BRICK)
        return hipErrorInvalidValue;
    switch (n.A) {
    case 64: return launch_mfma_a<64>(n, a, two_planes, samples_per_wg, st);
    case 128: return launch_mfma_a<128>(n, a, two_planes, samples_per_wg, st);
    case 256: return launch_mfma_a<256>(n, a, two_planes, samples_per_wg, st);
    case 512: return launch_mfma_a<512>(n, a, two_planes, samples_per_wg, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ranc
