// kern_mfma.hip -- one tick of integrate + leak/threshold/reset on int8 MFMA.
//
// With many samples, the integration of one core (GPU-RANC Sec. II: sum over
// spiking connected axons of the neuron's weight for the axon's type) is the
// dense product X[samples x A] * B[A x N] with X the 0/1 axon spikes and
// B[a][n] = crossbar(a, n) * weight(n, type(a)). It runs on
// V_MFMA_I32_16X16X64_I8 with int32 accumulation, which is exact:
//   - weights of up to 8 bits are int8 as they are (one B plane);
//   - 9-bit weights w in [-256, 255] are split as w = 128*hi + lo with
//     lo = w & 127 in [0, 127] and hi = w >> 7 in [-2, 1]. The hi term is
//     formed as (-128 * x) * (-hi): the spike byte shifted left by 7 is the
//     int8 value -128, and -hi lies in [-1, 2], so both planes accumulate into
//     the same int32 register and no rescaling pass is needed.
//   |sum| <= 512 * 256 < 2^31, so int32 never overflows.
//
// Mapping: one workgroup of 16 wavefronts per (core, chunk of samples); the
// core's B tiles stay in VGPRs for the whole chunk (A*N*planes/4096 VGPRs per
// lane). Samples are taken 64 at a time: the spike bits are expanded to an
// int8 [64 x A] tile in LDS once (shared by all wavefronts), then each
// wavefront multiplies 16-sample sub-tiles against its 16-neuron block(s) and
// applies the potential update in the epilogue (V is [C][S][N], so a wave's
// 16 neurons of one sample are 64 contiguous bytes). Spikes leave as 16-bit
// ballot halves, i.e. the same bytes as the 32-bit spike words of the plain
// path. Synaptic events are counted during the expansion as sum over spiking
// axons of their number of connected neurons.
//
// MFMA operand convention used for both A and B: in k-step k, lane l holds 16
// bytes for row/column l % 16 and axons 64k + 16*(l/16) + [0, 16). The sum
// over k does not depend on which hardware k each byte stands for as long as
// A and B agree. Result: lane l, element r is row 4*(l/16) + r, column l % 16.
#include "kern_common.h"
#include "ranc_internal.h"

namespace ranc {

typedef int v4i __attribute__((ext_vector_type(4)));

static constexpr int MFMA_TS = 64;  // samples per LDS tile

template <int A_, int N_, bool TWO>
__global__ __launch_bounds__(1024) void k_integrate_mfma(DevNet n, TickArgs ta, int spw)
{
    constexpr int NB = N_ / 16;                     // 16-neuron blocks
    constexpr int KS = A_ / 64;                     // 64-axon k-steps
    constexpr int PL = TWO ? 2 : 1;                 // B planes
    constexpr int NBW = NB > 16 ? NB / 16 : 1;      // neuron blocks per wave
    constexpr int WPB = NB >= 16 ? 1 : 16 / NB;     // waves sharing a neuron block
    constexpr int STW = 4 / WPB;                    // 16-sample sub-tiles per wave per tile
    constexpr int W_ = A_ / 32;
    constexpr int NW_ = N_ / 32;
    constexpr int ROWB = A_ + 16;                   // padded LDS row (bytes)
    constexpr int QD = A_ / 4;                      // axon dwords per sample row
    constexpr int QPL = (QD + 63) / 64;             // axon dwords per lane in the expansion

    __shared__ __attribute__((aligned(16))) int8_t a_lds[MFMA_TS * ROWB];
    __shared__ unsigned s_cnt[MFMA_TS][5];          // emitted, routed, out, delivered, events

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x % n.C;
    const int chunk = blockIdx.x / n.C;
    const int s_begin = chunk * spw;
    const int s_end = min(n.S, s_begin + spw);
    const int g4 = lane >> 4, jj = lane & 15;

    // B tiles of this wave's neuron block(s), resident for the whole chunk.
    v4i breg[NBW][KS][PL];
    int nbs[NBW];
    int32_t lk[NBW], th[NBW], rs[NBW];
    const v4i *planes = reinterpret_cast<const v4i *>(n.planes);
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
        const int nb = NB >= 16 ? wave + 16 * b : wave % NB;
        nbs[b] = nb;
#pragma unroll
        for (int k = 0; k < KS; ++k)
#pragma unroll
            for (int p = 0; p < PL; ++p)
                breg[b][k][p] = planes[((((size_t)c * NB + nb) * KS + k) * PL + p) * 64 + lane];
        const size_t cj = (size_t)c * N_ + nb * 16 + jj;
        lk[b] = n.leak[cj];
        th[b] = n.thr[cj];
        rs[b] = n.rst[cj];
    }
    const int stg = NB >= 16 ? 0 : wave / NB;

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
    const uint32_t *slot_c = n.ring + (size_t)ta.q_now * n.S * n.C * W_ + (size_t)c * W_;

    for (int s0 = s_begin; s0 < s_end; s0 += MFMA_TS) {
        // Expand the axon spikes of 64 samples to an int8 tile.
        for (int i = wave; i < MFMA_TS; i += 16) {
            const int s = s0 + i;
            const bool valid = s < s_end;
            unsigned dl = 0, ev = 0;
#pragma unroll
            for (int qi = 0; qi < QPL; ++qi) {
                const int q = lane + 64 * qi;
                if (q < QD) {
                    uint32_t x = 0;
                    if (valid) {
                        const uint32_t r = slot_c[(size_t)s * n.C * W_ + (q >> 3)];
                        if ((q & 7) == 0)
                            dl += __popc(r);
                        x = r | (ext_c ? ext_c[(size_t)s * ta.ext_sstride + (q >> 3)] : 0u);
                    }
                    const uint32_t nib = (x >> (4 * (q & 7))) & 0xFu;
                    // nibble b3b2b1b0 -> bytes 0/1: bit i moves to bit 8i, no carries
                    *reinterpret_cast<uint32_t *>(&a_lds[i * ROWB + 4 * q]) = (nib * 0x00204081u) & 0x01010101u;
                    ev += (nib & 1u) * degv[qi][0] + ((nib >> 1) & 1u) * degv[qi][1] +
                          ((nib >> 2) & 1u) * degv[qi][2] + ((nib >> 3) & 1u) * degv[qi][3];
                }
            }
            dl = wave_sum(dl);
            ev = wave_sum(ev);
            if (lane == 0) {
                s_cnt[i][0] = 0;
                s_cnt[i][1] = 0;
                s_cnt[i][2] = 0;
                s_cnt[i][3] = dl;
                s_cnt[i][4] = ev;
            }
        }
        __syncthreads();

#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            const int nb = nbs[b];
            const size_t mword = (size_t)c * NW_ + (nb >> 1);
            const int hsh = 16 * (nb & 1);
            const uint32_t cm16 = (n.coremask[mword] >> hsh) & 0xFFFFu;
            const uint32_t om16 = (n.outmask[mword] >> hsh) & 0xFFFFu;
            const int ow = n.outword[mword];
            for (int t = 0; t < STW; ++t) {
                const int st = stg * STW + t;
                // Potentials of this sub-tile (issued before the products).
                int32_t vold[4];
                size_t vidx[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int s = s0 + st * 16 + 4 * g4 + r;
                    vidx[r] = ((size_t)c * n.S + s) * N_ + nb * 16 + jj;
                    vold[r] = s < s_end ? n.V[vidx[r]] : 0;
                }
                v4i acc = {0, 0, 0, 0};
                const int8_t *arow = &a_lds[(st * 16 + jj) * ROWB + 16 * g4];
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const v4i a = *reinterpret_cast<const v4i *>(arow + 64 * k);
                    if (TWO) {
                        const v4i ah = a << 7;
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah, breg[b][k][0], acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, breg[b][k][1], acc, 0, 0, 0);
                    } else {
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, breg[b][k][0], acc, 0, 0, 0);
                    }
                }
                unsigned long long bal[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int s = s0 + st * 16 + 4 * g4 + r;
                    int32_t vnew;
                    const bool fire = lif_update(vold[r], acc[r], lk[b], th[b], rs[b], n.vmin, n.vmax, vnew) &&
                                      s < s_end;
                    if (s < s_end)
                        n.V[vidx[r]] = vnew;
                    bal[r] = __ballot(fire);
                }
                if (jj < 4) {
                    const int i = st * 16 + 4 * g4 + jj;
                    const int s = s0 + i;
                    if (s < s_end) {
                        const unsigned long long bs = jj == 0 ? bal[0] : jj == 1 ? bal[1] : jj == 2 ? bal[2] : bal[3];
                        const uint32_t hw = (uint32_t)(bs >> (16 * g4)) & 0xFFFFu;
                        reinterpret_cast<uint16_t *>(n.spk)[((size_t)s * n.C + c) * NB + nb] = (uint16_t)hw;
                        atomicAdd(&s_cnt[i][0], (unsigned)__popc(hw));
                        atomicAdd(&s_cnt[i][1], (unsigned)__popc(hw & cm16));
                        atomicAdd(&s_cnt[i][2], (unsigned)__popc(hw & om16));
                        if (ow >= 0)
                            reinterpret_cast<uint16_t *>(n.raster)[(((size_t)ta.r_row * n.S + s) * n.Wout + ow) * 2 +
                                                                   (nb & 1)] = (uint16_t)(hw & om16);
                    }
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < MFMA_TS) {
            const int s = s0 + threadIdx.x;
            if (s < s_end) {
                unsigned long long *cp = n.cnt + ((size_t)c * n.S + s) * CNT_N;
                cp[CNT_EMITTED] += s_cnt[threadIdx.x][0];
                cp[CNT_ROUTED] += s_cnt[threadIdx.x][1];
                cp[CNT_OUT] += s_cnt[threadIdx.x][2];
                cp[CNT_DELIVERED] += s_cnt[threadIdx.x][3];
                cp[CNT_EVENTS] += s_cnt[threadIdx.x][4];
            }
        }
        __syncthreads();
    }
}

bool mfma_shape_supported(int A, int N, int two_planes)
{
    const bool ok_a = A == 64 || A == 128 || A == 256 || A == 512;
    const bool ok_n = N == 64 || N == 128 || N == 256 || N == 512;
    // B tiles must fit in 32 VGPRs per lane (A * N * planes / 4096) with one
    // neuron block per wavefront; larger cores would spill.
    // 512-axon cores with two planes also spill (wider expansion state).
    return ok_a && ok_n && N <= 256 && (long)A * N * (two_planes ? 2 : 1) <= (1L << 17) &&
           !(A == 512 && two_planes);
}

template <int A_, int N_>
static hipError_t launch_mfma_an(const DevNet &n, const TickArgs &a, int two, int spw, hipStream_t st)
{
    const int chunks = (n.S + spw - 1) / spw;
    const dim3 grid(n.C * chunks), block(1024);
    if constexpr (N_ <= 256 && (long)A_ * N_ * 2 <= (1L << 17) && A_ < 512) {
        if (two)
            hipLaunchKernelGGL((k_integrate_mfma<A_, N_, true>), grid, block, 0, st, n, a, spw);
        else
            hipLaunchKernelGGL((k_integrate_mfma<A_, N_, false>), grid, block, 0, st, n, a, spw);
    } else if constexpr (N_ <= 256 && (long)A_ * N_ <= (1L << 17)) {
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
    if (!mfma_shape_supported(n.A, n.N, two_planes) || samples_per_wg <= 0 || samples_per_wg % MFMA_TS)
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
