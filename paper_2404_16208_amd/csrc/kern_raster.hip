// kern_raster.hip -- the output file of Sec. IV in bulk: the output-bus spikes
// of every sample over a range of retained ticks, packed into one bit array
// the caller owns, so that a run can be drained chunk by chunk while the next
// chunk runs (streaming, Sec. V) and the host decodes off the critical path.
//
// Output neurons are numbered in ascending (core, neuron) order among the
// neurons whose destination is the output bus. Two layouts:
//   by neuron: u64 [T][Nout][HG], HG = ceil(S / 64); bit i of word (t, o, w)
//              = sample 64 w + i spiked from output neuron o at tick t0 + t;
//   by sample: u32 [T][S][ceil(Nout / 32)]; bit o % 32 of word (t, s, o / 32)
//              = the same event (the compact form for few samples).
// Bits of samples >= S and of output neurons >= Nout are zero; every word of
// the range is written.
//
// Sources: the MFMA and event-driven paths keep the raster neuron-major
// already (history words; on the MFMA path the bits of each 32-sample half
// follow the MFMA result row order sigma32 and are permuted back); the plain
// path keeps, per sample, the cores' neuron words that hold output neurons
// (raster columns).
#include <algorithm>

#include "kern_bits.h"
#include "ranc_internal.h"

namespace ranc {

// Sample-ordered 32-bit word from an MFMA-ordered one: bit i of the result is
// bit sigma32_inv(i) of x.
__device__ inline uint32_t unsigma32(uint32_t x)
{
    uint32_t y = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i)
        y |= ((x >> sigma32_inv(i)) & 1u) << i;
    return y;
}

// Sample (within its 64-sample tile) of bit p of a history word.
__device__ inline int sample_of_bit(const DevNet &n, int p)
{
    return n.vlayout == VLAYOUT_BRICK ? 32 * (p >> 5) + sigma32(p & 31) : p;
}

// ---- by neuron

__global__ __launch_bounds__(256) void k_raster_hist_by_neuron(DevNet n, long long t0, int T, uint64_t *dst)
{
    const long long HG = n.S64 / 64;
    const long long total = (long long)T * n.Nout * HG;
    const bool mfma = n.vlayout == VLAYOUT_BRICK;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(n.raster);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long t = i / ((long long)n.Nout * HG);
        const long long rest = i - t * n.Nout * HG;   // o * HG + w
        const int row = (int)((t0 + t) % n.RT);
        uint64_t w = src[(size_t)row * n.Nout * HG + rest];
        if (mfma)
            w = (uint64_t)unsigma32((uint32_t)w) | (uint64_t)unsigma32((uint32_t)(w >> 32)) << 32;
        dst[i] = w;
    }
}

// outcol[ow] = (index c * NW + w of raster column ow's neuron word, output
// index of the column's first output neuron). One wavefront per (tick, raster
// column, 64 samples), lane = sample.
__global__ __launch_bounds__(256) void k_raster_plain_by_neuron(DevNet n, const int2 *outcol, long long t0, int T,
                                                                uint64_t *dst)
{
    const int HG = n.S64 / 64;
    const long long wv = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv >= (long long)T * n.Wout * HG)
        return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int w = (int)(wv % HG);
    const long long r = wv / HG;
    const int ow = (int)(r % n.Wout);
    const int t = (int)(r / n.Wout);
    const int row = (int)((t0 + t) % n.RT);
    const int s = 64 * w + lane;
    const uint32_t word = s < n.S ? n.raster[((size_t)row * n.S + s) * n.Wout + ow] : 0u;
    const int2 oc = outcol[ow];
    uint32_t mask = n.outmask[oc.x];   // uniform
    int o = oc.y;
    uint64_t *drow = dst + ((size_t)t * n.Nout) * HG + w;
    while (mask) {
        const int b = __builtin_ctz(mask);
        mask &= mask - 1u;
        const uint64_t bits = __ballot((word >> b) & 1u);
        if (lane == 0)
            drow[(size_t)o * HG] = bits;
        ++o;
    }
}

// ---- by sample

// Workgroup (tick, 64-sample tile, block of 256 output neurons); wave w forms
// the words of output-neuron groups 2w and 2w + 1 (32 neurons each) for the
// 64 samples, lane = bit of the history word, from 32 wave-uniform history
// loads per group; the 64 x 8 words go through LDS so that each sample's 8
// words are written as one 32-byte run.
__global__ __launch_bounds__(256) void k_raster_hist_by_sample(DevNet n, long long t0, int T, uint32_t *dst)
{
    __shared__ uint32_t sw[64][9];
    const int HG = n.S64 / 64;
    const int NOW = (n.Nout + 31) / 32;
    const int OB = (n.Nout + 255) / 256;
    const int ob = blockIdx.x % OB;
    const int tile = (blockIdx.x / OB) % HG;
    const int t = blockIdx.x / (OB * HG);
    const int row = (int)((t0 + t) % n.RT);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(n.raster) + (size_t)row * n.Nout * HG + tile;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int g = 2 * wave + h;
        const int o0 = 256 * ob + 32 * g;
        uint32_t word = 0;
        for (int k = 0; k < 32; ++k) {
            const int o = o0 + k;
            const uint64_t w = o < n.Nout ? src[(size_t)o * HG] : 0ull;
            word |= (uint32_t)((w >> lane) & 1ull) << k;
        }
        sw[sample_of_bit(n, lane)][g] = word;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 8; i += 256) {
        const int sl = i >> 3, g = i & 7;
        const int s = 64 * tile + sl, dw = 8 * ob + g;
        if (s < n.S && dw < NOW)
            dst[((size_t)t * n.S + s) * NOW + dw] = sw[sl][g];
    }
}

// opos[o] = raster column of output neuron o << 5 | its bit in the column.
// One thread per (tick, sample, output word).
__global__ __launch_bounds__(256) void k_raster_plain_by_sample(DevNet n, const int32_t *opos, long long t0, int T,
                                                                uint32_t *dst)
{
    const int NOW = (n.Nout + 31) / 32;
    const long long total = (long long)T * n.S * NOW;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int dw = (int)(i % NOW);
        const long long ts = i / NOW;   // t * S + s
        const int s = (int)(ts % n.S);
        const int t = (int)(ts / n.S);
        const int row = (int)((t0 + t) % n.RT);
        const uint32_t *rrow = n.raster + ((size_t)row * n.S + s) * n.Wout;
        uint32_t word = 0;
        const int kmax = min(32, n.Nout - 32 * dw);
        for (int k = 0; k < kmax; ++k) {
            const int p = opos[32 * dw + k];
            word |= ((rrow[p >> 5] >> (p & 31)) & 1u) << k;
        }
        dst[i] = word;
    }
}

hipError_t launch_pack_raster(const DevNet &n, const int2 *outcol, const int32_t *opos, int by_sample, long long t0,
                              int T, void *dst, hipStream_t st)
{
    if (T < 1 || !dst)
        return hipErrorInvalidValue;
    if (n.Nout == 0)
        return hipSuccess;
    const bool plain = n.vlayout == VLAYOUT_CSN;
    if (plain && !(by_sample ? (const void *)opos : (const void *)outcol))
        return hipErrorInvalidValue;
    const int HG = n.S64 / 64;
    if (by_sample) {
        uint32_t *d = static_cast<uint32_t *>(dst);
        if (plain) {
            const long long total = (long long)T * n.S * ((n.Nout + 31) / 32);
            const long long blocks = std::min<long long>((total + 255) / 256, 16384);
            hipLaunchKernelGGL(k_raster_plain_by_sample, dim3((unsigned)blocks), dim3(256), 0, st, n, opos, t0, T, d);
        } else {
            const long long blocks = (long long)T * HG * ((n.Nout + 255) / 256);
            hipLaunchKernelGGL(k_raster_hist_by_sample, dim3((unsigned)blocks), dim3(256), 0, st, n, t0, T, d);
        }
    } else {
        uint64_t *d = static_cast<uint64_t *>(dst);
        if (plain) {
            const long long waves = (long long)T * n.Wout * HG;
            hipLaunchKernelGGL(k_raster_plain_by_neuron, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, n,
                               outcol, t0, T, d);
        } else {
            const long long total = (long long)T * n.Nout * HG;
            const long long blocks = std::min<long long>((total + 255) / 256, 8192);
            hipLaunchKernelGGL(k_raster_hist_by_neuron, dim3((unsigned)blocks), dim3(256), 0, st, n, t0, T, d);
        }
    }
    return hipGetLastError();
}

}  // namespace ranc
