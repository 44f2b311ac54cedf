// kern_links.hip -- packets per mesh link, per sample, for the tick just run.
//
// GPU-RANC Sec. III-D (Fig. 2): a spike packet reaches its destination core
// through the routers of the cores between, along x first, then along y; the
// simulation itself delivers it directly (the destination is known at load
// time), so which mesh links the packet would have taken is a statistic of
// its own. A packet from core (xs, ys) with offset (dx, dy) leaves every core
// (x, ys) with x from xs up to (not including) xd = xs + dx over its x link
// (+x or -x), then every core (xd, y) with y from ys up to yd = ys + dy over
// its y link.
//
// Each such run of links along a mesh row or column is recorded as two
// entries of a difference array per direction, +1 where the run starts and -1
// where it ends; a prefix sum along the row (+x), the row reversed (-x), the
// column (+y) or the column reversed (-y) then gives every link's count. The
// sums are taken when the counts are read, so a tick costs at most three
// entries per packet: the run starts at the source core are the same for all
// of a core's neurons and are added once per core and sample. Entries are
// 64-bit and signed (two's complement in unsigned atomics).
//
// Sample-tiled paths (MFMA, event-driven), where the tick's spikes are
// history words (64 samples of one neuron per word): the entries are gathered
// by the difference-array row they land on. At load, every (direction, core)
// row gets the list of its entries (source neuron, +1 or -1). One wavefront
// per (row, 64-sample word) reads the history words of 64 listed neurons at a
// time (lane = entry), transposes the 64 x 64 bit block so that a lane holds
// one sample's bits of those entries, and adds popcount(+1 entries) -
// popcount(-1 entries): the row's 64 counters of that word are the
// wavefront's alone, so they are updated without atomics. The wavefronts of
// one row (its 64-sample words) run in one workgroup and read the same
// history lines (a neuron's words are consecutive).
//
// Plain path (spike words per (sample, core)): one wavefront per (core,
// 64-sample word), lane = sample. The neurons' spike words of the tick and
// their precomputed path ends are read 64 neurons at a time, one per lane,
// and walked neuron by neuron with the word of the current neuron broadcast
// from its lane; entries are atomic adds into [direction][core][S64]
// (consecutive samples at consecutive addresses).
#include "kern_bits.h"
#include "ranc_internal.h"

namespace ranc {

static constexpr int LINK_WAVES = 4;   // wavefronts per workgroup

__global__ __launch_bounds__(64 * LINK_WAVES) void k_link_counts(DevNet n, LinkArgs l, int k)
{
    const int HG = n.S64 / 64;
    const int wv = blockIdx.x * LINK_WAVES + (int)(threadIdx.x >> 6);
    if (wv >= n.C * HG)
        return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int c = wv / HG, i = wv - c * HG;
    const int s = 64 * i + lane;   // this lane's sample
    const bool live = s < n.S;
    const size_t CS = (size_t)n.C * n.S64;
    unsigned long long *D = reinterpret_cast<unsigned long long *>(l.d);
    unsigned src_xp = 0, src_xm = 0, src_yp = 0, src_ym = 0;   // runs that start at this core
    for (int jb = 0; jb < n.N; jb += 64) {
        const size_t g = (size_t)c * n.N + jb + lane;
        const int2 rec = l.rec[g];
        uint32_t sw0 = 0, sw1 = 0;
        if (live) {
            const uint32_t *sp = n.spk + ((size_t)s * n.C + c) * n.NW + jb / 32;
            sw0 = sp[0];
            sw1 = sp[1];
        }
        for (int q = 0; q < 64; ++q) {
            const int xc = __builtin_amdgcn_readlane(rec.x, q);
            const int yc = __builtin_amdgcn_readlane(rec.y, q);
            if ((xc & yc) < 0)
                continue;   // no hop (not routed to a core, or to its own core)
            const bool fire = (((q < 32 ? sw0 : sw1) >> (q & 31)) & 1u) != 0u;
            if (!__ballot(fire))
                continue;
            if (xc >= 0) {
                if (xc & 1)
                    src_xm += fire;
                else
                    src_xp += fire;
                if (fire)
                    atomicAdd(&D[(size_t)(xc & 1) * CS + (size_t)(xc >> 1) * n.S64 + s], ~0ull);
            }
            if (yc >= 0) {
                const int dir = 2 + (yc & 1);
                if (xc < 0) {
                    if (yc & 1)
                        src_ym += fire;
                    else
                        src_yp += fire;
                } else if (fire) {
                    atomicAdd(&D[(size_t)dir * CS + (size_t)(xc >> 1) * n.S64 + s], 1ull);
                }
                if (fire)
                    atomicAdd(&D[(size_t)dir * CS + (size_t)(yc >> 1) * n.S64 + s], ~0ull);
            }
        }
    }
    const size_t at = (size_t)c * n.S64 + s;
    if (src_xp)
        atomicAdd(&D[at], (unsigned long long)src_xp);
    if (src_xm)
        atomicAdd(&D[CS + at], (unsigned long long)src_xm);
    if (src_yp)
        atomicAdd(&D[2 * CS + at], (unsigned long long)src_yp);
    if (src_ym)
        atomicAdd(&D[3 * CS + at], (unsigned long long)src_ym);
}

static constexpr int LINK_GATHER_WAVES = 16;   // wavefronts per workgroup of the gather form

__global__ __launch_bounds__(64 * LINK_GATHER_WAVES) void k_link_counts_gather(DevNet n, LinkArgs l, int k)
{
    const int HG = n.S64 / 64;
    const long long wv = (long long)blockIdx.x * LINK_GATHER_WAVES + (threadIdx.x >> 6);
    if (wv >= 4LL * n.C * HG)
        return;   // whole wavefronts
    const int lane = threadIdx.x & 63;
    const int row = (int)(wv / HG);   // direction * C + core
    const int i = (int)(wv - (long long)row * HG);
    const size_t CN = (size_t)n.C * n.N;
    const int slot = tick_slot(n, k);
    const uint32_t b = l.rows[row], e = l.rows[row + 1];
    int acc_lo = 0, acc_hi = 0;   // lanes x < 32: history bits x and 32 + x of word i
    for (uint32_t c0 = b; c0 < e; c0 += 64) {
        uint64_t w = 0;
        bool neg = false;
        if (c0 + lane < e) {
            const uint32_t en = l.ents[c0 + lane];
            neg = (en & 1u) != 0u;
            w = n.hist[((size_t)slot * CN + (en >> 1)) * HG + i];
        }
        // lane (h, x): bit j = history bit x (tl) or 32 + x (th) of entry 32 h + j
        const uint32_t m = (uint32_t)(__ballot(neg) >> (32 * (lane >> 5)));
        const uint32_t tl = transpose32((uint32_t)w, lane), th = transpose32((uint32_t)(w >> 32), lane);
        int cl = __popc(tl & ~m) - __popc(tl & m);
        int ch = __popc(th & ~m) - __popc(th & m);
        acc_lo += cl + __shfl_xor(cl, 32, 64);
        acc_hi += ch + __shfl_xor(ch, 32, 64);
    }
    if (lane < 32) {
        // sample of history bit p: the MFMA result row order within each
        // 32-sample half on the MFMA path, else bit p = sample p
        const bool mf = n.vlayout == VLAYOUT_BRICK;
        const int s_lo = 64 * i + (mf ? sigma32(lane) : lane);
        const int s_hi = 64 * i + 32 + (mf ? sigma32(lane) : lane);
        unsigned long long *D = reinterpret_cast<unsigned long long *>(l.d) + (size_t)row * n.S64;
        if (acc_lo)
            D[s_lo] += (unsigned long long)(long long)acc_lo;
        if (acc_hi)
            D[s_hi] += (unsigned long long)(long long)acc_hi;
    }
}

hipError_t launch_link_counts(const DevNet &n, const LinkArgs &l, int k, hipStream_t st)
{
    if (n.N % 64 || !l.d || !l.rec)
        return hipErrorInvalidValue;
    if (n.vlayout != VLAYOUT_CSN) {
        if (!l.rows || !l.ents)
            return hipErrorInvalidValue;
        const long long waves = 4LL * n.C * (n.S64 / 64);
        const dim3 grid((unsigned)((waves + LINK_GATHER_WAVES - 1) / LINK_GATHER_WAVES)),
            block(64 * LINK_GATHER_WAVES);
        hipLaunchKernelGGL(k_link_counts_gather, grid, block, 0, st, n, l, k);
        return hipGetLastError();
    }
    const long long waves = (long long)n.C * (n.S64 / 64);
    const dim3 grid((unsigned)((waves + LINK_WAVES - 1) / LINK_WAVES)), block(64 * LINK_WAVES);
    hipLaunchKernelGGL(k_link_counts, grid, block, 0, st, n, l, k);
    return hipGetLastError();
}

}  // namespace ranc
