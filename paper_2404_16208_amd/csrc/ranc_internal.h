// ranc_internal.h -- device data layout shared by the host runtime and the kernels.
//
// Notation: C cores, A axons and N neurons per core, G axon types,
// W = A/32 axon words, NW = N/32 neuron words, D = max delay, Q = D + 1
// scheduler slots, S samples, RT retained raster ticks, Wout output words.
//
// Parameters (written once at load):
//   colbits  u32 [C][W][N]     bit b of colbits[c][w][n] = crossbar(c, 32w+b, n)
//   typemask u32 [C][G][W]     bit b of typemask[c][g][w] = (type(c, 32w+b) == g)
//   wts      i32 [C][G][N]     weight of neuron n for axon type g
//   leak, thr, rst, vinit i32 [C][N]
//   coremask, outmask u32 [C][NW]  neurons whose destination is a core / the output bus
//   outword  i32 [C][NW]       raster column of that neuron word, -1 if it has no output neuron
//   in_index i32 [C]           input slot of the core, -1 if it takes no external input
//   rt_ptr   u32 [C*W*D + 1]   CSR over (destination core, axon word, delay-1):
//   rt_src   u32 [E]           (source neuron g = c*N + n) << 5 | (destination axon % 32)
//   deg      i32 [C][A]        connected neurons per axon (synaptic-event counter, MFMA path)
//   planes   int8 MFMA B operand tiles (MFMA path), see kern_mfma.hip
// State:
//   V        i32 [C][S][N]
//   ring     u32 [Q][S][C][W]  scheduler: slot t%Q holds the axon spikes of tick t
//   spk      u32 [S][C][NW]    spikes of the current tick
//   raster   u32 [RT][S][Wout] output-bus spikes of tick t in row t%RT
//   cnt      u64 [C][S][5]     emitted, routed, delivered, out, events
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranc {

enum { CNT_EMITTED = 0, CNT_ROUTED, CNT_DELIVERED, CNT_OUT, CNT_EVENTS, CNT_N };

struct DevNet {
    int C, A, N, G, W, NW, D, Q, S, RT, Wout, Cin;
    int32_t vmin, vmax;
    // parameters
    const uint32_t *colbits, *typemask;
    const int32_t *wts, *leak, *thr, *rst, *vinit;
    const uint32_t *coremask, *outmask;
    const int32_t *outword, *in_index;
    const uint32_t *rt_ptr, *rt_src;
    const int32_t *deg;
    const uint4 *planes;
    // state
    int32_t *V;
    uint32_t *ring, *spk, *raster;
    unsigned long long *cnt;
};

// Per-tick launch arguments.
struct TickArgs {
    int q_now;              // t % Q
    int r_row;              // t % RT
    const uint32_t *ext_t;  // external input of this tick for sample 0, or nullptr
    long long ext_sstride;  // words between consecutive samples of the input block
};

// Launchers (return the first HIP error, hipSuccess otherwise).
hipError_t launch_integrate_plain(const DevNet &n, const TickArgs &a, hipStream_t st);
hipError_t launch_integrate_mfma(const DevNet &n, const TickArgs &a, int two_planes,
                                 int samples_per_wg, hipStream_t st);
hipError_t launch_route(const DevNet &n, int q_now, hipStream_t st);
hipError_t launch_reset_state(const DevNet &n, hipStream_t st);
bool mfma_shape_supported(int A, int N, int two_planes);

}  // namespace ranc
