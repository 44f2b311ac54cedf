// kern_mfma_cb.hip -- the MFMA path's kernels (kern_mfma_unit.h) with the
// B tiles built in registers from the compact crossbar (column words,
// per-type plane bytes, axon types) instead of read as int8 weight planes:
// used when one workgroup covers all samples of a core, so that the core's
// B source is read once per tick (a sweep of 64-sample networks: the planes
// were a third of the tick's bytes). Kept in a translation unit of its own,
// apart from the plane form (kern_mfma.hip).
#include "kern_mfma_unit.h"

namespace ranc {

hipError_t launch_integrate_mfma_cb(const DevNet &n, const TickArgs &a, int two_planes, int samples_per_wg,
                                    hipStream_t st)
{
    return launch_mfma_shape<true>(n, a, two_planes, samples_per_wg, st);
}

hipError_t launch_integrate_mfma_group_cb(const MfmaGroupArgs &g, int total, int k, int code, int ext,
                                          hipStream_t st)
{
    return launch_group_code<true>(g, total, k, code, ext, st);
}

}  // namespace ranc
