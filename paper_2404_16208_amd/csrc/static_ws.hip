// static_ws.hip -- a workspace that the library itself holds, one per device,
// for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops and harnesses that forbid hipMalloc).
//
// The array below lives in the library's code object: every device the
// library runs on holds its own copy, from the moment the code object is
// loaded on that device until the process ends. In host code its name is only
// a host-side stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to the loader and, through the handle's region pointers, to every
// kernel.
//
// One handle at a time may hold a device's array: a claim is taken when a
// network is loaded into it and released by ranc_free. The array keeps what
// the last handle left in it; loading writes every parameter and resets every
// piece of state a kernel reads before writing, as for a caller's workspace
// of unknown contents.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ranc.h"
#include "ranc_internal.h"

namespace ranc {

static __device__ __align__(256) uint8_t scratch[RANC_STATIC_WORKSPACE_BYTES];

namespace {
std::mutex g_mu;
void *g_addr[STATIC_WS_MAX_DEVICES];   // device address of `scratch`, per device (null: not looked up yet)
bool g_held[STATIC_WS_MAX_DEVICES];    // a live handle uses the device's array
}  // namespace

hipError_t static_ws_claim(int dev, void **addr, bool *held)
{
    *addr = nullptr;
    *held = false;
    if (dev < 0 || dev >= STATIC_WS_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != dev)
            return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p || (uintptr_t)p % 256)
            return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    if (g_held[dev]) {
        *held = true;
        return hipSuccess;
    }
    g_held[dev] = true;
    *addr = g_addr[dev];
    return hipSuccess;
}

void static_ws_release(int dev)
{
    if (dev < 0 || dev >= STATIC_WS_MAX_DEVICES)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_held[dev] = false;
}

}  // namespace ranc
