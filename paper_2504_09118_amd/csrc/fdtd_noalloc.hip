// fdtd_step_noalloc: fdtd_step for callers that cannot allocate device memory.
//
// The temporal sweeps hand out tiles from scheduling counters (kSchedWords
// 32-bit words that every launch leaves at zero). fdtd_step keeps them in the
// solver's arena; this entry point takes them from a file-scope device array
// instead, so a call touches no memory beyond the solver's state and makes no
// allocation of any kind. Each GPU holds its own copy of the array for the life
// of the process; every call on that GPU shares it, so calls that overlap on
// one GPU race (they must be ordered, e.g. on one stream).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fdtd.h"
#include "fdtd_internal.h"
#include "solver.h"

namespace {

constexpr int kScratchWords = 64;  // 256 bytes; the sweeps use kSchedWords of them
static_assert(fdtd::kSchedWords <= kScratchWords, "scheduling counters exceed the scratch array");

static __device__ __align__(256) unsigned scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned *g_ptr[kMaxDevices];  // device address of scratch, per device (null: not set up)

// Clears the counters at the start of a call (a kernel, not hipMemsetAsync: the call may be
// captured into a graph).
__global__ void k_clear(unsigned *p, int n)
{
    const int i = (int)threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

// The device address of this device's scratch array, looked up once per device with the
// device current.
int scratch_of(int dev, unsigned **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        fdtd::set_last_error("fdtd_step_noalloc: device index out of range");
        return FDTD_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fdtd::set_last_error("fdtd_step_noalloc: hipGetSymbolAddress(scratch) failed");
            return FDTD_E_DEVICE;
        }
        g_ptr[dev] = (unsigned *)p;
    }
    *out = g_ptr[dev];
    return FDTD_OK;
}

}  // namespace

extern "C" int fdtd_step_noalloc(fdtd_t h, long long n)
{
    int st = fdtd::solver_check(h);
    if (st)
        return st;
    // argument checks before anything is enqueued (step_with_queue repeats them)
    if (n < 0) {
        fdtd::set_last_error("fdtd_step_noalloc: negative step count");
        return FDTD_E_ARG;
    }
    if (!h->fields_set) {
        fdtd::set_last_error("fdtd_step_noalloc: fields were never set");
        return FDTD_E_STATE;
    }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess)
        return fdtd::solver_device_fail(h, e, "hipSetDevice");
    unsigned *q = nullptr;
    if ((st = scratch_of(h->device, &q)))
        return st;
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, h->stream, q, fdtd::kSchedWords);
    if ((e = hipGetLastError()) != hipSuccess)
        return fdtd::solver_device_fail(h, e, "kernel launch");
    return fdtd::step_with_queue(h, n, q);
}
