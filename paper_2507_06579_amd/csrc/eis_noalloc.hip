// eis_noalloc.hip -- the device scratch of eis_classify_async_noalloc.
//
// The no-allocation entry point runs the same pass as eis_classify_async,
// but every buffer its kernels need beyond the caller's inputs and outputs
// (segment table, prime offsets, work lists, counters, queue heads, the pass
// bitmaps and the giant-step lists, tables, window records and tasks) is
// carved out of one file-scope device array.  The loaded code object holds
// one copy of it per device until the process ends; nothing is allocated
// per call.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress
// (noalloc_scratch_init, called by eis_create with the device current) and
// only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "eis_internal.h"

namespace eis {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return g_status[device];
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_status[device] = e;
    g_addr[device] = (e == hipSuccess) ? ptr : nullptr;
    g_done[device] = true;
    return e;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_done[device] ? g_addr[device] : nullptr;
}

// Store one segment-table entry from a kernel argument (no host staging).
__global__ void k_store_seg(SegInfo s, SegInfo *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = s;
}

hipError_t launch_store_seg(const SegInfo &s, SegInfo *dst, hipStream_t stream)
{
    (void)hipGetLastError();  // the check below reports this launch only
    hipLaunchKernelGGL(k_store_seg, dim3(1), dim3(64), 0, stream, s, dst);
    return hipGetLastError();
}

}  // namespace eis
