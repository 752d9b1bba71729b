// nc_noalloc.hip -- the fixed device scratch of nc_render_batch_noalloc.
//
// A file-scope device array holds what a batched render launch writes before
// it runs (the work-queue heads, the launch record, the job table), so that
// the entry point needs no device allocation.  Each GPU the library runs on
// holds its own copy of the array at its own address; host code never uses
// the array's name as an address (in host code it names a host-side stand-in):
// the device address is resolved once per device with hipGetSymbolAddress
// and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nc_internal.hpp"

namespace nc {
namespace {

constexpr size_t kQueueBytes = 128 * sizeof(unsigned long long);
constexpr size_t kRareOffset = kQueueBytes;
constexpr size_t kJobsOffset = (kRareOffset + kRareBytes + 255) & ~(size_t)255;
constexpr size_t kScratchBytes = kJobsOffset + (size_t)kNoallocMaxJobs * sizeof(JobView);
static_assert(kJobsOffset % alignof(JobView) == 0, "aligned job records");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_addr[kMaxDevices] = {};   // the array's address on each device (nullptr: not resolved)

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t noalloc_init_device(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_addr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // on the current device
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = static_cast<unsigned char *>(p);
    return hipSuccess;
}

RenderScratch noalloc_render_scratch(int device)
{
    unsigned char *base = nullptr;
    if (device >= 0 && device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_mu);
        base = g_addr[device];
    }
    if (!base) return RenderScratch{nullptr, nullptr, nullptr, 0};
    return RenderScratch{reinterpret_cast<JobView *>(base + kJobsOffset),
                         reinterpret_cast<unsigned long long *>(base + kRareOffset),
                         reinterpret_cast<unsigned long long *>(base), 1};
}

}  // namespace nc
