// Device scratch for the entry points that allocate nothing.
//
// A file-scope device array holds the staging a rescale needs between its
// passes (the dropped limb in coefficient form, then the column pass's
// intermediate), so a caller that cannot allocate device memory (code under
// graph capture, a serving loop that forbids allocation) can still rescale.
// Each device the library runs on holds its own copy of the array until the
// process ends.  In host code the array's name is only a stand-in: its device
// address is looked up once per device at context creation and kept here;
// every launch takes that address.
#include <mutex>

#include "ckks.hpp"

namespace hk {

namespace {
constexpr size_t kScratchWords = kNoAllocScratchBytes / sizeof(u64);
static __device__ __align__(256) u64 scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
u64 *g_ptr[kMaxDevices] = {};
}  // namespace

u64 *noalloc_scratch_setup()
{
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw HeError(-6, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HeError(-6, "no device address for the scratch array");
        g_ptr[dev] = static_cast<u64 *>(p);
    }
    return g_ptr[dev];
}

}  // namespace hk
