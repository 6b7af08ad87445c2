// Library-resident scratch of the allocation-free forward entry point
// (cgh_progressive_hologram_noalloc): a file-scope device array that every GPU
// the library runs on holds from the loading of this code object until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it only names a shadow variable): the device address of each GPU's copy
// is looked up once per device, with that device current, and cached here.
#include <mutex>

#include "../../include/cgh.h"
#include "common.h"

namespace cgh {
namespace {

static __device__ __align__(256) unsigned char scratch[CGH_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];

}  // namespace

hipError_t noalloc_scratch(void** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace cgh
