// Fixed device scratch of the entry points that allocate nothing
// (mlb_dilate_noalloc_dev): one file-scope array per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel (in
// host code it is only a stand-in for the symbol): scratch_address() looks
// up the array's device address once per device, with that device current,
// and every caller uses that address.
#include <mutex>

#include "kernels.h"

namespace mlb {

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[device] = static_cast<double*>(p);
    }
    *out = scratch_addr[device];
    return hipSuccess;
}

}  // namespace mlb
