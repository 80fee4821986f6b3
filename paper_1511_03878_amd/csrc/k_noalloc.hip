// Static device scratch of the allocation-free charge-density entry point
// (pic_rho_get_noalloc), for callers that cannot allocate device memory.
//
// `scratch` is one array per GPU, created when the code object is loaded on
// that GPU and held until the process ends.  In host code its name is only a
// host-side stand-in: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// handed to kernels and copies.  Every call on one GPU shares its array (the
// last call's contents stay), so concurrent calls on one GPU race.
#include <mutex>

#include "runtime.h"

namespace pic {

namespace {

static __device__ __align__(256) double scratch[PIC_NOALLOC_MAX_NODES];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

}  // namespace

double *noalloc_scratch()
{
    int dev = 0;
    hipcheck(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) throw Error(PIC_ENOTSUP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw Error(PIC_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_ptr[dev] = (double *)ptr;
    }
    return g_ptr[dev];
}

}  // namespace pic
