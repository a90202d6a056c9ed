// Fixed device scratch for the allocation-free entry point
// (adscl_constraints_noalloc): a file-scope device array, one copy per GPU, whose
// address on each device is looked up once, with that device current, when the
// first context is created on it.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); it passes the
// looked-up device address.
#include <mutex>

#include "internal.h"

namespace adscl {
namespace {

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = (double*)p;
    return hipSuccess;
}

double* static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace adscl
