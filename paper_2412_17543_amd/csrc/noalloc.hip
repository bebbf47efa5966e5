// Device scratch of the allocation-free entry point bddc_apply_schur_noalloc:
// a file-scope array in device memory (one copy per GPU, held until the
// process ends) instead of memory the context allocates, for callers that
// cannot allocate.  Host code never passes the array's name to a kernel: it
// resolves the array's device address once per device with
// hipGetSymbolAddress (with that device current) and passes that pointer.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace bddc {

constexpr int64_t NOALLOC_SCRATCH_DOUBLES = int64_t(1) << 20;   // 8 MiB per device

static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
double *g_scratch[MAX_DEVICES] = {};
std::mutex g_scratch_mu;
}  // namespace

int64_t noalloc_scratch_doubles() { return NOALLOC_SCRATCH_DOUBLES; }

// Device address of the current device's scratch array (resolved on the
// first call per device, then kept).
int noalloc_scratch(double **out, std::string &err) {
    *out = nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        err = "no current HIP device (or device index above 63) for the static scratch array";
        return BDDC_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress of the static scratch array failed: ") + hipGetErrorString(e);
            return BDDC_EHIP;
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return 0;
}

}  // namespace bddc
