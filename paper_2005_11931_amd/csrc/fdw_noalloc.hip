// fdw_noalloc.hip - the receiver misfit for callers that cannot allocate device memory (code
// under stream capture, tight loops, harnesses that forbid allocation).  Same kernels as
// fdw_misfit; the reduction's block partials live in a file-scope device array instead of a
// context's workspace, so no context and no workspace are needed.
#include "../../include/fdw.h"
#include "fdw_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

using namespace fdw;

namespace {

// Block partials of the misfit reduction (kRedBlocks of them) and the final sum's slack; every
// GPU the library runs on holds one copy of this array until the process ends.
constexpr int kNoAllocScratchDoubles = 4 * kRedBlocks + 16;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (null: not looked up)
thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

// Device address of this device's copy of `scratch`, looked up once per device with that device
// current.  The array's name is not a device address in host code; only this pointer is used.
int scratch_for_current_device(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FDW_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(FDW_ENOTSUP, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FDW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return FDW_OK;
}

}  // namespace

extern "C" {

int fdw_misfit_noalloc(int32_t dtype, const void* traces, const double* d, int64_t rows, int32_t R, double* J_dev,
                       double* trace_grad, void* hip_stream)
{
    if (dtype != FDW_F32 && dtype != FDW_F64) return fail(FDW_EINVAL, "dtype must be FDW_F32 or FDW_F64");
    if (!traces || !d || !J_dev) return fail(FDW_EINVAL, "traces, d and J_dev are required");
    if (rows < 0 || R < 0) return fail(FDW_EINVAL, "rows and R must be >= 0");
    if (R > kMaxReceivers || rows > (int64_t)INT32_MAX)
        return fail(FDW_EINVAL, "rows must be <= 2^31 - 1 and R <= 16384 (the library's trace limits)");
    double* red = nullptr;
    int rc = scratch_for_current_device(&red);
    if (rc) return rc;
    const int64_t n = rows * (int64_t)R;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = (dtype == FDW_F32) ? launch_misfit<float>(traces, d, n, J_dev, trace_grad, red, s)
                                      : launch_misfit<double>(traces, d, n, J_dev, trace_grad, red, s);
    if (e != hipSuccess) return fail(FDW_EHIP, std::string("misfit launch: ") + hipGetErrorString(e));
    return FDW_OK;
}

const char* fdw_noalloc_last_error(void) { return g_err.c_str(); }

}  // extern "C"
