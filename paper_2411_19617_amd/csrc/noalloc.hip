// Fixed device scratch for the entry point that allocates nothing
// (mala_integrate_noalloc): the per-block FP64 partial rows of the DOS column
// sums and the FP64 occupation weights of the final Fermi pass.
//
// The array lives in the library's code object, so every device the library
// runs on holds its own copy for the life of the process.  In host code the
// name `scratch` is only a host-side stand-in: the device address of each
// copy comes from hipGetSymbolAddress, looked up once per device with that
// device current (scratch_device_ptr, first called by mala_create) and used from then on
// for every kernel argument.
#include <mutex>

#include "mala_internal.h"

namespace mala {

static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
hipError_t g_status[kMaxDevices];
double* g_ptr[kMaxDevices];
}  // namespace

// Device address of `device`'s copy of the scratch array, looked up on the
// first call for that device (the caller has made `device` current); later
// calls return the first result.  mala_create calls it at set-up.
hipError_t scratch_device_ptr(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(g_once[device], [device] {
        void* p = nullptr;
        g_status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[device] = g_status[device] == hipSuccess ? static_cast<double*>(p) : nullptr;
    });
    if (g_status[device] != hipSuccess) return g_status[device];
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace mala
