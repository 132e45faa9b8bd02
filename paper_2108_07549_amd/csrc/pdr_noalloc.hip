// pdr_set_state_noalloc: pdr_set_state without any device allocation.
//
// The host rows of the state are staged through `scratch`, a file-scope
// device array of kScratchDoubles doubles (32 MiB) that every GPU the library
// runs on holds until the process ends, in chunks of whole arc rows. Its
// device address is resolved once per device (at pdr_init, else at the first
// call on that device) and kept; host code passes that address, never the
// array's name, to copies and kernels. All calls on one GPU share the array:
// calls that overlap in time on one GPU race. Nothing in it must start at
// zero: each chunk is copied in full before the kernel that reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pdr.h"
#include "pdr_context.h"

namespace {
constexpr int64_t kScratchDoubles = int64_t(1) << 22;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace pdr_host {
hipError_t noalloc_scratch(int device, double **out, int64_t *doubles)
{
    *out = nullptr;
    if (doubles) *doubles = kScratchDoubles;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace pdr_host

extern "C" {

static pdr_status set_state_noalloc_body(pdr_ctx *c, const double *f, const double *beta,
                                         const double *v, int64_t t, double z_prev)
{
    if (!c) return PDR_ERR_INVALID;
    if (c->poisoned) return PDR_ERR_DEVICE;
    hipError_t e = hipSetDevice(c->device);
    double *buf = nullptr;
    int64_t cap = 0;
    if (e == hipSuccess) e = pdr_host::noalloc_scratch(c->device, &buf, &cap);
    if (e != hipSuccess) {
        c->poisoned = true;
        c->err = std::string("pdr_set_state_noalloc: ") + hipGetErrorString(e);
        return PDR_ERR_DEVICE;
    }
    if (c->m > 0 && c->K > cap) {
        c->err = "pdr_set_state_noalloc: one arc row of K doubles exceeds its 4,194,304-double "
                 "staging array";
        return PDR_ERR_INVALID;
    }
    pdr_status st = pdr_host::check_state_args(c, f, beta, v, t, z_prev);
    if (st != PDR_OK) return st;
    return pdr_host::set_state_impl(c, f, beta, v, t, z_prev, buf, cap);
}

pdr_status pdr_set_state_noalloc(pdr_ctx *c, const double *f, const double *beta,
                                 const double *v, int64_t t, double z_prev)
{
    return pdr_host::abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr, [&] {
        return set_state_noalloc_body(c, f, beta, v, t, z_prev);
    });
}

}  // extern "C"
