// Device scratch of the allocation-free entry point (ltl_learn_noalloc): a fixed
// array in the library's code object, one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel: on the host it is a
// stand-in, not a device address.  The device address of each GPU's copy is
// looked up once per device (with that device current) and every kernel gets it
// as an ordinary pointer argument.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ltl.h"

namespace ltl {

static __device__ __align__(256) unsigned char scratch[LTL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};
std::mutex g_dev_mu[MAX_DEVICES];
}  // namespace

// Device address of `device`'s copy of the scratch array (device must be current).
// Returns nullptr and sets *err on failure.
void *noalloc_scratch(int device, hipError_t *err) {
    *err = hipSuccess;
    if (device < 0 || device >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = (e != hipSuccess) ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

// Calls on one device share its array: they take turns (the entry point is
// synchronous, so a call's work has ended when it releases the lock).
std::mutex &noalloc_lock(int device) { return g_dev_mu[device]; }

}  // namespace ltl
