// rkc_integrate_device_noalloc (include/rkc.h): rkc_integrate with device
// arrays whose launch scratch -- the aggregate counters and the work-queue
// head that the integrator kernels update -- is a file-scope device array
// instead of memory owned by the mechanism handle, and which allocates
// nothing.
#include <atomic>
#include <cstring>

#include "rkc.h"
#include "rkc_internal.h"

namespace {

// Scratch of one launch: AGG_N aggregate counters, then the work-queue head
// (an int in the next 8-byte word); the rest is spare.  Every device the
// library runs on holds its own copy until the process ends.
constexpr int SCRATCH_WORDS = 32;
static_assert(rkchost::AGG_N + 1 <= SCRATCH_WORDS, "scratch too small");
static __device__ __align__(256) unsigned long long scratch[SCRATCH_WORDS];

// Device address of `scratch` on each device, resolved on the first call with
// that device current (the host-side name is not a device address).
constexpr int MAX_DEVICES = 64;
std::atomic<unsigned long long *> scratch_ptr[MAX_DEVICES];

int scratch_on(int dev, unsigned long long **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return RKC_ENOTSUP;
    unsigned long long *p = scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        void *a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) {
            (void)hipGetLastError();
            return RKC_EDEVICE;
        }
        p = static_cast<unsigned long long *>(a);
        scratch_ptr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return RKC_OK;
}

}  // namespace

extern "C" int rkc_integrate_device_noalloc(const rkc_mech *mc, size_t n, double *T,
                                            const double *P, double *Y, double dt, double rtol,
                                            double atol, const rkc_opts *opts,
                                            int32_t *cell_status) {
    if (!mc || !opts) return RKC_EINVAL;
    rkc_mech *m = const_cast<rkc_mech *>(mc);
    const rkc_opts o = *opts;
    if (!o.device_ptrs) return RKC_EINVAL;   // host arrays would need staging memory
    int rc = rkchost::check_integrate_args(dt, rtol, atol, o);
    if (rc) return rc;
    if (n == 0) return RKC_OK;
    if (!T || !P || !Y) return RKC_EINVAL;
    if (n > RKC_MAX_CELLS) return RKC_ENOTSUP;
    const int dev = rkchost::mech_device(m);
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return RKC_EDEVICE;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return RKC_EDEVICE;
    unsigned long long *sp = nullptr;
    rc = scratch_on(dev, &sp);
    if (rc == RKC_OK) {
        rkchost::LaunchInfo li;
        rc = rkchost::enqueue_integrate(m, n, T, P, Y, dt, rtol, atol, o, cell_status,
                                        o.cell_counters, sp,
                                        reinterpret_cast<int *>(sp + rkchost::AGG_N),
                                        (hipStream_t)o.stream, &li, false);
    }
    if (prev != dev) (void)hipSetDevice(prev);
    return rc;
}
