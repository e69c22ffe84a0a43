// dmrt_noalloc.hip -- dmrt_residual_noalloc: the residual / non-finite
// watchdog of dmrt_residual for callers that cannot allocate device memory.
//
// dmrt_residual allocates its reference fields and its FP64 partial sums on
// first use.  Here the caller brings the reference fields, and the partial
// sums live in `scratch`, a fixed-size file-scope device array: every GPU the
// library runs on holds one copy until the process ends, at its own address,
// which is looked up once per device with hipGetSymbolAddress.  The kernels
// are the ones dmrt_residual launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "dmrt.h"
#include "dmrt_device.hpp"
#include "dmrt_internal.hpp"

using namespace dmrt;

// Partial sums of at most kMaxParts workgroups, 5 doubles each, and the 5
// final sums after them: 41,000 bytes per device.
constexpr int kMaxParts = 1024;
constexpr int kScratchDoubles = 5 * (kMaxParts + 1);

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Device address of `scratch` per device (the host-side name is not a
// device address and is never passed to a kernel or a copy).
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

// Called with device `dev` current.
int scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_last_error("dmrt_residual_noalloc: device index beyond the library's table");
        return DMRT_EINVAL;
    }
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? static_cast<double*>(p) : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess)
        return record_hip(g_scratch_err[dev], "hipGetSymbolAddress(scratch)");
    *out = g_scratch_ptr[dev];
    return DMRT_OK;
}

template <typename real>
void launch_residual(const dmrt_cavity* h, int parts, double* ref, double* part)
{
    const double gy0 = -h->d.gbeta * h->p.theta_ref;
    const real* fs = static_cast<const real*>(h->fbuf) + (size_t)h->cur * 9 * h->plane;
    const real* gs = static_cast<const real*>(h->gbuf) + (size_t)h->cur * 5 * h->plane;
    // FP32 storage: coefficients rounded as the step kernel rounds them
    const bool f32 = sizeof(real) == sizeof(float);
    const double gb = f32 ? (double)(float)h->d.gbeta : h->d.gbeta;
    const double g0 = f32 ? (double)(float)gy0 : gy0;
    const double gx = f32 ? (double)(float)h->p.force_x : h->p.force_x;
    hipLaunchKernelGGL((residual_kernel<real>), dim3(parts), dim3(256), 0, h->stream, fs, gs, h->n,
                       h->pitch, h->plane, gb, g0, gx, ref, part);
}

}  // namespace

extern "C" int dmrt_residual_noalloc(dmrt_cavity* h, double* ref, double* res_theta, double* res_u)
{
    if (!h || !ref || ((uintptr_t)ref % alignof(double))) return DMRT_EINVAL;
    int cur = -1;
    DMRT_HIPCHK(hipGetDevice(&cur));
    if (cur != h->dev) DMRT_HIPCHK(hipSetDevice(h->dev));
    struct Restore {
        int dev;
        ~Restore() { (void)hipSetDevice(dev); }
    } restore{cur};
    double* sp = nullptr;
    int rc = scratch_address(h->dev, &sp);
    if (rc) return rc;
    const size_t nn = (size_t)h->n * h->n;
    const int parts = (int)std::min<size_t>(kMaxParts, (nn + 255) / 256);
    if (5 * (parts + 1) > kScratchDoubles) {
        set_last_error("dmrt_residual_noalloc: partial sums exceed the fixed scratch array");
        return DMRT_EINVAL;
    }
    double* fin = sp + 5 * parts;
    if (h->esz == sizeof(double))
        launch_residual<double>(h, parts, ref, sp);
    else
        launch_residual<float>(h, parts, ref, sp);
    DMRT_HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(64), 0, h->stream, sp, parts, fin);
    DMRT_HIPCHK(hipGetLastError());
    double r[5];
    DMRT_HIPCHK(hipMemcpyAsync(r, fin, sizeof r, hipMemcpyDeviceToHost, h->stream));
    DMRT_HIPCHK(hipStreamSynchronize(h->stream));
    if (res_theta) *res_theta = r[1] > 0 ? std::sqrt(r[0] / r[1]) : std::sqrt(r[0]);
    if (res_u) *res_u = r[3] > 0 ? std::sqrt(r[2] / r[3]) : std::sqrt(r[2]);
    return r[4] > 0 ? DMRT_ENONFINITE : DMRT_OK;
}
