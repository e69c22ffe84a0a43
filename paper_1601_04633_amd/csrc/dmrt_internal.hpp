// dmrt_internal.hpp -- host helpers shared by the translation units of libdmrt.
#pragma once

#include <hip/hip_runtime.h>

#include "dmrt.h"
#include "dmrt_device.hpp"

namespace dmrt {

// Records the HIP error text for dmrt_last_error() and maps it to a code.
int record_hip(hipError_t e, const char* what);

// Parameter map of dmrt_derive (Eq. 9, Eqs. 11-13, 32, 38-43).
int derive(const dmrt_params* p, dmrt_derived* d);

// Row pitch in elements: n rounded up to a multiple of 64.
int pitch_of(int n);

inline size_t elem_size(int precision) { return precision == DMRT_FP64 ? sizeof(double) : sizeof(float); }

// Kernel coefficients in the compute precision.
template <typename real>
Coef<real> make_coef(const dmrt_params& p, const dmrt_derived& d)
{
    Coef<real> c;
    c.s_nu = real(d.s_nu); c.s_q = real(d.s_q);
    c.sk = real(d.sigma_k); c.se = real(d.sigma_e); c.sn = real(d.sigma_nu);
    c.a = real(d.a);
    c.cabb = real((4.0 + d.a) / 10.0);
    c.gbeta = real(d.gbeta);
    c.gy0 = real(-d.gbeta * p.theta_ref);
    c.gx = real(p.force_x);
    c.cold = real((4.0 + d.a) / 10.0 * p.theta_cold);
    return c;
}

// Thread-local text of the last HIP error.
void set_last_error(const char* msg);

}  // namespace dmrt

#define DMRT_HIPCHK(expr)                                          \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return ::dmrt::record_hip(e_, #expr); \
    } while (0)
