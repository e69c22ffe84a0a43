// dmrt_internal.hpp -- host helpers shared by the translation units of libdmrt.
#pragma once

#include <hip/hip_runtime.h>

#include "dmrt.h"

namespace dmrt {

// Records the HIP error text for dmrt_last_error() and maps it to a code.
int record_hip(hipError_t e, const char* what);

// Parameter map of dmrt_derive (Eq. 9, Eqs. 11-13, 32, 38-43).
int derive(const dmrt_params* p, dmrt_derived* d);

// Row pitch in elements: n rounded up to a multiple of 64.
int pitch_of(int n);

}  // namespace dmrt
