// Host-side helpers shared by the translation units of the C ABI: the
// thread-local error message read by cdi_last_error and the HIP status check.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cdi.h"

namespace cdi_host {

// Record a formatted message for cdi_last_error and return s.
cdi_status fail(cdi_status s, const char* fmt, ...);

}  // namespace cdi_host

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      return cdi_host::fail(CDI_ERR_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_)); \
  } while (0)
