// errors.hip -- names of HIP runtime error codes for the diagnostics of the
// C-ABI (the launchers report the raw code of a failed launch).
#include <hip/hip_runtime.h>

#include "glass_internal.hpp"

namespace glass {

const char* hip_error_name(int code) { return hipGetErrorName(static_cast<hipError_t>(code)); }

}  // namespace glass
