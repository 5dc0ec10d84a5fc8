// Shared host-side helpers of libhawkes.so: error reporting and HIP checks.
#pragma once

#include <hip/hip_runtime.h>

#include "hawkes.h"

namespace hawkes {

// Records a printf-style message as the calling thread's last error.
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

// Records the HIP failure `e` of `what` and returns HAWKES_EHIP.
int hip_failure(hipError_t e, const char *what);

// Returns HAWKES_EHIP if the last kernel launch failed, else HAWKES_OK.
int check_launch(const char *what);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace hawkes
