// Device utility entry points (util.hip).
#pragma once
#include "common.h"

namespace svr {
const char *last_error();
// Exclusive scan of n int32 counts into out[0..n] (out[n] = total); fails
// with SVR_EINVAL if the total exceeds int32.  Waits on the host for the total.
int exclusive_scan(const int *in, int64_t n, int *out, int64_t *total, hipStream_t s);
}  // namespace svr
