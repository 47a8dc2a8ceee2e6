// Device-wide prefix sums.
#pragma once
#include "common.hpp"

namespace pg {

// out[i] = in[0] + ... + in[i-1]; *total (device, may be NULL) = sum of all.
// in and out may alias.  n < 2^31.
pg_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                             hipStream_t s);

}  // namespace pg
