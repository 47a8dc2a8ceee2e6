// Device-wide prefix sums.
#pragma once
#include "common.hpp"

namespace pg {

// out[i] = in[0] + ... + in[i-1]; *total (device, may be NULL) = sum of all.
// in and out may alias.  n < 2^31.
pg_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                             hipStream_t s);
// The same over int32 inputs with int64 sums (in and out do not alias).
pg_status exclusive_scan_i32_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                                 hipStream_t s);
// Partial sums a scan of n entries keeps (workspace entries of the _ws form).
int64_t scan_partials(int64_t n);
// exclusive_scan_u32 with caller-provided workspace sums[scan_partials(n)].
pg_status exclusive_scan_u32_ws(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                                uint32_t* sums, hipStream_t s);
// p[0..n) = v with a kernel (no memset node, so it may be captured).
pg_status fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// The same over uint64 (in and out may alias).
pg_status exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                             hipStream_t s);
// exclusive_scan_u64 with caller-provided workspace sums[scan_partials(n)].
pg_status exclusive_scan_u64_ws(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total,
                                uint64_t* sums, hipStream_t s);

// Scans whose count is read on the device when they run: n = mul * *cnt +
// add <= n_max (grids and the workspace sums[scan_partials(n_max)] are
// sized for n_max).  The total goes to *total (may be NULL) and, with
// at_end, to out[n].  in and out may alias.
pg_status exclusive_scan_u32_dev(const uint32_t* in, uint32_t* out, const uint32_t* cnt, uint32_t mul,
                                 uint32_t add, int64_t n_max, uint32_t* total, bool at_end,
                                 uint32_t* sums, hipStream_t s);
pg_status exclusive_scan_u64_dev(const uint64_t* in, uint64_t* out, const uint32_t* cnt, uint32_t mul,
                                 uint32_t add, int64_t n_max, uint64_t* total, bool at_end,
                                 uint64_t* sums, hipStream_t s);

}  // namespace pg
