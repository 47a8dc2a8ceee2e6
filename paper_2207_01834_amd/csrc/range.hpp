// Orthogonal range search over a static kd-tree (host entry points).
#pragma once
#include "common.hpp"

namespace pg {

// Counting pass: counts[i] = points in box i; the exclusive prefix sum goes
// to offsets (m+1 entries) when given, the total to the host when asked.
pg_status range_count(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                      int64_t* offsets, int64_t* total_host, hipStream_t s);
// Reporting pass: rows of box i's points to out_idx[offsets[i] ...], leaf
// order; slots at or beyond `capacity` are not written (PG_ERR_INVALID).
pg_status range_report(const pg_tree* t, const void* boxes, int64_t m, const int64_t* offsets,
                       int32_t* out_idx, int64_t capacity, hipStream_t s);

// Both passes with one box ordering: counts (caller's, or a temporary when
// NULL), offsets (m+1), then rows when the total fits `capacity`; otherwise
// PG_ERR_INVALID with counts, offsets and *total_host written.
pg_status range_search(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                       int64_t* offsets, int32_t* out_idx, int64_t capacity, int64_t* total_host,
                       hipStream_t s);

}  // namespace pg
