// Static kd-tree construction (host entry points of build.hip).
#pragma once
#include "common.hpp"

namespace pg {

// Largest subtree (points) finished in LDS by one workgroup.
int subtree_capacity(int d);

// Caller rows [n][d] -> key planes keys[d][n] and idx[i] = i; reads back the
// range flag, the per-dimension OR of (key ^ key of row 0) and row 0's keys.
// Synchronises the stream.
pg_status ingest_points(const void* points, int64_t n, int d, bool fl, uint32_t* keys,
                        int32_t* idx, uint32_t* vary_host, uint32_t* keybase_host,
                        hipStream_t s);

// Builds the levels of T (T->n, d, L, dtype and the output arrays set) from key
// planes kA[d][n] and input rows iA[n]; kB/iB are scratch of the same size.
// kA/iA may be T->pts/T->pidx.
pg_status build_from_keys(uint32_t* kA, int32_t* iA, uint32_t* kB, int32_t* iB, int64_t n,
                          int d, int leaf, bool fl, const uint32_t* vary,
                          const uint32_t* keybase, hipStream_t s, pg_tree* T);

// Boxes of T's internal nodes from its leaf boxes (bottom-up).
pg_status internal_boxes(pg_tree* T, hipStream_t s);
// Every box of a tree with explicit leaf offsets (T->loff), from its points.
pg_status offset_boxes(pg_tree* T, hipStream_t s);

// Allocates T's arrays and builds it from device rows [n][d].
pg_status build_tree(const void* points, int64_t n, int d, int leaf, int dtype, hipStream_t s,
                     pg_tree* T);

// Allocates T's arrays and builds the spatial-median tree as an
// explicit-node tree (T->xn and friends) from device rows [n][d]; rule bit 0:
// split dimension = the space's widest side instead of depth mod d; bit 1:
// nodes cut the bounding box of their points instead of their cell.
pg_status build_tree_spatial(const void* points, int64_t n, int d, int leaf, int dtype, int rule,
                             hipStream_t s, pg_tree* T);

// Node boxes and empty flags of an explicit-node tree from its points and
// leaf offsets (after points were added in place).
pg_status xtree_boxes(pg_tree* T, hipStream_t s);

}  // namespace pg
