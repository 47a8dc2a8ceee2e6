// The forest of a batch-dynamic kd-tree (Section 5: a buffer tree plus
// static trees of doubling capacity) as the k-NN kernels see it: each tree
// with its point ids in leaf order and its liveness bits.
#pragma once

#include "knn.hpp"

namespace pg {

constexpr int kMaxTrees = 31;        // static trees 0..30
constexpr int kSlots = kMaxTrees + 1;  // + the buffer tree

struct ForestSlot {
    TreeView tv;
    const int64_t* ids;
    uint32_t* alive;
    int idrec;  // the records' row words hold the ids' low 32 bits
};

struct Forest {
    ForestSlot s[kSlots];
    int count;
};

// k-NN of m queries over every tree of f, one k-list per query (Section 5's
// data-parallel k-NN on the BDL-tree): ids into out_id [m][k] (-1 where fewer
// than k live points exist), squared distances into out_dist.  tk: the tree
// kind shared by every tree; o: the queries' order (or null) and qk where
// their descents in the first tree ended (or none); id_end: every
// id in the forest is below it; redo [m] and nredo [1]: device scratch for
// the queries handed from the packed-key search to the exact one.  A
// translation unit per coordinate type.
pg_status forest_knn_int(int tk, const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d,
                         int k, int64_t id_end, int32_t* redo, uint32_t* nredo, int64_t* out_id,
                         void* out_dist, hipStream_t s);
pg_status forest_knn_float(int tk, const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d,
                           int k, int64_t id_end, int32_t* redo, uint32_t* nredo, int64_t* out_id,
                           void* out_dist, hipStream_t s);

}  // namespace pg
