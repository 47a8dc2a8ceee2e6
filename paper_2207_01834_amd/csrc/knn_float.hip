// Static-tree k-NN kernels instantiated for float coordinates (a translation
// unit per coordinate type keeps the build parallel).
#include "knn.hpp"
#include "knn_static.hpp"

namespace pg {

pg_status knn_static_float(const pg_tree* t, const void* queries, const int32_t* o, QueryKeys qk, int64_t m, int k,
                 bool all, int32_t* out_idx, void* out_dist, hipStream_t s, bool no_self,
                 const KnnWs* ws) {
    using namespace knn_detail;
    const int tk = tree_kind(t);
    if (no_self) {
        if (tk == kTreeX) return dispatch_d<float, true, kTreeX>(t, nullptr, nullptr, QueryKeys{}, m, k, true, out_idx, out_dist, s, ws);
        if (tk == kTreeLoff) return dispatch_d<float, true, kTreeLoff>(t, nullptr, nullptr, QueryKeys{}, m, k, true, out_idx, out_dist, s, ws);
        return dispatch_d<float, true, kTreeHeap>(t, nullptr, nullptr, QueryKeys{}, m, k, true, out_idx, out_dist, s, ws);
    }
    if (tk == kTreeX) return dispatch_d<float, false, kTreeX>(t, queries, o, qk, m, k, all, out_idx, out_dist, s, ws);
    if (tk == kTreeLoff) return dispatch_d<float, false, kTreeLoff>(t, queries, o, qk, m, k, all, out_idx, out_dist, s, ws);
    return dispatch_d<float, false, kTreeHeap>(t, queries, o, qk, m, k, all, out_idx, out_dist, s, ws);
}

}  // namespace pg
