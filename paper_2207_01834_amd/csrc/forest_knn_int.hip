// Forest k-NN kernels instantiated for int32_t coordinates (a translation unit
// per coordinate type keeps the build parallel).
#include "forest_knn.hpp"

namespace pg {

pg_status forest_knn_int(int tk, const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d,
                         int k, int64_t id_end, int32_t* redo, uint32_t* nredo, int64_t* out_id,
                         void* out_dist, hipStream_t s) {
    return forest_detail::forest_knn_any<int32_t>(tk, f, q, o, qk, m, d, k, id_end, redo, nredo, out_id, out_dist, s);
}

}  // namespace pg
