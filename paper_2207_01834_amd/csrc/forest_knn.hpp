// Forest k-NN kernels (the k-NN of the BDL-tree and of its baselines), as
// templates instantiated by forest_knn_int.hip and forest_knn_float.hip.
//
// One lane per query walks the trees largest first with one k-list, so the
// k-th distance found in the large trees prunes the small ones: a smaller
// tree's descent already notes which of its path's split planes are out of
// reach, and the walk skips those ancestors on its way back.  While
// every id is below 2^31 the list holds packed (distance, id) keys, and the
// trees whose records carry the ids in their row words need no id load.
// Tombstoned points are skipped by their liveness bit, read only for points
// within the current k-th distance.
#pragma once

#include "forest.hpp"
#include "knn.hpp"
#include "scan.hpp"
#include "xsearch.hpp"

namespace pg {
namespace forest_detail {

constexpr int kNT = 256;

// Ids of a forest's points: from the record's row word (idrec: exact while
// every id is below 2^31) or from the tree's id array.
struct BdlIds {
    static constexpr bool kLazy = true;  // the liveness bits are a load of their own
    const int64_t* ids;
    const uint32_t* alive;
    int idrec;
    __device__ inline int64_t id(int64_t i, uint32_t idw) const { return idrec ? (int64_t)idw : ids[i]; }
    __device__ inline bool live(int64_t i) const { return (alive[i >> 5] >> (i & 31)) & 1u; }
};

// Forest k-NN: every tree, largest first, one k-list per lane.  PK: the list
// holds packed (distance, id) keys (ids below 2^idbits <= 2^31); a query
// whose k-th key ends clamped (int32 trees, see PackedList) is appended to
// `redo` instead of written.  Otherwise exact (distance, id) pairs.
template <typename T, int MD, int KT, bool EX, int TK, bool PK>
__global__ void __launch_bounds__(kNT)
bdl_knn_kernel(Forest f, const uint32_t* __restrict__ queries, const int32_t* __restrict__ order,
               QueryKeys qk, int64_t m, int d, int k, int idbits, int32_t* __restrict__ redo,
               uint32_t* __restrict__ nredo, int64_t* __restrict__ out_id,
               typename Metric<T>::D* __restrict__ out_dist) {
    using M = Metric<T>;
    const int64_t i0 = xcd_block() * kNT + threadIdx.x;
    if (i0 >= m) return;
    const int64_t qi = order ? (int64_t)order[i0] : i0;  // leaf order of the largest tree
    T q[MD];
#pragma unroll
    for (int c = 0; c < MD; c++) q[c] = M::load(c < d ? queries[qi * d + c] : 0u);
    if constexpr (PK) {
        PackedList<T, KT, EX> kl;
        kl.init(idbits);
        if (f.count > 0)
            tree_search<T, MD, decltype(kl), BdlIds, TK>(
                f.s[0].tv, BdlIds{f.s[0].ids, f.s[0].alive, f.s[0].idrec}, q, d, kl, k,
                search_start<TK>(f.s[0].tv, false, 0),
                descend_from<T, MD, TK>(f.s[0].tv, q, d, search_from<TK>(f.s[0].tv, qk, qi)));
        for (int t = 1; t < f.count; t++)
            tree_search_next<T, MD, decltype(kl), BdlIds, TK>(
                f.s[t].tv, BdlIds{f.s[t].ids, f.s[t].alive, f.s[t].idrec}, q, d, kl, k);
        if (kl.needs_redo()) {
            redo[atomicAdd(nredo, 1u)] = (int32_t)qi;
            return;
        }
#pragma unroll
        for (int s = 0; s < KT; s++) {
            if (EX || s < k) {
                out_id[qi * k + s] = (int64_t)kl.id_of(kl.key[s]);  // float: an empty slot reads -1
                out_dist[qi * k + s] = kl.dist_of(kl.key[s]);
            }
        }
    } else {
        KList<typename M::D, int64_t, KT, EX> kl;
        kl.init(M::inf(), INT64_MAX);
        if (f.count > 0)
            tree_search<T, MD, decltype(kl), BdlIds, TK>(
                f.s[0].tv, BdlIds{f.s[0].ids, f.s[0].alive, 0}, q, d, kl, k,
                search_start<TK>(f.s[0].tv, false, 0),
                descend_from<T, MD, TK>(f.s[0].tv, q, d, search_from<TK>(f.s[0].tv, qk, qi)));
        for (int t = 1; t < f.count; t++)
            tree_search_next<T, MD, decltype(kl), BdlIds, TK>(f.s[t].tv, BdlIds{f.s[t].ids, f.s[t].alive, 0},
                                                             q, d, kl, k);
#pragma unroll
        for (int s = 0; s < KT; s++) {
            if (EX || s < k) {
                out_id[qi * k + s] = kl.id[s] == INT64_MAX ? -1 : kl.id[s];
                out_dist[qi * k + s] = kl.d[s];
            }
        }
    }
}

// The queries the packed search handed over, with exact pairs.
template <typename T, int MD, int KT, bool EX, int TK>
__global__ void __launch_bounds__(kNT)
bdl_knn_redo_kernel(Forest f, const uint32_t* __restrict__ queries, int d, int k,
                    const int32_t* __restrict__ redo, const uint32_t* __restrict__ nredo,
                    int64_t* __restrict__ out_id, typename Metric<T>::D* __restrict__ out_dist) {
    using M = Metric<T>;
    const int64_t cnt = *nredo;
    for (int64_t r = (int64_t)blockIdx.x * kNT + threadIdx.x; r < cnt; r += (int64_t)gridDim.x * kNT) {
        const int64_t qi = redo[r];
        T q[MD];
#pragma unroll
        for (int c = 0; c < MD; c++) q[c] = M::load(c < d ? queries[qi * d + c] : 0u);
        KList<typename M::D, int64_t, KT, EX> kl;
        kl.init(M::inf(), INT64_MAX);
        for (int t = 0; t < f.count; t++)
            tree_search<T, MD, decltype(kl), BdlIds, TK>(f.s[t].tv, BdlIds{f.s[t].ids, f.s[t].alive, 0}, q,
                                                         d, kl, k, search_start<TK>(f.s[t].tv, false, 0));
#pragma unroll
        for (int s = 0; s < KT; s++) {
            if (EX || s < k) {
                out_id[qi * k + s] = kl.id[s] == INT64_MAX ? -1 : kl.id[s];
                out_dist[qi * k + s] = kl.d[s];
            }
        }
    }
}

// Ids below 2^31 pack beside the distance (PackedList); larger ones take
// exact pairs.  id_end: every id of the forest is below it; redo [m] and
// nredo [1]: the list of queries the packed search hands to the exact one.
template <typename T, int MD, int KT, bool EX, int TK>
pg_status launch_bdl_knn(const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d, int k,
                         int64_t id_end, int32_t* redo, uint32_t* nredo, int64_t* oi, void* od,
                         hipStream_t s) {
    using DT = typename Metric<T>::D;
    const unsigned grid = grid_for_xcd(cdiv(m, kNT));
    if (id_end > ((int64_t)1 << 31)) {
        hipLaunchKernelGGL((bdl_knn_kernel<T, MD, KT, EX, TK, false>), dim3(grid), dim3(kNT), 0, s, f,
                           (const uint32_t*)q, o, qk, m, d, k, 0, nullptr, nullptr, oi, (DT*)od);
        PG_LAUNCH_CHECK();
        return PG_OK;
    }
    PG_TRY(fill_u32(nredo, 1, 0u, s));
    hipLaunchKernelGGL((bdl_knn_kernel<T, MD, KT, EX, TK, true>), dim3(grid), dim3(kNT), 0, s, f,
                       (const uint32_t*)q, o, qk, m, d, k, id_bits(id_end), redo, nredo, oi, (DT*)od);
    PG_LAUNCH_CHECK();
    if (!PackedList<T, KT, EX>::kFloat) {
        hipLaunchKernelGGL((bdl_knn_redo_kernel<T, MD, KT, EX, TK>), dim3(512), dim3(kNT), 0, s, f,
                           (const uint32_t*)q, d, k, redo, nredo, oi, (DT*)od);
        PG_LAUNCH_CHECK();
    }
    return PG_OK;
}

template <typename T, int MD, int TK>
pg_status bdl_knn_k(const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d, int k,
                    int64_t mx, int32_t* rd, uint32_t* nr, int64_t* oi, void* od, hipStream_t s) {
    if (k == 5) return launch_bdl_knn<T, MD, 5, true, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k == 10) return launch_bdl_knn<T, MD, 10, true, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k == 16) return launch_bdl_knn<T, MD, 16, true, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k <= 2) return launch_bdl_knn<T, MD, 2, false, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k <= 4) return launch_bdl_knn<T, MD, 4, false, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k <= 8) return launch_bdl_knn<T, MD, 8, false, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k <= 16) return launch_bdl_knn<T, MD, 16, false, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    if (k <= 32) return launch_bdl_knn<T, MD, 32, false, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    return launch_bdl_knn<T, MD, 64, false, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
}

template <typename T, int TK>
pg_status bdl_knn_d(const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d, int k,
                    int64_t mx, int32_t* rd, uint32_t* nr, int64_t* oi, void* od, hipStream_t s) {
    switch (d) {
        case 2: return bdl_knn_k<T, 2, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
        case 3: return bdl_knn_k<T, 3, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
        case 5: return bdl_knn_k<T, 5, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
        default: return bdl_knn_k<T, 8, TK>(f, q, o, qk, m, d, k, mx, rd, nr, oi, od, s);
    }
}

// id_end: every id of the forest is below it (the next id to be given).
template <typename T>
pg_status forest_knn_any(int tk, const Forest& f, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int d,
                      int k, int64_t id_end, int32_t* rd, uint32_t* nr, int64_t* oi, void* od,
                      hipStream_t s) {
    if (tk == kTreeX) return bdl_knn_d<T, kTreeX>(f, q, o, qk, m, d, k, id_end, rd, nr, oi, od, s);
    if (tk == kTreeLoff) return bdl_knn_d<T, kTreeLoff>(f, q, o, qk, m, d, k, id_end, rd, nr, oi, od, s);
    return bdl_knn_d<T, kTreeHeap>(f, q, o, qk, m, d, k, id_end, rd, nr, oi, od, s);
}

}  // namespace forest_detail
}  // namespace pg
