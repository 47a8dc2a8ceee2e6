// Static-tree k-NN kernels and their launch dispatch (one query per lane,
// Appendix C "Data-Parallel k-NN"), instantiated per coordinate type in
// knn_int.hip and knn_float.hip.  In all-points mode lane i takes the tree's
// own leaf-order point i, so the lanes of a wave hold neighbouring points and
// walk nearly the same nodes; the result row is the point's input row.
#pragma once

#include <cstdlib>
#include <string>

#include "scan.hpp"
#include "xsearch.hpp"
#include "wave.hpp"

namespace pg {
namespace knn_detail {

constexpr int kNT = 256;

template <typename T, int MD>
__device__ inline void load_query(const TreeView& tv, const uint32_t* queries, int all, int64_t i,
                                  int d, T (&q)[MD]) {
#pragma unroll
    for (int c = 0; c < MD; c++) {
        uint32_t b = 0;
        if (MD < 8 || c < d) b = all ? tv.pts[(int64_t)c * tv.n + i] : queries[i * d + c];
        q[c] = Metric<T>::load(b);
    }
}

// Searches with packed (distance, id) keys.  A query whose k-th distance
// reached the packed range's limit (int32 coordinates: 2^(64-B) - 1, or fewer
// than k points) is appended to `redo` for knn_redo_kernel instead of written.
// NS (all-points only): the query's own point is not a candidate (k-NN graph).
// TK: the tree kind (kTreeHeap, kTreeLoff, kTreeX).
template <typename T, int MD, int KT, bool EX, bool NS, int TK>
__global__ void __launch_bounds__(kNT)
knn_static_kernel(TreeView tv, const uint32_t* __restrict__ queries,
                  const int32_t* __restrict__ order, QueryKeys qk, int64_t m, int k, int all, int idbits,
                  int32_t* __restrict__ out_idx, typename Metric<T>::D* __restrict__ out_dist,
                  int32_t* __restrict__ redo, uint32_t* __restrict__ nredo) {
    const int d = MD < 8 ? MD : tv.d;
    const int64_t i0 = xcd_block() * kNT + threadIdx.x;
    if (i0 >= m) return;
    // queries are taken in leaf order when an order is given (neighbouring
    // lanes then walk nearly the same nodes); results go to the query's row
    const int64_t i = order ? (int64_t)order[i0] : i0;
    T q[MD];
    load_query<T, MD>(tv, queries, all, i, d, q);
    using KL = PackedList<T, KT, EX>;
    KL kl;
    kl.init(idbits);
    const uint32_t start = search_start<TK>(tv, all != 0, i);
    if constexpr (NS) tree_search<T, MD, KL, OtherIds, TK>(tv, OtherIds{i}, q, d, kl, k, start);
    else tree_search<T, MD, KL, PlainIds, TK>(tv, PlainIds{}, q, d, kl, k, start,
                                              all ? root_from<TK>()
                                                  : descend_from<T, MD, TK>(tv, q, d, search_from<TK>(tv, qk, i)));
    if (kl.needs_redo()) {
        redo[atomicAdd(nredo, 1u)] = (int32_t)i;
        return;
    }
    const int64_t row = all ? (int64_t)tv.pidx[i] : i;
#pragma unroll
    for (int s = 0; s < KT; s++) {
        if (EX || s < k) {
            out_idx[row * k + s] = kl.id_of(kl.key[s]);
            out_dist[row * k + s] = kl.dist_of(kl.key[s]);
        }
    }
}

// The queries knn_static_kernel handed over, searched with exact
// (distance, id) pairs.
template <typename T, int MD, int KT, bool EX, bool NS, int TK>
__global__ void __launch_bounds__(kNT)
knn_redo_kernel(TreeView tv, const uint32_t* __restrict__ queries, int k, int all,
                const int32_t* __restrict__ redo, const uint32_t* __restrict__ nredo,
                int32_t* __restrict__ out_idx, typename Metric<T>::D* __restrict__ out_dist) {
    using M = Metric<T>;
    const int d = MD < 8 ? MD : tv.d;
    const int64_t cnt = *nredo;
    for (int64_t r = (int64_t)blockIdx.x * kNT + threadIdx.x; r < cnt; r += (int64_t)gridDim.x * kNT) {
        const int64_t i = redo[r];
        T q[MD];
        load_query<T, MD>(tv, queries, all, i, d, q);
        using KL = KList<typename M::D, int32_t, KT, EX>;
        KL kl;
        kl.init(M::inf(), INT32_MAX);
        const uint32_t start = search_start<TK>(tv, all != 0, i);
        if constexpr (NS) tree_search<T, MD, KL, OtherIds, TK>(tv, OtherIds{i}, q, d, kl, k, start);
        else tree_search<T, MD, KL, PlainIds, TK>(tv, PlainIds{}, q, d, kl, k, start);
        const int64_t row = all ? (int64_t)tv.pidx[i] : i;
#pragma unroll
        for (int s = 0; s < KT; s++) {
            if (EX || s < k) {
                out_idx[row * k + s] = kl.id[s] == INT32_MAX ? -1 : kl.id[s];
                out_dist[row * k + s] = kl.d[s];
            }
        }
    }
}

constexpr unsigned kRedoBlocks = 512;

}  // namespace knn_detail
}  // namespace pg

#include "knn_wave.hpp"

namespace pg {
namespace knn_detail {

// Whether a heap tree with node boxes takes the wave-per-block walk
// (knn_wave.hpp) instead of the per-lane walk.  The per-lane walk is the
// default: measured on 3-D n = 10M all-points k = 10, the wave walk issues
// about twice the vector instructions per wave (each lane measures every
// point of the union of the wave's leaves, about ten times the points of its
// own search) and runs about five times longer.  PG_KNN_WAVE selects it, read
// at every launch: "all" (all-points searches), "sep" (separate queries),
// "both"; anything else, or unset, keeps the per-lane walk.
inline bool use_wave_kernel(bool all) {
    const char* e = std::getenv("PG_KNN_WAVE");
    if (!e) return false;
    const std::string v(e);
    const int mode = v == "all" ? 1 : v == "sep" ? 2 : v == "both" ? 3 : 0;
    return all ? (mode & 1) != 0 : (mode & 2) != 0;
}

template <typename T, int MD, int KT, bool EX, bool NS, int TK>
pg_status launch_static(const pg_tree* t, const void* queries, const int32_t* order, QueryKeys qk, int64_t m,
                        int k, bool all, int32_t* out_idx, void* out_dist, hipStream_t s,
                        const KnnWs* ws) {
    using DT = typename Metric<T>::D;
    constexpr bool exact = PackedList<T, KT, EX>::kFloat;  // float keys: no redo pass
    DevBuf rbuf(s);
    int32_t* redo = nullptr;
    uint32_t* nredo = nullptr;
    if (!exact) {
        if (ws) {
            redo = ws->redo;
            nredo = ws->nredo;
        } else {
            PG_TRY(rbuf.alloc(sizeof(int32_t) * (m + 1)));
            nredo = rbuf.as<uint32_t>();
            redo = rbuf.as<int32_t>() + 1;
        }
        PG_TRY(fill_u32(nredo, 1, 0u, s));
    }
    const TreeView tv = t->view();
    bool wave = false;
    if constexpr (TK == kTreeHeap && MD <= 7) {
        if (tv.nbox != nullptr && t->leaf <= kWave && use_wave_kernel(all)) {
            wave = true;
            hipLaunchKernelGGL((knn_wave_kernel<T, MD, KT, EX, NS>), dim3(grid_for_xcd(cdiv(m, kNT))),
                               dim3(kNT), 0, s, tv, (const uint32_t*)queries, order, m, k, all ? 1 : 0,
                               id_bits(t->n), out_idx, (DT*)out_dist, redo, nredo, tv.split, tv.nbox,
                               tv.rec);
        }
    }
    if (!wave)
        hipLaunchKernelGGL((knn_static_kernel<T, MD, KT, EX, NS, TK>), dim3(grid_for_xcd(cdiv(m, kNT))),
                           dim3(kNT), 0, s, tv, (const uint32_t*)queries, order, qk, m, k,
                           all ? 1 : 0, id_bits(t->n), out_idx, (DT*)out_dist, redo, nredo);
    PG_LAUNCH_CHECK();
    if (!exact) {
        hipLaunchKernelGGL((knn_redo_kernel<T, MD, KT, EX, NS, TK>), dim3(kRedoBlocks), dim3(kNT), 0, s,
                           t->view(), (const uint32_t*)queries, k, all ? 1 : 0, redo, nredo, out_idx,
                           (DT*)out_dist);
        PG_LAUNCH_CHECK();
    }
    return PG_OK;
}

// k-list capacities: exact lists for the common k = 5, 10, 16, otherwise the
// next power of two with uniform guards.
template <typename T, int MD, bool NS, int TK>
pg_status dispatch_k(const pg_tree* t, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int k, bool all,
                     int32_t* oi, void* od, hipStream_t s, const KnnWs* ws) {
    if (k == 5) return launch_static<T, MD, 5, true, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k == 10) return launch_static<T, MD, 10, true, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k == 16) return launch_static<T, MD, 16, true, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k <= 2) return launch_static<T, MD, 2, false, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k <= 4) return launch_static<T, MD, 4, false, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k <= 8) return launch_static<T, MD, 8, false, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k <= 16) return launch_static<T, MD, 16, false, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    if (k <= 32) return launch_static<T, MD, 32, false, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    return launch_static<T, MD, 64, false, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
}

template <typename T, bool NS, int TK>
pg_status dispatch_d(const pg_tree* t, const void* q, const int32_t* o, QueryKeys qk, int64_t m, int k, bool all,
                     int32_t* oi, void* od, hipStream_t s, const KnnWs* ws) {
    switch (t->d) {
        case 2: return dispatch_k<T, 2, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
        case 3: return dispatch_k<T, 3, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
        case 5: return dispatch_k<T, 5, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
        default: return dispatch_k<T, 8, NS, TK>(t, q, o, qk, m, k, all, oi, od, s, ws);
    }
}

}  // namespace knn_detail
}  // namespace pg
