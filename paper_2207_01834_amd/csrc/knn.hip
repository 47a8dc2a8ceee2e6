// Batched k-NN over a static kd-tree: one query per lane (Appendix C,
// "Data-Parallel k-NN").  In all-points mode lane i takes the tree's own
// leaf-order point i, so the lanes of a wave hold neighbouring points and
// walk nearly the same nodes; the result row is the point's input row.
#include "scan.hpp"
#include "search.hpp"
#include "wave.hpp"

namespace pg {

namespace {

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
// LOFF: the tree's leaf ranges are explicit offsets (spatial-median trees).
template <typename T, int MD, int KT, bool EX, bool NS, bool LOFF>
__global__ void __launch_bounds__(kNT)
knn_static_kernel(TreeView tv, const uint32_t* __restrict__ queries,
                  const int32_t* __restrict__ order, int64_t m, int k, int all, int idbits,
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
    const uint32_t start =
        all ? (1u << tv.L) + (LOFF ? leaf_at(tv.loff, tv.L, i) : leaf_of(tv.n, tv.L, i)) : 0u;
    if constexpr (NS) kd_search<T, MD, KL, OtherIds, LOFF>(tv, OtherIds{i}, q, d, kl, k, start);
    else kd_search<T, MD, KL, PlainIds, LOFF>(tv, PlainIds{}, q, d, kl, k, start);
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
template <typename T, int MD, int KT, bool EX, bool NS, bool LOFF>
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
        const uint32_t start =
            all ? (1u << tv.L) + (LOFF ? leaf_at(tv.loff, tv.L, i) : leaf_of(tv.n, tv.L, i)) : 0u;
        if constexpr (NS) kd_search<T, MD, KL, OtherIds, LOFF>(tv, OtherIds{i}, q, d, kl, k, start);
        else kd_search<T, MD, KL, PlainIds, LOFF>(tv, PlainIds{}, q, d, kl, k, start);
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

// Sort key of each query: the node of level `levels` its descent reaches
// (left below the split, right at or above it).  A box query (rows lo[d],
// hi[d]) descends by its centre.  The splits of the top kTopLevels levels
// are read from LDS (the deeper ones are gathers from the split array), and
// a workgroup takes kLeafQpt * kNT queries to share that copy.
constexpr int kTopLevels = 12;
constexpr int kLeafQpt = 4;

__global__ void __launch_bounds__(kNT)
query_leaf_kernel(TreeView tv, int fl, const uint32_t* __restrict__ queries, int64_t m,
                  int levels, int box, uint32_t* __restrict__ key) {
    __shared__ uint32_t top[1 << kTopLevels];
    const int tl = levels < kTopLevels ? levels : kTopLevels;
    for (int e = threadIdx.x; e < (1 << tl); e += kNT) top[e] = e ? tv.split[e] : 0u;
    __syncthreads();
    const int d = tv.d;
    for (int r = 0; r < kLeafQpt; r++) {
        const int64_t i = ((int64_t)blockIdx.x * kLeafQpt + r) * kNT + threadIdx.x;
        if (i >= m) return;
        const int64_t row = box ? i * 2 * d : i * d;
        uint32_t cur = 1;
        int dim = 0;
        for (int lvl = 0; lvl < levels; lvl++) {
            const uint32_t qb = queries[row + dim];
            const uint32_t sb = lvl < tl ? top[cur] : tv.split[cur];
            bool right;
            if (box) {
                const uint32_t hb = queries[row + d + dim];
                right = fl ? 0.5f * __uint_as_float(qb) + 0.5f * __uint_as_float(hb) >= __uint_as_float(sb)
                           : (int64_t)(int32_t)qb + (int32_t)hb >= 2 * (int64_t)(int32_t)sb;
            } else {
                right = fl ? __uint_as_float(qb) >= __uint_as_float(sb) : (int32_t)qb >= (int32_t)sb;
            }
            cur = 2u * cur + (right ? 1u : 0u);
            dim = dim + 1 == d ? 0 : dim + 1;
        }
        key[i] = cur - (1u << levels);
    }
}

__global__ void bucket_count_kernel(const uint32_t* __restrict__ key, int64_t m,
                                    uint32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < m) atomicAdd(&cnt[key[i]], 1u);
}

__global__ void bucket_fill_kernel(const uint32_t* __restrict__ key, int64_t m,
                                   const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                                   int32_t* __restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < m) {
        const uint32_t b = key[i];
        order[start[b] + atomicAdd(&cursor[b], 1u)] = (int32_t)i;
    }
}

__global__ void check_queries_kernel(const uint32_t* __restrict__ q, int64_t count, int fl,
                                     uint32_t* __restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < count) {
        const uint32_t b = q[i];
        if (fl) bad = !(fabsf(__uint_as_float(b)) <= 1e18f);
        else bad = (int32_t)b < -(1 << 29) || (int32_t)b >= (1 << 29);
    }
    if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(err, 1u);
}

constexpr unsigned kRedoBlocks = 512;

template <typename T, int MD, int KT, bool EX, bool NS, bool LOFF>
pg_status launch_static(const pg_tree* t, const void* queries, const int32_t* order, int64_t m,
                        int k, bool all, int32_t* out_idx, void* out_dist, hipStream_t s) {
    using DT = typename Metric<T>::D;
    constexpr bool exact = PackedList<T, KT, EX>::kFloat;  // float keys: no redo pass
    DevBuf redo(s), nredo(s);
    if (!exact) {
        PG_TRY(redo.alloc(sizeof(int32_t) * m));
        PG_TRY(nredo.alloc(sizeof(uint32_t)));
        PG_HIP(hipMemsetAsync(nredo.p, 0, sizeof(uint32_t), s));
    }
    hipLaunchKernelGGL((knn_static_kernel<T, MD, KT, EX, NS, LOFF>), dim3(grid_for_xcd(cdiv(m, kNT))),
                       dim3(kNT), 0, s, t->view(), (const uint32_t*)queries, order, m, k,
                       all ? 1 : 0, id_bits(t->n), out_idx, (DT*)out_dist, redo.as<int32_t>(),
                       nredo.as<uint32_t>());
    PG_LAUNCH_CHECK();
    if (!exact) {
        hipLaunchKernelGGL((knn_redo_kernel<T, MD, KT, EX, NS, LOFF>), dim3(kRedoBlocks), dim3(kNT), 0, s,
                           t->view(), (const uint32_t*)queries, k, all ? 1 : 0,
                           redo.as<int32_t>(), nredo.as<uint32_t>(), out_idx, (DT*)out_dist);
        PG_LAUNCH_CHECK();
    }
    return PG_OK;
}

// k-list capacities: exact lists for the common k = 5, 10, 16, otherwise the
// next power of two with uniform guards.
template <typename T, int MD, bool NS, bool LOFF>
pg_status dispatch_k(const pg_tree* t, const void* q, const int32_t* o, int64_t m, int k, bool all,
                     int32_t* oi, void* od, hipStream_t s) {
    if (k == 5) return launch_static<T, MD, 5, true, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k == 10) return launch_static<T, MD, 10, true, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k == 16) return launch_static<T, MD, 16, true, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k <= 2) return launch_static<T, MD, 2, false, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k <= 4) return launch_static<T, MD, 4, false, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k <= 8) return launch_static<T, MD, 8, false, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k <= 16) return launch_static<T, MD, 16, false, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    if (k <= 32) return launch_static<T, MD, 32, false, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    return launch_static<T, MD, 64, false, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
}

template <typename T, bool NS, bool LOFF>
pg_status dispatch_d(const pg_tree* t, const void* q, const int32_t* o, int64_t m, int k, bool all,
                     int32_t* oi, void* od, hipStream_t s) {
    switch (t->d) {
        case 2: return dispatch_k<T, 2, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
        case 3: return dispatch_k<T, 3, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
        case 5: return dispatch_k<T, 5, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
        default: return dispatch_k<T, 8, NS, LOFF>(t, q, o, m, k, all, oi, od, s);
    }
}

}  // namespace

pg_status check_queries(const void* q, int64_t m, int d, bool fl, hipStream_t s) {
    if (m == 0) return PG_OK;
    DevBuf err(s);
    PG_TRY(err.alloc(sizeof(uint32_t)));
    PG_HIP(hipMemsetAsync(err.p, 0, sizeof(uint32_t), s));
    const int64_t count = m * d;
    hipLaunchKernelGGL(check_queries_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s,
                       (const uint32_t*)q, count, fl ? 1 : 0, err.as<uint32_t>());
    PG_LAUNCH_CHECK();
    uint32_t h = 0;
    PG_HIP(hipMemcpyAsync(&h, err.p, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h) return fail(PG_ERR_RANGE, "query coordinate out of range (int32: [-2^29, 2^29); float32: finite, |x| <= 1e18)");
    return PG_OK;
}

pg_status order_queries(const TreeView& tv, bool fl, const void* queries, int64_t m,
                        hipStream_t s, DevBuf& order, bool boxes) {
    // buckets: the leaves, coarsened to about one bucket per 4 queries
    int bits = 0;
    while (bits < 24 && ((int64_t)1 << (bits + 1)) * 4 <= m) bits++;
    const int shift = tv.L > bits ? tv.L - bits : 0;
    const int64_t nb = ((int64_t)1 << tv.L) >> shift;
    DevBuf key(s), cnt(s), start(s), cursor(s);
    PG_TRY(key.alloc(sizeof(uint32_t) * m));
    PG_TRY(cnt.alloc(sizeof(uint32_t) * nb));
    PG_TRY(start.alloc(sizeof(uint32_t) * nb));
    PG_TRY(cursor.alloc(sizeof(uint32_t) * nb));
    PG_TRY(order.alloc(sizeof(int32_t) * m));
    PG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t) * nb, s));
    PG_HIP(hipMemsetAsync(cursor.p, 0, sizeof(uint32_t) * nb, s));
    hipLaunchKernelGGL(query_leaf_kernel, dim3(cdiv(m, (int64_t)kNT * kLeafQpt)), dim3(kNT), 0, s,
                       tv, fl ? 1 : 0, (const uint32_t*)queries, m, tv.L - shift, boxes ? 1 : 0,
                       key.as<uint32_t>());
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(bucket_count_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s,
                       key.as<uint32_t>(), m, cnt.as<uint32_t>());
    PG_LAUNCH_CHECK();
    PG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), start.as<uint32_t>(), nb, nullptr, s));
    hipLaunchKernelGGL(bucket_fill_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s,
                       key.as<uint32_t>(), m, start.as<uint32_t>(), cursor.as<uint32_t>(),
                       order.as<int32_t>());
    PG_LAUNCH_CHECK();
    return PG_OK;
}

pg_status knn_static(const pg_tree* t, const void* queries, int64_t m, int k, bool all,
                     int32_t* out_idx, void* out_dist, hipStream_t s, bool no_self) {
    if (m == 0) return PG_OK;
    DevBuf order(s);
    const int32_t* o = nullptr;
    if (!all && m >= kOrderMin && t->n > 0) {
        PG_TRY(order_queries(t->view(), t->dtype == PG_FLOAT32, queries, m, s, order));
        o = order.as<int32_t>();
    }
    const bool fl = t->dtype == PG_FLOAT32;
    if (t->loff) {
        if (no_self)
            return fl ? dispatch_d<float, true, true>(t, nullptr, nullptr, m, k, true, out_idx, out_dist, s)
                      : dispatch_d<int32_t, true, true>(t, nullptr, nullptr, m, k, true, out_idx, out_dist, s);
        return fl ? dispatch_d<float, false, true>(t, queries, o, m, k, all, out_idx, out_dist, s)
                  : dispatch_d<int32_t, false, true>(t, queries, o, m, k, all, out_idx, out_dist, s);
    }
    if (no_self)
        return fl ? dispatch_d<float, true, false>(t, nullptr, nullptr, m, k, true, out_idx, out_dist, s)
                  : dispatch_d<int32_t, true, false>(t, nullptr, nullptr, m, k, true, out_idx, out_dist, s);
    return fl ? dispatch_d<float, false, false>(t, queries, o, m, k, all, out_idx, out_dist, s)
              : dispatch_d<int32_t, false, false>(t, queries, o, m, k, all, out_idx, out_dist, s);
}

}  // namespace pg
