// Batched k-NN over a static kd-tree: one query per lane (Appendix C,
// "Data-Parallel k-NN").  In all-points mode lane i takes the tree's own
// leaf-order point i, so the lanes of a wave hold neighbouring points and
// walk nearly the same nodes; the result row is the point's input row.
#include "search.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;

template <typename T, int MD, int KT, bool EX>
__global__ void __launch_bounds__(kNT)
knn_static_kernel(TreeView tv, const uint32_t* __restrict__ queries, int64_t m, int k, int all,
                  int32_t* __restrict__ out_idx, typename Metric<T>::D* __restrict__ out_dist) {
    using M = Metric<T>;
    const int d = MD < 8 ? MD : tv.d;
    const int64_t i = xcd_block() * kNT + threadIdx.x;
    if (i >= m) return;
    T q[MD];
#pragma unroll
    for (int c = 0; c < MD; c++) {
        uint32_t b = 0;
        if (MD < 8 || c < d) b = all ? tv.pts[(int64_t)c * tv.n + i] : queries[i * d + c];
        q[c] = M::load(b);
    }
    KList<typename M::D, int32_t, KT, EX> kl;
    kl.init(M::inf(), INT32_MAX);
    const uint32_t start = all ? (1u << tv.L) + leaf_of(tv.n, tv.L, i) : 0u;
    kd_search<T, MD, KT, EX, int32_t>(tv, PlainIds{}, q, d, kl, k, start);
    const int64_t row = all ? (int64_t)tv.pidx[i] : i;
#pragma unroll
    for (int s = 0; s < KT; s++) {
        if (EX || s < k) {
            out_idx[row * k + s] = kl.id[s] == INT32_MAX ? -1 : kl.id[s];
            out_dist[row * k + s] = kl.d[s];
        }
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

template <typename T, int MD, int KT, bool EX>
pg_status launch_static(const pg_tree* t, const void* queries, int64_t m, int k, bool all,
                        int32_t* out_idx, void* out_dist, hipStream_t s) {
    using DT = typename Metric<T>::D;
    hipLaunchKernelGGL((knn_static_kernel<T, MD, KT, EX>), dim3(grid_for_xcd(cdiv(m, kNT))),
                       dim3(kNT), 0, s, t->view(), (const uint32_t*)queries, m, k, all ? 1 : 0,
                       out_idx, (DT*)out_dist);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

// k-list capacities: exact lists for the common k = 5, 10, 16, otherwise the
// next power of two with uniform guards.
template <typename T, int MD>
pg_status dispatch_k(const pg_tree* t, const void* q, int64_t m, int k, bool all, int32_t* oi,
                     void* od, hipStream_t s) {
    if (k == 5) return launch_static<T, MD, 5, true>(t, q, m, k, all, oi, od, s);
    if (k == 10) return launch_static<T, MD, 10, true>(t, q, m, k, all, oi, od, s);
    if (k == 16) return launch_static<T, MD, 16, true>(t, q, m, k, all, oi, od, s);
    if (k <= 2) return launch_static<T, MD, 2, false>(t, q, m, k, all, oi, od, s);
    if (k <= 4) return launch_static<T, MD, 4, false>(t, q, m, k, all, oi, od, s);
    if (k <= 8) return launch_static<T, MD, 8, false>(t, q, m, k, all, oi, od, s);
    if (k <= 16) return launch_static<T, MD, 16, false>(t, q, m, k, all, oi, od, s);
    if (k <= 32) return launch_static<T, MD, 32, false>(t, q, m, k, all, oi, od, s);
    return launch_static<T, MD, 64, false>(t, q, m, k, all, oi, od, s);
}

template <typename T>
pg_status dispatch_d(const pg_tree* t, const void* q, int64_t m, int k, bool all, int32_t* oi,
                     void* od, hipStream_t s) {
    switch (t->d) {
        case 2: return dispatch_k<T, 2>(t, q, m, k, all, oi, od, s);
        case 3: return dispatch_k<T, 3>(t, q, m, k, all, oi, od, s);
        case 5: return dispatch_k<T, 5>(t, q, m, k, all, oi, od, s);
        default: return dispatch_k<T, 8>(t, q, m, k, all, oi, od, s);
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

pg_status knn_static(const pg_tree* t, const void* queries, int64_t m, int k, bool all,
                     int32_t* out_idx, void* out_dist, hipStream_t s) {
    if (m == 0) return PG_OK;
    if (t->dtype == PG_FLOAT32) return dispatch_d<float>(t, queries, m, k, all, out_idx, out_dist, s);
    return dispatch_d<int32_t>(t, queries, m, k, all, out_idx, out_dist, s);
}

}  // namespace pg
