// Batched k-NN over a static kd-tree (Appendix C, "Data-Parallel k-NN"):
// query checks, query ordering by leaf, and the dispatch to the per-type
// kernels (knn_static.hpp, instantiated in knn_int.hip / knn_float.hip).
#include "scan.hpp"
#include "xsearch.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;

// Sort key of each query: the node of level `levels` its descent reaches
// (left below the split, right at or above it).  A box query (rows lo[d],
// hi[d]) descends by its centre.  The splits of the top kTopLevels levels
// are read from LDS (the deeper ones are gathers from the split array), and
// a workgroup takes kLeafQpt * kNT queries to share that copy.
constexpr int kTopLevels = 12;
constexpr int kLeafQpt = 4;

__global__ void __launch_bounds__(kNT)
query_leaf_kernel(TreeView tv, int fl, const uint32_t* __restrict__ queries, int64_t m,
                  int levels, int box, uint32_t* __restrict__ key, uint32_t* __restrict__ cnt) {
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
            if (tv.sdim) dim = tv.sdim[cur];
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
        atomicAdd(&cnt[cur - (1u << levels)], 1u);  // the bucket's count
    }
}

// The same for explicit-node trees: the leaf index the descent reaches.
__global__ void __launch_bounds__(kNT)
query_xleaf_kernel(TreeView tv, int fl, const uint32_t* __restrict__ queries, int64_t m, int box,
                   int shift, uint32_t* __restrict__ key, uint32_t* __restrict__ cnt) {
    const int d = tv.d;
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= m) return;
    const int64_t row = box ? i * 2 * d : i * d;
    uint32_t cur = 0;
    uint4 r = tv.xn[0];
    while (!(r.w & kXLeaf)) {
        const int dim = r.w & 15u;
        const uint32_t qb = queries[row + dim], sb = r.x;
        bool right;
        if (box) {
            const uint32_t hb = queries[row + d + dim];
            right = fl ? 0.5f * __uint_as_float(qb) + 0.5f * __uint_as_float(hb) >= __uint_as_float(sb)
                       : (int64_t)(int32_t)qb + (int32_t)hb >= 2 * (int64_t)(int32_t)sb;
        } else {
            right = fl ? __uint_as_float(qb) >= __uint_as_float(sb) : (int32_t)qb >= (int32_t)sb;
        }
        cur = r.y + (right ? 1u : 0u);
        r = tv.xn[cur];
    }
    key[i] = r.x;
    atomicAdd(&cnt[r.x >> shift], 1u);  // the bucket's count
}

// Bucket of a query: its key shifted right by `shift`.  start[b] is the
// next free slot of bucket b (the exclusive prefix sum of the counts the
// descent kernels took); each query takes one.
__global__ void bucket_fill_kernel(const uint32_t* __restrict__ key, int64_t m, int shift,
                                   uint32_t* __restrict__ start, int32_t* __restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < m) order[atomicAdd(&start[key[i] >> shift], 1u)] = (int32_t)i;
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

}  // namespace

pg_status check_queries_ws(const void* q, int64_t m, int d, bool fl, uint32_t* err, hipStream_t s) {
    if (m == 0) return PG_OK;
    PG_TRY(fill_u32(err, 1, 0u, s));
    const int64_t count = m * d;
    hipLaunchKernelGGL(check_queries_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s,
                       (const uint32_t*)q, count, fl ? 1 : 0, err);
    PG_LAUNCH_CHECK();
    uint32_t h = 0;
    PG_HIP(hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h) return fail(PG_ERR_RANGE, "query coordinate out of range (int32: [-2^29, 2^29); float32: finite, |x| <= 1e18)");
    return PG_OK;
}

pg_status check_queries(const void* q, int64_t m, int d, bool fl, hipStream_t s) {
    if (m == 0) return PG_OK;
    DevBuf err(s);
    PG_TRY(err.alloc(sizeof(uint32_t)));
    return check_queries_ws(q, m, d, fl, err.as<uint32_t>(), s);
}

// Bucket shift and count of the query ordering: the leaves, coarsened to
// about one bucket per 4 queries.
static void bucket_plan(const TreeView& tv, int64_t m, int* shift_out, int64_t* nb_out) {
    int bits = 0;
    while (bits < 24 && ((int64_t)1 << (bits + 1)) * 4 <= m) bits++;
    int lbits = tv.L;  // leaves < 2^lbits
    if (tv.xn) {
        lbits = 0;
        while (((int64_t)1 << lbits) < tv.nleaves) lbits++;
    }
    const int shift = lbits > bits ? lbits - bits : 0;
    *shift_out = shift;
    *nb_out = tv.xn ? ((tv.nleaves + ((int64_t)1 << shift) - 1) >> shift)
                    : (((int64_t)1 << tv.L) >> shift);
}

int64_t order_buckets(const TreeView& tv, int64_t m) {
    int shift;
    int64_t nb;
    bucket_plan(tv, m, &shift, &nb);
    return nb;
}

pg_status order_queries(const TreeView& tv, bool fl, const void* queries, int64_t m,
                        hipStream_t s, DevBuf& order, bool boxes, QueryKeys* keys) {
    // one allocation: the order, the queries' keys, the bucket counts, the
    // scan's partial sums
    const int64_t nb = order_buckets(tv, m);
    PG_TRY(order.alloc(sizeof(uint32_t) * (m + m + nb + scan_partials(nb))));
    uint32_t* work = order.as<uint32_t>() + m;
    return order_queries_ws(tv, fl, queries, m, s, order.as<int32_t>(), work, work + m + nb, boxes, keys);
}

pg_status order_queries_ws(const TreeView& tv, bool fl, const void* queries, int64_t m,
                           hipStream_t s, int32_t* order, uint32_t* work, uint32_t* sums,
                           bool boxes, QueryKeys* keys) {
    int shift;
    int64_t nb;
    bucket_plan(tv, m, &shift, &nb);
    // heap trees: keys are the nodes of level L - shift (the buckets);
    // explicit-node trees: leaf indices, shifted into buckets
    // the queries' bucket keys, then the bucket counts (which the scan turns,
    // in place, into each bucket's next free slot)
    uint32_t* key = work;
    uint32_t* cnt = key + m;
    PG_TRY(fill_u32(cnt, nb, 0u, s));
    const int kshift = tv.xn ? shift : 0;
    // (the descent kernels also count each bucket's queries)
    if (tv.xn)
        hipLaunchKernelGGL(query_xleaf_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, tv, fl ? 1 : 0,
                           (const uint32_t*)queries, m, boxes ? 1 : 0, kshift, key, cnt);
    else
        hipLaunchKernelGGL(query_leaf_kernel, dim3(cdiv(m, (int64_t)kNT * kLeafQpt)), dim3(kNT), 0, s,
                           tv, fl ? 1 : 0, (const uint32_t*)queries, m, tv.L - shift, boxes ? 1 : 0, key, cnt);
    PG_LAUNCH_CHECK();
    PG_TRY(exclusive_scan_u32_ws(cnt, cnt, nb, nullptr, sums, s));
    hipLaunchKernelGGL(bucket_fill_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, key, m, kshift, cnt, order);
    PG_LAUNCH_CHECK();
    if (keys) {
        keys->key = key;
        keys->lev = tv.xn ? -1 : tv.L - shift;
    }
    return PG_OK;
}

pg_status knn_static(const pg_tree* t, const void* queries, int64_t m, int k, bool all,
                     int32_t* out_idx, void* out_dist, hipStream_t s, bool no_self, const KnnWs* ws) {
    if (m == 0) return PG_OK;
    DevBuf order(s);
    const int32_t* o = nullptr;
    QueryKeys qk;
    if (!all && m >= kOrderMin && t->n > 0) {
        if (ws) {
            PG_TRY(order_queries_ws(t->view(), t->dtype == PG_FLOAT32, queries, m, s, ws->order,
                                    ws->work, ws->sums, false, &qk));
            o = ws->order;
        } else {
            PG_TRY(order_queries(t->view(), t->dtype == PG_FLOAT32, queries, m, s, order, false, &qk));
            o = order.as<int32_t>();
        }
    }
    if (t->dtype == PG_FLOAT32)
        return knn_static_float(t, queries, o, qk, m, k, all, out_idx, out_dist, s, no_self, ws);
    return knn_static_int(t, queries, o, qk, m, k, all, out_idx, out_dist, s, no_self, ws);
}

}  // namespace pg
