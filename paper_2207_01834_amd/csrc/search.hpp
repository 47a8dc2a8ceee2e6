// Single-query kd-tree search used by every k-NN kernel (static trees, BDL
// forests, batched clouds): one query per lane, stack-free.
//
// Semantics (Appendix C, "Data-Parallel k-NN"): queries are independent and
// each search is serial; the result is the k smallest (distance, id) keys.
// The traversal differs from the paper's recursive one, for the GPU:
//   * the tree is an implicit heap (children 2h, 2h+1, parent h/2), so the
//     walk keeps only (current, previous) node in registers: coming from the
//     parent it enters the child on the query's side; coming back from that
//     child it enters the other child unless the squared distance to the
//     split plane exceeds the current k-th distance (strict, so equal keys
//     with smaller ids are still found); otherwise it returns to the parent;
//   * a leaf is scanned only when the squared distance from the query to the
//     leaf's bounding box does not exceed the current k-th distance;
//   * candidates go into a register-resident sorted k-list (KList).
#pragma once

#include "knn.hpp"

namespace pg {

template <int MD, typename T>
__device__ inline T pick(const T (&q)[MD], int dim) {
    T r = q[0];
#pragma unroll
    for (int c = 1; c < MD; c++) r = dim == c ? q[c] : r;
    return r;
}

// Points of leaf-order position i: id and liveness.
struct PlainIds {
    const int32_t* pidx;
    __device__ inline int32_t id(int64_t i) const { return pidx[i]; }
    __device__ inline bool live(int64_t) const { return true; }
};

template <typename T, int MD, int KT, typename IT, typename Ids>
__device__ inline void kd_search(const TreeView& tv, const Ids& ids, const T (&q)[MD], int d,
                                 KList<typename Metric<T>::D, IT, KT>& kl, int k) {
    using M = Metric<T>;
    using DT = typename M::D;
    const int64_t n = tv.n;
    if (n == 0) return;
    const int L = tv.L;
    const uint32_t first_leaf = 1u << L;
    uint32_t cur = 1, prev = 0;
    int dim = 0;
    while (cur != 0) {
        while (cur != 0 && cur < first_leaf) {
            const T s = M::load(tv.split[cur]);
            const T qd = pick<MD>(q, dim);
            const uint32_t nearc = 2u * cur + (qd >= s ? 1u : 0u);
            uint32_t next;
            if (prev == (cur >> 1)) next = nearc;
            else if (prev == nearc && !(M::sq(qd, s) > kl.kd)) next = nearc ^ 1u;
            else next = cur >> 1;
            if (next > cur) dim = (dim + 1 == d) ? 0 : dim + 1;
            else dim = (dim == 0) ? d - 1 : dim - 1;
            prev = cur;
            cur = next;
        }
        if (cur == 0) break;
        const uint32_t leaf = cur - first_leaf;
        const uint32_t* bb = tv.bbox + (size_t)leaf * 2 * d;
        DT lb = 0;
#pragma unroll
        for (int c = 0; c < MD; c++)
            if (c < d) lb = M::acc_gap(lb, q[c], M::load(bb[c]), M::load(bb[d + c]));
        if (!(lb > kl.kd)) {
            const int64_t lo = node_start(n, L, leaf), hi = node_start(n, L, leaf + 1);
            for (int64_t i = lo; i < hi; i++) {
                if (!ids.live(i)) continue;
                DT dd = 0;
#pragma unroll
                for (int c = 0; c < MD; c++)
                    if (c < d) dd = M::acc(dd, q[c], M::load(tv.pts[(int64_t)c * n + i]));
                const IT id = ids.id(i);
                if (kl.admits(dd, id)) kl.insert(dd, id, k);
            }
        }
        prev = cur;
        cur >>= 1;
        dim = (dim == 0) ? d - 1 : dim - 1;
    }
}

}  // namespace pg
