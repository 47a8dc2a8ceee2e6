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
//   * when the query is a point of the tree (all-points mode) the walk starts
//     at the leaf holding it: on the way up, the child it came from along that
//     path counts as the first-visited child (the split-plane bound is valid
//     for the other child whichever side the query lies on, since a point on
//     the wrong side can only lie on the plane);
//   * entering the other child also needs the squared distance from the
//     query to that child's bounding box to be at most the current k-th
//     distance (the subtree-box test of Appendix C; the plane test alone lets
//     a query beside a dense cluster walk every node of it), and a leaf is
//     scanned only when the same holds for the leaf's box;
//   * the walk's leaves are the grandparents of the tree's leaves: a walk
//     leaf box-tests and scans its four leaves in near-first order (leaf
//     boxes prune at least as tightly as the split planes they replace,
//     and a wave takes fewer, fuller rounds of walk and scan);
//   * a lane may walk one walk leaf ahead of its scans (see kd_search);
//   * leaf points are read as packed records (coordinates + row: one 16-byte
//     load for d <= 3), the next record is requested before the current one
//     is used;
//   * candidates go into a register-resident sorted k-list (KList, or
//     PackedList where ids fit beside the distance in 64 bits).
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

// Coordinates and the row word of leaf-order record i.  MD <= 3 and
// MD in 4..7 use compile-time record widths 4 and 8; MD == 8 reads a record
// of tv.rw words for the runtime dimension d.
template <typename T, int MD>
__device__ inline void load_point(const TreeView& tv, int64_t i, int d, T (&p)[MD], uint32_t& idw) {
    using M = Metric<T>;
    if constexpr (MD <= 3) {
        const uint4 r = reinterpret_cast<const uint4*>(tv.rec)[i];
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int c = 0; c < MD; c++) p[c] = M::load(w[c]);
        idw = w[MD];
    } else if constexpr (MD <= 7) {
        const uint4* b = reinterpret_cast<const uint4*>(tv.rec) + i * 2;
        const uint4 r0 = b[0], r1 = b[1];
        const uint32_t w[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
        for (int c = 0; c < MD; c++) p[c] = M::load(w[c]);
        idw = w[MD];
    } else {
        const uint32_t* r = tv.rec + i * tv.rw;
#pragma unroll
        for (int c = 0; c < MD; c++) p[c] = c < d ? M::load(r[c]) : T(0);
        idw = r[d];
    }
}

// Points of leaf-order position i: id and liveness.  kLazy: the id and the
// liveness cost loads of their own, so a point is measured first and they
// are read only for a point within the current k-th distance.
struct PlainIds {
    static constexpr bool kLazy = false;
    __device__ inline int32_t id(int64_t, uint32_t idw) const { return (int32_t)idw; }
    __device__ inline bool live(int64_t) const { return true; }
};

// Every point but the one at leaf-order position `self` (the query's own
// point, for the k-NN graph).
struct OtherIds {
    static constexpr bool kLazy = false;
    int64_t self;
    __device__ inline int32_t id(int64_t, uint32_t idw) const { return (int32_t)idw; }
    __device__ inline bool live(int64_t i) const { return i != self; }
};

// Offers leaf-order point i (coordinates p, row word idw) to the k-list.
template <typename T, int MD, typename List, typename Ids>
__device__ inline void visit_point(const Ids& ids, const T (&q)[MD], int d, List& kl, int k,
                                   uint32_t i, const T (&p)[MD], uint32_t idw) {
    using M = Metric<T>;
    if constexpr (Ids::kLazy) {
        typename M::D dd = 0;
#pragma unroll
        for (int c = 0; c < MD; c++)
            if (MD < 8 || c < d) dd = M::acc(dd, q[c], p[c]);
        if (!(dd > kl.kd) && ids.live(i)) kl.offer(dd, ids.id(i, idw), k);
    } else if (ids.live(i)) {
        typename M::D dd = 0;
#pragma unroll
        for (int c = 0; c < MD; c++)
            if (MD < 8 || c < d) dd = M::acc(dd, q[c], p[c]);
        kl.offer(dd, ids.id(i, idw), k);
    }
}

// Leaf j of a tree with n points at depth L that holds leaf-order position i.
__device__ inline uint32_t leaf_of(int64_t n, int L, int64_t i) {
    return (uint32_t)((((uint64_t)(i + 1) << L) - 1) / (uint64_t)n);
}

// The same with explicit leaf offsets: the last leaf j with loff[j] <= i.
__device__ inline uint32_t leaf_at(const int64_t* loff, int L, int64_t i) {
    uint32_t lo = 0, hi = 1u << L;  // loff[lo] <= i < loff[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (loff[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// k-NN walk of one query.  start: 0 = a separate query; otherwise the heap
// index of the leaf holding the query (all-points mode).  from (separate
// queries): a node of the query's own descent -- the root, or the node where
// the query ordering's descent stopped -- where the walk begins, as if
// entered from its parent: the nodes above it were entered on the query's
// side, so the climb treats them as any other.
//
// The walk (cur, entered from prev: its parent when prev < cur) hands leaves
// to a scan phase.  A lane holds up to two reached-but-unscanned leaves: all
// lanes walk while some lane has none, so a lane that reaches its leaf early
// walks on to its next one instead of idling (that step sees the k-th
// distance before the pending scan: it may enter more nodes, never fewer).
// Stepping into a leaf only records it; the walk then stands at the leaf's
// parent as if back from it.
// LOFF: leaf ranges come from tv.loff (trees grown in place).
// DUE (separate queries whose `from` is their walk leaf): bit l of `due` is
// clear when the split plane of the descent path's node at level l was
// beyond the k-th distance when the descent passed it.  That node can never
// send the walk into its other child (the distance only shrinks), so a walk
// leaving a path node upward goes straight to the deepest path ancestor
// whose bit is set, as if back from its child on the path, and ends when
// there is none: the same nodes are entered in the same order.
template <typename T, int MD, typename List, typename Ids, bool LOFF = false, bool DUE = false>
__device__ inline void kd_search(const TreeView& tv, const Ids& ids, const T (&q)[MD], int d,
                                 List& kl, int k, uint32_t start = 0, uint32_t from = 1,
                                 uint32_t due = ~0u) {
    using M = Metric<T>;
    using DT = typename M::D;
    const int64_t n = tv.n;
    if (n == 0) return;
    const int L = tv.L;
    // the walk stops two levels above the leaves: a walk leaf is the
    // grandparent of four leaves (the parent of two when L = 1, the root
    // leaf itself when L = 0)
    const int sub = L < 2 ? L : 2;
    const int W = L - sub;
    const uint32_t first_wleaf = 1u << W;
    const uint32_t first_leaf = 1u << L;
    const uint32_t wstart = start >> sub;
    // the descent path's walk leaf (DUE), 0 when `from` lies above it
    uint32_t pleaf = 0;
    if constexpr (DUE) {
        const int lf = 31 - __clz(from);
        pleaf = (start == 0 && W > 0 && lf >= W) ? from >> (lf - W) : 0u;
    }
    uint32_t cur, prev, p0, p1 = 0;
    if (W == 0) {
        p0 = 1;
        prev = 0;
        cur = 0;
    } else if (start != 0) {
        p0 = wstart;
        prev = wstart;
        cur = wstart >> 1;
    } else {
        // at or below the walk leaves: the walk leaf above `from` is the
        // first leaf pending, and the walk stands at its parent
        const int lv = 31 - __clz(from);
        if (lv >= W) {
            p0 = from >> (lv - W);
            prev = p0;
            cur = p0 >> 1;
        } else {
            p0 = 0;
            prev = from >> 1;
            cur = from;
        }
    }
    // split dimension of internal node h at level lvl (trees with offsets may
    // carry one per node)
    auto dim_of = [&](uint32_t h, int lvl) -> int {
        if constexpr (LOFF) {
            if (tv.sdim != nullptr) return tv.sdim[h];
        }
        return MD < 8 ? lvl % MD : lvl % d;
    };
    bool more;
    do {
        while (__ballot(p0 == 0 && cur != 0) != 0) {
            if (cur != 0 && p1 == 0) {
                const int lvl = 31 - __clz(cur);
                const T s = M::load(tv.split[cur]);
                const T qd = pick<MD>(q, dim_of(cur, lvl));
                const uint32_t nearc = 2u * cur + (qd >= s ? 1u : 0u);
                uint32_t next = nearc;
                uint32_t jprev = cur;  // prev after the step when it moves up
                if (prev > cur) {
                    // back from child prev: the other child is due when prev
                    // was entered first -- the start leaf's side on its path,
                    // the query's side elsewhere -- and is not out of reach
                    const bool prev_on_path = (wstart >> (W - lvl - 1)) == prev;
                    const bool cur_on_path = (wstart >> (W - lvl)) == cur;
                    const bool from_first = prev_on_path || (!cur_on_path && prev == nearc);
                    next = cur >> 1;
                    if (from_first && !(M::sq(qd, s) > kl.kd)) {
                        const uint32_t other = prev ^ 1u;
                        bool reach = true;
                        if (tv.nbox != nullptr) {
                            const uint32_t* nb = tv.nbox + (size_t)other * 2 * d;
                            DT lb = 0;
#pragma unroll
                            for (int c = 0; c < MD; c++)
                                if (MD < 8 || c < d)
                                    lb = M::acc_gap(lb, q[c], M::load(nb[c]), M::load(nb[d + c]));
                            reach = !(lb > kl.kd);
                        }
                        if (reach) next = other;
                    }
                    if constexpr (DUE) {
                        // leaving a path node upward: to the deepest path
                        // ancestor still due, or done
                        if (next == (cur >> 1) && pleaf != 0 && (pleaf >> (W - lvl)) == cur) {
                            const uint32_t m = due & ((1u << lvl) - 1u);
                            if (m == 0) {
                                next = 0;
                            } else {
                                const int la = 31 - __clz(m);
                                next = pleaf >> (W - la);
                                jprev = pleaf >> (W - la - 1);
                            }
                        }
                    }
                }
                if (next >= first_wleaf) {
                    if (p0 == 0) p0 = next;
                    else p1 = next;
                    prev = next;
                } else {
                    prev = jprev;
                    cur = next;
                }
            }
        }
        more = __ballot(p0 != 0) != 0;
        if (p0 != 0) {
            // the walk leaf's leaves, the query's side first at each of the
            // two levels; each is scanned when its box is within reach
            uint32_t c0 = p0, g0 = 0, g1 = 0;
            if (sub >= 1) {
                const T s = M::load(tv.split[p0]);
                const T qd = pick<MD>(q, dim_of(p0, W));
                c0 = 2u * p0 + (qd >= s ? 1u : 0u);
            }
            if (sub == 2) {
                const T qd0 = pick<MD>(q, dim_of(c0, W + 1));
                const T qd1 = pick<MD>(q, dim_of(c0 ^ 1u, W + 1));
                g0 = qd0 >= M::load(tv.split[c0]) ? 1u : 0u;
                g1 = qd1 >= M::load(tv.split[c0 ^ 1u]) ? 1u : 0u;
            }
            for (int t = 0; t < (1 << sub); t++) {
                uint32_t lh = c0 ^ (uint32_t)t;
                if (sub == 2) {
                    const uint32_t ch = (t >> 1) ? c0 ^ 1u : c0;
                    lh = 2u * ch + (((t >> 1) ? g1 : g0) ^ (uint32_t)(t & 1));
                }
                const uint32_t leaf = lh - first_leaf;
                const uint32_t* bb = tv.bbox + (size_t)leaf * 2 * d;
                DT lb = 0;
#pragma unroll
                for (int c = 0; c < MD; c++)
                    if (MD < 8 || c < d)
                        lb = M::acc_gap(lb, q[c], M::load(bb[c]), M::load(bb[d + c]));
                if (!(lb > kl.kd)) {
                    const uint32_t lo = LOFF ? (uint32_t)tv.loff[leaf] : (uint32_t)node_start(n, L, leaf);
                    const uint32_t hi = LOFF ? (uint32_t)tv.loff[leaf + 1]
                                             : (uint32_t)node_start(n, L, leaf + 1);
                    if (lo < hi) {
                        // two record registers, alternately loading and in
                        // use; positions past the leaf reread its last record
                        const uint32_t last = hi - 1;
                        T pa[MD], pb[MD];
                        uint32_t ia, ib;
                        load_point<T, MD>(tv, lo, d, pa, ia);
                        for (uint32_t i = lo; i < hi; i += 2) {
                            load_point<T, MD>(tv, i + 1 < last ? i + 1 : last, d, pb, ib);
                            visit_point(ids, q, d, kl, k, i, pa, ia);
                            load_point<T, MD>(tv, i + 2 < last ? i + 2 : last, d, pa, ia);
                            if (i + 1 < hi) visit_point(ids, q, d, kl, k, i + 1, pb, ib);
                        }
                    }
                }
            }
        }
        p0 = p1;
        p1 = 0;
    } while (more);
}

// Workgroup index for a grid whose size is a multiple of 8: consecutive
// workgroups are dealt round-robin to the 8 XCDs, so hand each XCD one
// contiguous eighth of the work (its L2 then holds one region of the tree).
__device__ inline int64_t xcd_block() {
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

inline unsigned grid_for_xcd(int64_t blocks) { return (unsigned)((blocks + 7) / 8 * 8); }

}  // namespace pg
