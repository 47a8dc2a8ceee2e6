// Walks over explicit-node kd-trees (the spatial-median trees, which split
// until a node holds at most `leaf` points and so have no fixed depth).
//
// A node record is {split | leaf index, first child, parent, meta}; the
// children of a node are consecutive and numbered above it, so the walk keeps
// only (current, previous) node in registers and tells "came from the parent"
// from "came back from a child" by comparing the previous node with the
// parent field.  The meta word flags which children are leaves and which are
// empty, so a leaf is handed to the scan phase (or an empty one skipped)
// without visiting it.
//
// Semantics are those of kd_search (Appendix C, "Data-Parallel k-NN"): the
// child on the query's side first; the other child is entered unless the
// squared distance to the split plane, or to the child's bounding box,
// exceeds the current k-th distance (strict); a leaf is scanned when its box
// is within reach.  Points with coordinate < split lie in the first child,
// the others in the second, so a query that is a point of the tree lies on
// its leaf's side of every split above it.
#pragma once

#include "search.hpp"

namespace pg {

// Last leaf j in [0, count) with loff[j] <= i (the leaf holding leaf-order
// position i; empty leaves at i come before the leaf that starts there).
__device__ inline uint32_t leaf_at_n(const int64_t* loff, int64_t count, int64_t i) {
    uint32_t lo = 0, hi = (uint32_t)count;  // loff[lo] <= i < loff[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (loff[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Leaf node reached by a point with coordinate bits qb (dimension c at qb[c]):
// right at or above each split.
template <typename T>
__device__ inline uint32_t xdescend(const TreeView& tv, const uint32_t* qb) {
    using M = Metric<T>;
    uint32_t cur = 0;
    uint4 r = tv.xn[0];
    while (!(r.w & kXLeaf)) {
        const int dim = r.w & 15u;
        cur = r.y + (M::load(qb[dim]) >= M::load(r.x) ? 1u : 0u);
        r = tv.xn[cur];
    }
    return cur;
}

// Squared distance from q to the box of node u (min[d], max[d]).
template <typename T, int MD>
__device__ inline typename Metric<T>::D xnode_gap(const TreeView& tv, uint32_t u, const T (&q)[MD],
                                                  int d) {
    using M = Metric<T>;
    const uint32_t* nb = tv.nbox + (size_t)u * 2 * d;
    typename M::D lb = 0;
#pragma unroll
    for (int c = 0; c < MD; c++)
        if (MD < 8 || c < d) lb = M::acc_gap(lb, q[c], M::load(nb[c]), M::load(nb[d + c]));
    return lb;
}

// k-NN walk of one query over an explicit-node tree.  start: kXNone = a
// separate query; otherwise the leaf node holding the query (all-points mode:
// the walk scans it first and then climbs its path, where the child it came
// from counts as the one entered first).  from (separate queries): a node of
// the query's own descent (0: the root) where the walk begins, as if entered
// from its parent.
//
// As in kd_search a lane holds up to two reached-but-unscanned leaves, and
// all lanes walk while some lane has none.
template <typename T, int MD, typename List, typename Ids>
__device__ inline void kdx_search(const TreeView& tv, const Ids& ids, const T (&q)[MD], int d,
                                  List& kl, int k, uint32_t start = kXNone, uint32_t from = 0) {
    using M = Metric<T>;
    if (tv.n == 0) return;
    uint32_t cur, prev, pathc = kXNone, pathp = kXNone, p0 = kXNone, p1 = kXNone;
    if (start != kXNone) {
        p0 = start;
        prev = start;
        pathp = start;
        cur = tv.xn[start].z;
        pathc = cur;
    } else {
        const uint4 r = tv.xn[from];
        if (r.w & kXLeaf) {
            // the leaf pending (an empty one skipped), the walk at its parent
            p0 = (r.w & kXEmpty) ? kXNone : from;
            prev = from;
            cur = r.z;
        } else {
            cur = from;
            prev = r.z;
        }
    }
    bool more;
    do {
        while (__ballot(p0 == kXNone && cur != kXNone) != 0) {
            if (cur != kXNone && p1 == kXNone) {
                const uint4 r = tv.xn[cur];
                const T s = M::load(r.x);
                const T qd = pick<MD>(q, (int)(r.w & 15u));
                const uint32_t nearc = r.y + (qd >= s ? 1u : 0u);
                uint32_t next;
                if (prev == r.z) {
                    next = nearc;  // from the parent: the query's side first
                } else {
                    // back from child prev: the other child is due when prev
                    // was entered first and the other is within reach
                    const bool from_first = cur == pathc ? prev == pathp : prev == nearc;
                    next = r.z;
                    if (from_first && !(M::sq(qd, s) > kl.kd)) {
                        const uint32_t os = (prev - r.y) ^ 1u;
                        if (!(r.w & (kXChildEmpty << os)) &&
                            !(xnode_gap<T, MD>(tv, r.y + os, q, d) > kl.kd))
                            next = r.y + os;
                    }
                    if (next == r.z && cur == pathc) {
                        pathp = cur;
                        pathc = r.z;
                    }
                }
                if (next != r.z) {
                    const uint32_t cs = next - r.y;
                    if (r.w & (kXChildLeaf << cs)) {
                        // a leaf is only recorded (an empty one skipped); the
                        // walk stands at cur as if back from it
                        if (!(r.w & (kXChildEmpty << cs))) {
                            if (p0 == kXNone) p0 = next;
                            else p1 = next;
                        }
                        prev = next;
                    } else {
                        prev = cur;
                        cur = next;
                    }
                } else {
                    prev = cur;
                    cur = next;  // kXNone above the root: done
                }
            }
        }
        more = __ballot(p0 != kXNone) != 0;
        if (p0 != kXNone && !(xnode_gap<T, MD>(tv, p0, q, d) > kl.kd)) {
            const uint32_t j = tv.xn[p0].x;
            const uint32_t lo = (uint32_t)tv.loff[j], hi = (uint32_t)tv.loff[j + 1];
            if (lo < hi) {
                // two record registers, alternately loading and in use;
                // positions past the leaf reread its last record
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
        p0 = p1;
        p1 = kXNone;
    } while (more);
}

// Leaf node holding leaf-order position i of an explicit-node tree.
__device__ inline uint32_t xleaf_of(const TreeView& tv, int64_t i) {
    return tv.lnode[leaf_at_n(tv.loff, tv.nleaves, i)];
}

// Tree kinds the search kernels are instantiated for: implicit heaps with
// closed-form leaf ranges, implicit heaps with explicit leaf offsets (trees
// grown in place), and explicit-node trees.
constexpr int kTreeHeap = 0, kTreeLoff = 1, kTreeX = 2;

inline int tree_kind(const pg_tree* t) { return t->xn ? kTreeX : (t->loff ? kTreeLoff : kTreeHeap); }

// Where an all-points search of leaf-order point i starts (the leaf holding
// it), and the start of a search from the root.
template <int TK>
__device__ inline uint32_t search_start(const TreeView& tv, bool all, int64_t i) {
    if constexpr (TK == kTreeX) return all ? xleaf_of(tv, i) : kXNone;
    else if constexpr (TK == kTreeLoff) return all ? (1u << tv.L) + leaf_at(tv.loff, tv.L, i) : 0u;
    else return all ? (1u << tv.L) + leaf_of(tv.n, tv.L, i) : 0u;
}

// Where the walk of separate query i begins: the node its recorded descent
// reached (qk from the ordering by this same tree), else the root.
template <int TK>
__device__ inline uint32_t search_from(const TreeView& tv, const QueryKeys& qk, int64_t i) {
    if constexpr (TK == kTreeX) return (qk.key && qk.lev < 0) ? tv.lnode[qk.key[i]] : 0u;
    else return qk.key ? qk.key[i] + (1u << qk.lev) : 1u;
}

// The root as the start of a separate query's walk.
template <int TK>
__device__ inline uint32_t root_from() { return TK == kTreeX ? 0u : 1u; }

// Continues separate query q's descent from node `from` (the root, or where
// an earlier descent stopped) down to its walk leaf (heap trees: the level
// two above the leaves) or its leaf node (explicit trees), taking the
// query's side of every split as the walk does.  The walk may then begin
// there: its state is the one a walk from `from` would reach on the way
// down, and the descent, a plain loop of (for heap trees) uniform length,
// costs far fewer instructions than the same levels taken as walk steps.
template <typename T, int MD, int TK>
__device__ inline uint32_t descend_from(const TreeView& tv, const T (&q)[MD], int d, uint32_t from) {
    using M = Metric<T>;
    if (tv.n == 0) return from;
    if constexpr (TK == kTreeX) {
        uint32_t cur = from;
        uint4 r = tv.xn[cur];
        while (!(r.w & kXLeaf)) {
            cur = r.y + (pick<MD>(q, (int)(r.w & 15u)) >= M::load(r.x) ? 1u : 0u);
            r = tv.xn[cur];
        }
        return cur;
    } else {
        const int L = tv.L;
        const int W = L - (L < 2 ? L : 2);
        const int D = MD < 8 ? MD : d;
        int lv = 31 - __clz(from);
        uint32_t h = from;
        int dim = lv % D;
        for (; lv < W; lv++) {
            int dm = dim;
            if constexpr (TK == kTreeLoff) {
                if (tv.sdim != nullptr) dm = tv.sdim[h];
            }
            h = 2u * h + (pick<MD>(q, dm) >= M::load(tv.split[h]) ? 1u : 0u);
            dim = dim + 1 == D ? 0 : dim + 1;
        }
        return h;
    }
}

// descend_from from the root of a heap tree that also returns `due`: bit l
// set when the split plane of the path's node at level l is within kd of q
// (see kd_search).
template <typename T, int MD, int TK>
__device__ inline uint32_t descend_due(const TreeView& tv, const T (&q)[MD], int d,
                                       typename Metric<T>::D kd, uint32_t& due) {
    using M = Metric<T>;
    due = ~0u;
    if (tv.n == 0) return 1u;
    const int L = tv.L;
    const int W = L - (L < 2 ? L : 2);
    const int D = MD < 8 ? MD : d;
    uint32_t h = 1, bits = 0;
    int dim = 0;
    for (int lv = 0; lv < W; lv++) {
        int dm = dim;
        if constexpr (TK == kTreeLoff) {
            if (tv.sdim != nullptr) dm = tv.sdim[h];
        }
        const T qd = pick<MD>(q, dm);
        const T s = M::load(tv.split[h]);
        if (!(M::sq(qd, s) > kd)) bits |= 1u << lv;
        h = 2u * h + (qd >= s ? 1u : 0u);
        dim = dim + 1 == D ? 0 : dim + 1;
    }
    due = bits;
    return h;
}

// The k-NN walk for tree kind TK (start from search_start; from, for a
// separate query, from search_from or root_from).
template <typename T, int MD, typename List, typename Ids, int TK>
__device__ inline void tree_search(const TreeView& tv, const Ids& ids, const T (&q)[MD], int d,
                                   List& kl, int k, uint32_t start, uint32_t from = root_from<TK>()) {
    if constexpr (TK == kTreeX) kdx_search<T, MD, List, Ids>(tv, ids, q, d, kl, k, start, from);
    else kd_search<T, MD, List, Ids, TK == kTreeLoff>(tv, ids, q, d, kl, k, start, from);
}

// A separate query's walk of a tree other than the first of a forest: the
// descent with the current k-th distance, then the walk that skips the
// ancestors out of reach (heap trees; explicit trees walk from their root).
template <typename T, int MD, typename List, typename Ids, int TK>
__device__ inline void tree_search_next(const TreeView& tv, const Ids& ids, const T (&q)[MD], int d,
                                        List& kl, int k) {
    if constexpr (TK == kTreeX) {
        kdx_search<T, MD, List, Ids>(tv, ids, q, d, kl, k, kXNone, descend_from<T, MD, TK>(tv, q, d, 0u));
    } else {
        uint32_t due;
        const uint32_t from = descend_due<T, MD, TK>(tv, q, d, kl.kd, due);
        kd_search<T, MD, List, Ids, TK == kTreeLoff, true>(tv, ids, q, d, kl, k, 0u, from, due);
    }
}

}  // namespace pg
