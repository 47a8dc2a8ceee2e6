// BDL-tree: the batch-dynamic kd-tree of Section 5 (logarithmic method:
// a buffer tree of fewer than X points plus static trees i of capacity X 2^i),
// with batch insertion (Algorithm 3), batch deletion (Algorithms 2 and 4) and
// data-parallel k-NN over all trees with one k-list per query.
//
// GPU design:
//   * every tree (and the buffer) is an ordinary static tree (build.hip) plus
//     int64 point ids in leaf order and a liveness bitmask (tombstones);
//   * insert plans on the host from counts it already knows (no device
//     round-trip): F, buffer size, floor(|P|/X); gathers the live points of
//     destroyed trees in their staging order (scatter of liveness flags to
//     staging positions, prefix sum, gather), appends the tree-bound slice of
//     the batch, and builds each new tree;
//   * erase runs one lane per (erase point, tree), the points in the largest
//     tree's leaf order: a stack-free walk that
//     enters both children where the coordinate equals the split, and clears
//     the liveness bit of every live point with equal coordinates (atomic AND,
//     so duplicates count once); the per-tree counts come back in one read;
//   * k-NN walks the trees largest first with one register k-list per lane,
//     skipping tombstones.
#include <algorithm>
#include <new>
#include <vector>

#include "build.hpp"
#include "knn.hpp"
#include "scan.hpp"
#include "forest.hpp"
#include "xsearch.hpp"
#include "wave.hpp"

namespace pg {

struct BdlTree {
    pg_tree* t = nullptr;
    int64_t* ids = nullptr;     // [n] ids in leaf order
    uint32_t* alive = nullptr;  // [(n+31)/32] liveness bits
    int64_t live = 0;
    int64_t n() const { return t ? t->n : 0; }
};

namespace {

constexpr int kNT = 256;

// flags[pidx[i]] = liveness of leaf-order point i (staging order).
__global__ void stage_flags_kernel(const int32_t* __restrict__ pidx, const uint32_t* __restrict__ alive,
                                   int64_t n, uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < n) flags[pidx[i]] = (alive[i >> 5] >> (i & 31)) & 1u;
}

// Appends the live points of a tree in staging order: point i goes to row
// off + rank[pidx[i]] (rank == NULL: every point is live, rank = pidx).
__global__ void gather_live_kernel(TreeView tv, const int64_t* __restrict__ ids,
                                   const uint32_t* __restrict__ alive,
                                   const uint32_t* __restrict__ rank, int d,
                                   uint32_t* __restrict__ rows, int64_t* __restrict__ out_ids,
                                   int64_t off) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= tv.n) return;
    if (!((alive[i >> 5] >> (i & 31)) & 1u)) return;
    const int64_t st = tv.pidx[i];
    const int64_t r = off + (rank ? (int64_t)rank[st] : st);
    for (int c = 0; c < d; c++) rows[r * d + c] = tv.pts[(int64_t)c * tv.n + i];
    out_ids[r] = ids[i];
}

__global__ void iota64_kernel(int64_t* __restrict__ out, int64_t count, int64_t first) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < count) out[i] = first + i;
}

// Ids of the leaf-order points, also into the records' row words (low 32
// bits).
__global__ void leaf_ids_kernel(const int32_t* __restrict__ pidx, const int64_t* __restrict__ staged,
                                int64_t n, int64_t* __restrict__ ids, uint32_t* __restrict__ rec, int rw,
                                int d) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < n) {
        const int64_t v = staged[pidx[i]];
        ids[i] = v;
        rec[i * rw + d] = (uint32_t)v;
    }
}

// Erase: lane = erase point, blockIdx.y = tree slot.  Walks every node whose
// cell can hold the exact coordinates (both children where the coordinate
// equals the split) and clears live points with equal coordinates.  In an
// explicit-node tree (spatial-median splits: coordinate < split left, the
// rest right) that is the one path the point's descent takes.
template <typename T, int MD, int TK>
__global__ void __launch_bounds__(kNT)
erase_kernel(Forest f, const uint32_t* __restrict__ pts, const int32_t* __restrict__ order,
             int64_t m, int d, unsigned long long* __restrict__ erased) {
    using M = Metric<T>;
    const int64_t q0 = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const int slot = blockIdx.y;
    if (q0 >= m) return;
    // points taken in the largest tree's leaf order when an order is given:
    // neighbouring lanes then walk nearly the same nodes
    const int64_t qi = order ? (int64_t)order[q0] : q0;
    const ForestSlot& S = f.s[slot];
    const TreeView& tv = S.tv;
    if (tv.n == 0) return;
    T q[MD];
#pragma unroll
    for (int c = 0; c < MD; c++) q[c] = M::load(c < d ? pts[qi * d + c] : 0u);
    uint32_t hits = 0;
    // clears the live points of leaf-order range [lo, hi) equal to q when
    // the box bb holds q
    auto scan = [&](const uint32_t* bb, int64_t lo, int64_t hi) {
        bool inside = true;
#pragma unroll
        for (int c = 0; c < MD; c++)
            if (c < d) inside = inside && !(q[c] < M::load(bb[c])) && !(q[c] > M::load(bb[d + c]));
        if (!inside) return;
        for (int64_t i = lo; i < hi; i++) {
            T p[MD];
            uint32_t idw;
            load_point<T, MD>(tv, i, d, p, idw);
            bool eq = true;
#pragma unroll
            for (int c = 0; c < MD; c++)
                if (c < d) eq = eq && (p[c] == q[c]);
            if (eq) {
                const uint32_t bit = 1u << (i & 31);
                const uint32_t old = atomicAnd(&S.alive[i >> 5], ~bit);
                if (old & bit) hits++;
            }
        }
    };
    if constexpr (TK == kTreeX) {
        uint32_t cur = 0;
        uint4 r = tv.xn[0];
        while (!(r.w & kXLeaf)) {
            cur = r.y + (pick<MD>(q, (int)(r.w & 15u)) >= M::load(r.x) ? 1u : 0u);
            r = tv.xn[cur];
        }
        if (!(r.w & kXEmpty)) scan(tv.nbox + (size_t)cur * 2 * d, tv.loff[r.x], tv.loff[r.x + 1]);
    } else {
        const uint32_t first_leaf = 1u << tv.L;
        uint32_t cur = 1, prev = 0;
        int dim = 0;
        while (cur != 0) {
            while (cur != 0 && cur < first_leaf) {
                const T s = M::load(tv.split[cur]);
                const T qd = pick<MD>(q, dim);
                const uint32_t nearc = 2u * cur + (qd >= s ? 1u : 0u);
                uint32_t next;
                if (prev == (cur >> 1)) next = nearc;
                else if (prev == nearc && qd == s) next = nearc ^ 1u;
                else next = cur >> 1;
                if (next > cur) dim = (dim + 1 == d) ? 0 : dim + 1;
                else dim = (dim == 0) ? d - 1 : dim - 1;
                prev = cur;
                cur = next;
            }
            if (cur == 0) break;
            const uint32_t leaf = cur - first_leaf;
            scan(tv.bbox + (size_t)leaf * 2 * d,
                 TK == kTreeLoff ? tv.loff[leaf] : node_start(tv.n, tv.L, leaf),
                 TK == kTreeLoff ? tv.loff[leaf + 1] : node_start(tv.n, tv.L, leaf + 1));
            prev = cur;
            cur >>= 1;
            dim = (dim == 0) ? d - 1 : dim - 1;
        }
    }
    if (hits) atomicAdd(&erased[slot], (unsigned long long)hits);
}

template <typename T, int MD, int TK>
pg_status launch_erase(const Forest& f, const void* pts, const int32_t* order, int64_t m, int d,
                       unsigned long long* erased, hipStream_t s) {
    hipLaunchKernelGGL((erase_kernel<T, MD, TK>), dim3(cdiv(m, kNT), f.count), dim3(kNT), 0, s, f,
                       (const uint32_t*)pts, order, m, d, erased);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

template <typename T, int TK>
pg_status erase_d(const Forest& f, const void* pts, const int32_t* o, int64_t m, int d,
                  unsigned long long* e, hipStream_t s) {
    switch (d) {
        case 2: return launch_erase<T, 2, TK>(f, pts, o, m, d, e, s);
        case 3: return launch_erase<T, 3, TK>(f, pts, o, m, d, e, s);
        case 5: return launch_erase<T, 5, TK>(f, pts, o, m, d, e, s);
        default: return launch_erase<T, 8, TK>(f, pts, o, m, d, e, s);
    }
}

// The walk for the forest's tree kind (every tree of a forest is of one
// kind: explicit-node for spatial-median splits, heaps with leaf offsets for
// grown B2 trees, closed-form heaps otherwise).
template <typename T>
pg_status erase_any(int tk, const Forest& f, const void* pts, const int32_t* o, int64_t m, int d,
                    unsigned long long* e, hipStream_t s) {
    if (tk == kTreeX) return erase_d<T, kTreeX>(f, pts, o, m, d, e, s);
    if (tk == kTreeLoff) return erase_d<T, kTreeLoff>(f, pts, o, m, d, e, s);
    return erase_d<T, kTreeHeap>(f, pts, o, m, d, e, s);
}

// ---- B2 (Section 6.3's second baseline): one static tree whose splits stay
// fixed; inserted points join the leaf their descent reaches, erased points
// become tombstones.  Leaf ranges are explicit offsets from then on.

// Leaf of each new point (right at or above a split, as the search assumes)
// and its rank among the new points of that leaf.
__global__ void b2_leaf_kernel(TreeView tv, int fl, const uint32_t* __restrict__ pts, int64_t m,
                               uint32_t* __restrict__ leaf, uint32_t* __restrict__ rank,
                               uint32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= m) return;
    const int d = tv.d;
    uint32_t j;
    if (tv.xn) {
        j = tv.xn[fl ? xdescend<float>(tv, pts + i * d) : xdescend<int32_t>(tv, pts + i * d)].x;
    } else {
        const uint32_t first_leaf = 1u << tv.L;
        uint32_t cur = 1;
        int dim = 0;
        while (cur < first_leaf) {
            const uint32_t qb = pts[i * d + dim], sb = tv.split[cur];
            const bool right = fl ? __uint_as_float(qb) >= __uint_as_float(sb) : (int32_t)qb >= (int32_t)sb;
            cur = 2u * cur + (right ? 1u : 0u);
            dim = dim + 1 == d ? 0 : dim + 1;
        }
        j = cur - first_leaf;
    }
    leaf[i] = j;
    rank[i] = atomicAdd(&cnt[j], 1u);
}

// loff2[j] = loff[j] + (new points in leaves before j), j in [0, 2^L].
__global__ void b2_offsets_kernel(const int64_t* __restrict__ loff, const uint32_t* __restrict__ nstart,
                                  int64_t leaves, int64_t added, int64_t* __restrict__ loff2) {
    const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (j < leaves) loff2[j] = loff[j] + nstart[j];
    else if (j == leaves) loff2[j] = loff[j] + added;
}

// Old point at position p moves to p + (new points in leaves before its leaf).
__global__ void b2_move_kernel(TreeView tv, const int64_t* __restrict__ ids,
                               const uint32_t* __restrict__ alive, const uint32_t* __restrict__ nstart,
                               int64_t n2, uint32_t* __restrict__ pts2, uint32_t* __restrict__ rec2,
                               int32_t* __restrict__ pidx2, int64_t* __restrict__ ids2,
                               uint32_t* __restrict__ alive2) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= tv.n) return;
    // leaf of p: the last j with loff[j] <= p
    const int64_t p2 = p + nstart[leaf_at_n(tv.loff, tv.nleaves, p)];
    for (int c = 0; c < tv.d; c++) pts2[(int64_t)c * n2 + p2] = tv.pts[(int64_t)c * tv.n + p];
    for (int w = 0; w < tv.rw; w++) rec2[p2 * tv.rw + w] = tv.rec[p * tv.rw + w];
    pidx2[p2] = tv.pidx[p];
    ids2[p2] = ids[p];
    if ((alive[p >> 5] >> (p & 31)) & 1u) atomicOr(&alive2[p2 >> 5], 1u << (p2 & 31));
}

// New point i goes after its leaf's old points, at its rank.
__global__ void b2_place_kernel(TreeView tv, int fl, const uint32_t* __restrict__ pts, int64_t m,
                                const uint32_t* __restrict__ leaf, const uint32_t* __restrict__ rank,
                                const int64_t* __restrict__ loff2, int64_t first_id, int64_t n2,
                                uint32_t* __restrict__ pts2, uint32_t* __restrict__ rec2,
                                int32_t* __restrict__ pidx2, int64_t* __restrict__ ids2,
                                uint32_t* __restrict__ alive2) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= m) return;
    const uint32_t j = leaf[i];
    const int64_t p2 = loff2[j] + (tv.loff[j + 1] - tv.loff[j]) + rank[i];
    const int d = tv.d;
    for (int w = 0; w < tv.rw; w++) {
        uint32_t v = 0;
        if (w < d) {
            v = pts[i * d + w];
            if (fl && v == 0x80000000u) v = 0u;  // -0.0 is stored as +0.0
            pts2[(int64_t)w * n2 + p2] = v;
        }
        rec2[p2 * tv.rw + w] = v;
    }
    pidx2[p2] = 0;
    ids2[p2] = first_id + i;
    atomicOr(&alive2[p2 >> 5], 1u << (p2 & 31));
}

__global__ void closed_offsets_kernel(int64_t n, int L, int64_t* __restrict__ loff) {
    const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (j <= ((int64_t)1 << L)) loff[j] = node_start(n, L, j);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct Bdl {
    int d = 0, leaf = 0, dtype = 0;
    int split = 0;  // 0: object median; 1: spatial median (split dimension l mod d)
    int64_t X = 0;
    BdlTree tree[kMaxTrees];
    BdlTree buf;
    int64_t next_id = 0;

    uint64_t F() const {
        uint64_t f = 0;
        for (int i = 0; i < kMaxTrees; i++)
            if (tree[i].t) f |= 1ull << i;
        return f;
    }
};

static void free_tree(BdlTree& T) {
    if (T.t) {
        hipStream_t s = T.t->stream;
        dfree(T.ids, s);
        dfree(T.alive, s);
        pg_tree_free(T.t);
    }
    T = BdlTree();
}

// A contiguous set of staged points (rows [count][d] + ids), device memory.
struct Staged {
    uint32_t* rows = nullptr;
    int64_t* ids = nullptr;
    int64_t count = 0;
};

static pg_status append_live(const Bdl& B, const BdlTree& T, Staged& dst, int64_t off,
                             hipStream_t s) {
    if (!T.t || T.live == 0) return PG_OK;
    const int64_t n = T.t->n;
    DevBuf flags(s);
    const uint32_t* rank = nullptr;
    if (T.live != n) {
        PG_TRY(flags.alloc(sizeof(uint32_t) * n));
        hipLaunchKernelGGL(stage_flags_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, T.t->pidx,
                           T.alive, n, flags.as<uint32_t>());
        PG_LAUNCH_CHECK();
        PG_TRY(exclusive_scan_u32(flags.as<uint32_t>(), flags.as<uint32_t>(), n, nullptr, s));
        rank = flags.as<uint32_t>();
    }
    hipLaunchKernelGGL(gather_live_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, T.t->view(),
                       T.ids, T.alive, rank, B.d, dst.rows, dst.ids, off);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

static pg_status copy_slice(const Bdl& B, const Staged& src, int64_t from, int64_t count,
                            Staged& dst, int64_t off, hipStream_t s) {
    if (count <= 0) return PG_OK;
    PG_HIP(hipMemcpyAsync(dst.rows + off * B.d, src.rows + from * B.d,
                          sizeof(uint32_t) * B.d * count, hipMemcpyDeviceToDevice, s));
    PG_HIP(hipMemcpyAsync(dst.ids + off, src.ids + from, sizeof(int64_t) * count,
                          hipMemcpyDeviceToDevice, s));
    return PG_OK;
}

// Builds a BDL tree over staged points.
static pg_status build_bdl_tree(const Bdl& B, const Staged& S, hipStream_t s, BdlTree& out) {
    pg_tree* t = new (std::nothrow) pg_tree();
    if (!t) return fail(PG_ERR_NOMEM, "host allocation failed");
    pg_status st = B.split ? build_tree_spatial(S.rows, S.count, B.d, B.leaf, B.dtype, 0, s, t)
                           : build_tree(S.rows, S.count, B.d, B.leaf, B.dtype, s, t);
    if (st != PG_OK) {
        pg_tree_free(t);
        return st;
    }
    out.t = t;
    out.live = S.count;
    const int64_t n = S.count;
    const int64_t words = (n + 31) / 32;
    PG_TRY(dalloc(&out.ids, n > 0 ? n : 1, s));
    PG_TRY(dalloc(&out.alive, words > 0 ? words : 1, s));
    if (n > 0) {
        hipLaunchKernelGGL(leaf_ids_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, t->pidx, S.ids, n,
                           out.ids, t->rec, t->view().rw, B.d);
        PG_LAUNCH_CHECK();
        PG_HIP(hipMemsetAsync(out.alive, 0xff, sizeof(uint32_t) * words, s));
    }
    return PG_OK;
}

// Algorithm 3 on a staged batch (the batch's rows/ids stay the caller's).
static pg_status insert_core(Bdl& B, const Staged& S, hipStream_t s) {
    const int64_t X = B.X, m = S.count;
    const int64_t b = B.buf.live;
    const int64_t r = m % X;
    int64_t A = m / X;
    const bool overflow = b + r >= X;
    const int64_t n_fresh = overflow ? A * X + (X - b) : A * X;  // batch points bound for trees
    if (overflow) A++;
    const uint64_t F = B.F();
    const uint64_t Fnew = F + (uint64_t)A;
    const uint64_t nw = Fnew & ~F, destroyed = F & ~Fnew;
    for (int j = 0; j < 64; j++)
        if ((nw >> j) & 1ull) {
            if (j >= kMaxTrees || (X << j) >= ((int64_t)1 << 31))
                return fail(PG_ERR_UNSUPPORTED, "BDL-tree capacity exceeded (tree index or size)");
        }

    // Tree-bound points: the old buffer's live points first (on overflow), then
    // the first n_fresh batch points.
    Staged TB;
    DevBuf tb_rows(s), tb_ids(s);
    const int64_t tb_count = (overflow ? b : 0) + n_fresh;
    if (overflow && b > 0) {
        PG_TRY(tb_rows.alloc(sizeof(uint32_t) * B.d * tb_count));
        PG_TRY(tb_ids.alloc(sizeof(int64_t) * tb_count));
        TB.rows = tb_rows.as<uint32_t>();
        TB.ids = tb_ids.as<int64_t>();
        TB.count = tb_count;
        PG_TRY(append_live(B, B.buf, TB, 0, s));
        PG_TRY(copy_slice(B, S, 0, n_fresh, TB, b, s));
    } else {
        TB.rows = S.rows;
        TB.ids = S.ids;
        TB.count = n_fresh;
    }

    // New trees, ascending: destroyed trees assigned whole, then quota points.
    BdlTree built[kMaxTrees];
    int64_t pos = 0;
    for (int j = 0; j < kMaxTrees; j++) {
        if (!((nw >> j) & 1ull)) continue;
        int64_t assigned_cap = 0, assigned_live = 0;
        std::vector<int> from;
        for (int i = j - 1; i >= 0; i--) {
            if ((nw >> i) & 1ull) break;  // a lower new tree takes the rest
            if ((destroyed >> i) & 1ull) {
                from.push_back(i);
                assigned_cap += X << i;
                assigned_live += B.tree[i].live;
            }
        }
        std::sort(from.begin(), from.end());
        const int64_t quota = (X << j) - assigned_cap;
        Staged st;
        DevBuf rows(s), ids(s);
        st.count = assigned_live + quota;
        PG_TRY(rows.alloc(sizeof(uint32_t) * B.d * (st.count > 0 ? st.count : 1)));
        PG_TRY(ids.alloc(sizeof(int64_t) * (st.count > 0 ? st.count : 1)));
        st.rows = rows.as<uint32_t>();
        st.ids = ids.as<int64_t>();
        int64_t off = 0;
        for (int i : from) {
            PG_TRY(append_live(B, B.tree[i], st, off, s));
            off += B.tree[i].live;
        }
        PG_TRY(copy_slice(B, TB, pos, quota, st, off, s));
        pos += quota;
        PG_TRY(build_bdl_tree(B, st, s, built[j]));
    }
    if (pos != TB.count) return fail(PG_ERR_DEVICE, "BDL insert: internal count mismatch");

    // New buffer: (no overflow) old live buffer points + the last r batch
    // points; (overflow) the batch points after the tree-bound ones.
    const int64_t keep_old = overflow ? 0 : b;
    const int64_t from_batch = m - (overflow ? n_fresh : (m - r));
    Staged nb;
    DevBuf nb_rows(s), nb_ids(s);
    nb.count = keep_old + from_batch;
    const bool buffer_changes = overflow || from_batch > 0;
    BdlTree newbuf;
    if (buffer_changes) {
        PG_TRY(nb_rows.alloc(sizeof(uint32_t) * B.d * (nb.count > 0 ? nb.count : 1)));
        PG_TRY(nb_ids.alloc(sizeof(int64_t) * (nb.count > 0 ? nb.count : 1)));
        nb.rows = nb_rows.as<uint32_t>();
        nb.ids = nb_ids.as<int64_t>();
        if (keep_old) PG_TRY(append_live(B, B.buf, nb, 0, s));
        PG_TRY(copy_slice(B, S, m - from_batch, from_batch, nb, keep_old, s));
        if (nb.count > 0) PG_TRY(build_bdl_tree(B, nb, s, newbuf));
    }

    for (int i = 0; i < kMaxTrees; i++)
        if ((destroyed >> i) & 1ull) free_tree(B.tree[i]);
    for (int j = 0; j < kMaxTrees; j++)
        if ((nw >> j) & 1ull) B.tree[j] = built[j];
    if (buffer_changes) {
        free_tree(B.buf);
        B.buf = newbuf;
    }
    return PG_OK;
}

static Forest make_forest(const Bdl& B) {
    Forest f{};
    f.count = 0;
    for (int i = kMaxTrees - 1; i >= 0; i--)  // largest first
        if (B.tree[i].t) f.s[f.count++] = ForestSlot{B.tree[i].t->view(), B.tree[i].ids, B.tree[i].alive, 1};
    if (B.buf.t) f.s[f.count++] = ForestSlot{B.buf.t->view(), B.buf.ids, B.buf.alive, 1};
    return f;
}

// B2 baseline handle: the tree (with ids, liveness and explicit leaf
// offsets).
struct B2 {
    int d = 0, leaf = 0, dtype = 0;
    BdlTree T;
    int64_t next_id = 0;
};

static Forest b2_forest(const B2& B) {
    Forest f{};
    f.count = 0;
    if (B.T.t) f.s[f.count++] = ForestSlot{B.T.t->view(), B.T.ids, B.T.alive, 0};  // records move
    return f;
}

// Inserts m device rows into the leaves their descent reaches.
static pg_status b2_insert(B2& B, const void* points, int64_t m, hipStream_t s) {
    pg_tree* t = B.T.t;
    const int d = B.d;
    const int fl = B.dtype == PG_FLOAT32 ? 1 : 0;
    const int64_t n = t->n, n2 = n + m;
    if (n2 >= ((int64_t)1 << 31)) return fail(PG_ERR_UNSUPPORTED, "B2: more than 2^31 - 1 points");
    const int64_t leaves = t->view().nleaves;
    const int rw = record_words(d);
    const TreeView tv = t->view();
    DevBuf leaf(s), rank(s), cnt(s), nstart(s);
    PG_TRY(leaf.alloc(sizeof(uint32_t) * m));
    PG_TRY(rank.alloc(sizeof(uint32_t) * m));
    PG_TRY(cnt.alloc(sizeof(uint32_t) * leaves));
    PG_TRY(nstart.alloc(sizeof(uint32_t) * leaves));
    PG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t) * leaves, s));
    hipLaunchKernelGGL(b2_leaf_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, tv, fl,
                       (const uint32_t*)points, m, leaf.as<uint32_t>(), rank.as<uint32_t>(),
                       cnt.as<uint32_t>());
    PG_LAUNCH_CHECK();
    PG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), nstart.as<uint32_t>(), leaves, nullptr, s));
    uint32_t *pts2 = nullptr, *rec2 = nullptr, *alive2 = nullptr;
    int32_t* pidx2 = nullptr;
    int64_t *ids2 = nullptr, *loff2 = nullptr;
    const int64_t words = (n2 + 31) / 32;
    pg_status st = PG_OK;
    if ((st = dalloc(&pts2, (size_t)d * n2, s)) != PG_OK ||
        (st = dalloc(&rec2, ((size_t)n2 + kTreePad) * rw, s)) != PG_OK ||
        (st = dalloc(&pidx2, (size_t)n2 + kTreePad, s)) != PG_OK ||
        (st = dalloc(&ids2, (size_t)n2, s)) != PG_OK ||
        (st = dalloc(&alive2, (size_t)words, s)) != PG_OK ||
        (st = dalloc(&loff2, (size_t)leaves + 1, s)) != PG_OK) {
        dfree(pts2, s); dfree(rec2, s); dfree(pidx2, s); dfree(ids2, s); dfree(alive2, s); dfree(loff2, s);
        return st;
    }
    PG_HIP(hipMemsetAsync(alive2, 0, sizeof(uint32_t) * words, s));
    hipLaunchKernelGGL(b2_offsets_kernel, dim3(cdiv(leaves + 1, kNT)), dim3(kNT), 0, s, t->loff,
                       nstart.as<uint32_t>(), leaves, m, loff2);
    PG_LAUNCH_CHECK();
    if (n > 0) {
        hipLaunchKernelGGL(b2_move_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, tv, B.T.ids,
                           B.T.alive, nstart.as<uint32_t>(), n2, pts2, rec2, pidx2, ids2, alive2);
        PG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(b2_place_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, tv, fl,
                       (const uint32_t*)points, m, leaf.as<uint32_t>(), rank.as<uint32_t>(), loff2,
                       B.next_id, n2, pts2, rec2, pidx2, ids2, alive2);
    PG_LAUNCH_CHECK();
    // swap in the grown arrays
    dfree(t->pts, s); dfree(t->rec, s); dfree(t->pidx, s); dfree(B.T.ids, s); dfree(B.T.alive, s);
    dfree(t->loff, s);
    t->pts = pts2;
    t->rec = rec2;
    t->pidx = pidx2;
    t->n = n2;
    B.T.ids = ids2;
    B.T.alive = alive2;
    B.T.live += m;
    t->loff = loff2;
    return t->xn ? xtree_boxes(t, s) : offset_boxes(t, s);
}

// B1 baseline handle: one static tree over the live points, rebuilt whole
// after every batch.
struct B1 {
    Bdl shape;  // d, leaf, dtype
    BdlTree T;
    int64_t next_id = 0;
};

// Rebuilds B1's tree over its live points followed by `extra` (may be empty).
static pg_status b1_rebuild(B1& B, const Staged& extra, hipStream_t s) {
    const int64_t live = B.T.t ? B.T.live : 0;
    Staged S;
    DevBuf rows(s), ids(s);
    S.count = live + extra.count;
    PG_TRY(rows.alloc(sizeof(uint32_t) * B.shape.d * (S.count > 0 ? S.count : 1)));
    PG_TRY(ids.alloc(sizeof(int64_t) * (S.count > 0 ? S.count : 1)));
    S.rows = rows.as<uint32_t>();
    S.ids = ids.as<int64_t>();
    if (live > 0) PG_TRY(append_live(B.shape, B.T, S, 0, s));
    PG_TRY(copy_slice(B.shape, extra, 0, extra.count, S, live, s));
    BdlTree fresh;
    PG_TRY(build_bdl_tree(B.shape, S, s, fresh));
    free_tree(B.T);
    B.T = fresh;
    return PG_OK;
}

// Device memory a handle keeps between calls (grown, never shrunk) for the
// temporaries of its erase and k-NN calls: after a rebuild has freed and
// allocated large blocks, a fresh allocation can hold the host for
// milliseconds.  Calls on one handle must not overlap.
struct Workspace {
    void* p = nullptr;
    size_t cap = 0;
    hipStream_t s = nullptr;
    pg_status ensure(size_t bytes, hipStream_t st) {
        if (bytes <= cap) return PG_OK;
        release();
        const size_t want = bytes + bytes / 4;
        PG_TRY(dmalloc(&p, want, st));
        cap = want;
        s = st;
        return PG_OK;
    }
    void release() {
        if (p) dfree(p, s);
        p = nullptr;
        cap = 0;
    }
};

// Temporaries of one erase or k-NN call, carved from a Workspace.
struct CallWs {
    uint32_t* err = nullptr;              // range-check flag
    uint32_t* nredo = nullptr;            // redo count of the packed k-NN
    unsigned long long* cnt = nullptr;    // [kSlots] erase counts per tree
    int32_t* order = nullptr;             // [m] point order (null: unordered)
    QueryKeys keys;                       // where the ordering's descents ended
    int32_t* redo = nullptr;              // [m] redo list of the packed k-NN
};

inline size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Checks the m points' range and, when tv is given and m >= kOrderMin,
// orders them by tv's leaves; the erase counts start at zero.
static pg_status begin_call(Workspace& w, const TreeView* tv, const void* pts, int64_t m, int d,
                            bool fl, hipStream_t s, CallWs& c) {
    const bool ordered = tv && tv->n > 0 && m >= kOrderMin;
    const int64_t nb = ordered ? order_buckets(*tv, m) : 0;
    const size_t head = 512;  // err, nredo | cnt at 256
    const size_t o_order = head, o_work = o_order + (ordered ? up256(sizeof(int32_t) * m) : 0);
    const size_t o_sums = o_work + (ordered ? up256(sizeof(uint32_t) * (m + nb)) : 0);
    const size_t o_redo = o_sums + (ordered ? up256(sizeof(uint32_t) * scan_partials(nb)) : 0);
    PG_TRY(w.ensure(o_redo + up256(sizeof(int32_t) * m), s));
    uint8_t* b = static_cast<uint8_t*>(w.p);
    c.err = reinterpret_cast<uint32_t*>(b);
    c.nredo = reinterpret_cast<uint32_t*>(b + 4);
    c.cnt = reinterpret_cast<unsigned long long*>(b + 256);
    c.redo = reinterpret_cast<int32_t*>(b + o_redo);
    static_assert(sizeof(unsigned long long) * kSlots <= 256, "erase counts exceed their slot");
    PG_TRY(check_queries_ws(pts, m, d, fl, c.err, s));
    PG_TRY(fill_u32(reinterpret_cast<uint32_t*>(c.cnt), 2 * kSlots, 0u, s));
    c.order = nullptr;
    if (ordered) {
        c.order = reinterpret_cast<int32_t*>(b + o_order);
        PG_TRY(order_queries_ws(*tv, fl, pts, m, s, c.order, reinterpret_cast<uint32_t*>(b + o_work),
                                reinterpret_cast<uint32_t*>(b + o_sums), false, &c.keys));
    }
    return PG_OK;
}

}  // namespace pg

struct pg_bdl {
    pg::Bdl b;
    mutable pg::Workspace ws;
};

struct pg_b1 {
    pg::B1 b;
    mutable pg::Workspace ws;
};

struct pg_b2 {
    pg::B2 b;
    mutable pg::Workspace ws;
};

using namespace pg;

extern "C" {

static pg_status bdl_create(int32_t d, int32_t dtype, int32_t leaf, int64_t buffer_X, int split,
                            pg_bdl** out) {
    if (!out) return fail(PG_ERR_INVALID, "pg_bdl_create: out is NULL");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_bdl_create: d must be in [1, 8]");
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_bdl_create: leaf must be in [1, 64]");
    if (dtype != PG_INT32 && dtype != PG_FLOAT32) return fail(PG_ERR_INVALID, "pg_bdl_create: bad dtype");
    if (buffer_X < 1 || buffer_X >= ((int64_t)1 << 31))
        return fail(PG_ERR_INVALID, "pg_bdl_create: buffer_X must be in [1, 2^31)");
    pg_bdl* h = new (std::nothrow) pg_bdl();
    if (!h) return fail(PG_ERR_NOMEM, "pg_bdl_create: host allocation failed");
    h->b.d = d;
    h->b.dtype = dtype;
    h->b.leaf = leaf;
    h->b.X = buffer_X;
    h->b.split = split;
    *out = h;
    return PG_OK;
}

pg_status pg_bdl_create(int32_t d, int32_t dtype, int32_t leaf, int64_t buffer_X, pg_bdl** out) {
    return bdl_create(d, dtype, leaf, buffer_X, 0, out);
}

pg_status pg_bdl_create_spatial(int32_t d, int32_t dtype, int32_t leaf, int64_t buffer_X,
                                pg_bdl** out) {
    return bdl_create(d, dtype, leaf, buffer_X, 1, out);
}

pg_status pg_bdl_insert(pg_bdl* h, const void* points, int64_t m, void* stream, int64_t* first_id) {
    if (!h) return fail(PG_ERR_INVALID, "pg_bdl_insert: handle is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_bdl_insert: m must be in [0, 2^31)");
    if (m > 0 && !points) return fail(PG_ERR_INVALID, "pg_bdl_insert: points is NULL");
    Bdl& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    if (first_id) *first_id = B.next_id;
    if (m == 0) return PG_OK;
    PG_TRY(check_queries(points, m, B.d, B.dtype == PG_FLOAT32, s));
    DevBuf ids(s);
    PG_TRY(ids.alloc(sizeof(int64_t) * m));
    hipLaunchKernelGGL(iota64_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, ids.as<int64_t>(), m,
                       B.next_id);
    PG_LAUNCH_CHECK();
    Staged S;
    S.rows = (uint32_t*)points;
    S.ids = ids.as<int64_t>();
    S.count = m;
    PG_TRY(insert_core(B, S, s));
    B.next_id += m;
    return PG_OK;
}

pg_status pg_bdl_erase(pg_bdl* h, const void* points, int64_t m, void* stream, int64_t* n_erased) {
    if (!h) return fail(PG_ERR_INVALID, "pg_bdl_erase: handle is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_bdl_erase: m must be in [0, 2^31)");
    if (m > 0 && !points) return fail(PG_ERR_INVALID, "pg_bdl_erase: points is NULL");
    Bdl& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    if (n_erased) *n_erased = 0;
    if (m == 0) return PG_OK;
    Forest f = make_forest(B);
    CallWs c;
    PG_TRY(begin_call(h->ws, f.count > 0 ? &f.s[0].tv : nullptr, points, m, B.d, B.dtype == PG_FLOAT32, s, c));
    if (f.count == 0) return PG_OK;
    // slot -> tree index (-1: buffer), same order as make_forest
    int slot_tree[kSlots];
    {
        int c = 0;
        for (int i = kMaxTrees - 1; i >= 0; i--)
            if (B.tree[i].t) slot_tree[c++] = i;
        if (B.buf.t) slot_tree[c++] = -1;
    }
    unsigned long long* e = c.cnt;
    const int32_t* o = c.order;
    const int tk = B.split ? kTreeX : kTreeHeap;
    if (B.dtype == PG_FLOAT32) PG_TRY(erase_any<float>(tk, f, points, o, m, B.d, e, s));
    else PG_TRY(erase_any<int32_t>(tk, f, points, o, m, B.d, e, s));
    unsigned long long host[kSlots];
    PG_HIP(hipMemcpyAsync(host, e, sizeof(host), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    int64_t total = 0;
    for (int c = 0; c < f.count; c++) {
        BdlTree& T = slot_tree[c] < 0 ? B.buf : B.tree[slot_tree[c]];
        T.live -= (int64_t)host[c];
        total += (int64_t)host[c];
    }
    if (n_erased) *n_erased = total;

    // Trees below half capacity: gather their live points (ascending tree
    // index, each in staging order) into R, clear them, reinsert R.
    int64_t r_count = 0;
    std::vector<int> dep;
    for (int i = 0; i < kMaxTrees; i++)
        if (B.tree[i].t && 2 * B.tree[i].live < (B.X << i)) {
            dep.push_back(i);
            r_count += B.tree[i].live;
        }
    if (dep.empty()) return PG_OK;
    Staged R;
    DevBuf rrows(s), rids(s);
    PG_TRY(rrows.alloc(sizeof(uint32_t) * B.d * (r_count > 0 ? r_count : 1)));
    PG_TRY(rids.alloc(sizeof(int64_t) * (r_count > 0 ? r_count : 1)));
    R.rows = rrows.as<uint32_t>();
    R.ids = rids.as<int64_t>();
    R.count = r_count;
    int64_t off = 0;
    for (int i : dep) {
        PG_TRY(append_live(B, B.tree[i], R, off, s));
        off += B.tree[i].live;
    }
    for (int i : dep) free_tree(B.tree[i]);
    if (r_count > 0) PG_TRY(insert_core(B, R, s));
    return PG_OK;
}

pg_status pg_bdl_knn(const pg_bdl* h, const void* queries, int64_t m, int32_t k, int64_t* out_id,
                     void* out_dist, void* stream) {
    if (!h) return fail(PG_ERR_INVALID, "pg_bdl_knn: handle is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_bdl_knn: k must be in [1, 64]");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_bdl_knn: m must be in [0, 2^31)");
    if (m > 0 && (!queries || !out_id || !out_dist)) return fail(PG_ERR_INVALID, "pg_bdl_knn: NULL pointer");
    if (m == 0) return PG_OK;
    const Bdl& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    Forest f = make_forest(B);
    CallWs c;
    PG_TRY(begin_call(h->ws, f.count > 0 ? &f.s[0].tv : nullptr, queries, m, B.d, B.dtype == PG_FLOAT32, s, c));
    const int tk = B.split ? kTreeX : kTreeHeap;
    if (B.dtype == PG_FLOAT32)
        return forest_knn_float(tk, f, queries, c.order, c.keys, m, B.d, k, B.next_id, c.redo, c.nredo, out_id,
                                out_dist, s);
    return forest_knn_int(tk, f, queries, c.order, c.keys, m, B.d, k, B.next_id, c.redo, c.nredo, out_id, out_dist,
                          s);
}

int64_t pg_bdl_size(const pg_bdl* h) {
    if (!h) return -1;
    int64_t tot = h->b.buf.live;
    for (int i = 0; i < kMaxTrees; i++) tot += h->b.tree[i].live;
    return tot;
}

pg_status pg_bdl_stats(const pg_bdl* h, int64_t* tree_mask, int64_t* buffer_count,
                       int64_t* live_counts, int32_t max_trees) {
    if (!h) return fail(PG_ERR_INVALID, "pg_bdl_stats: handle is NULL");
    if (max_trees < 0) return fail(PG_ERR_INVALID, "pg_bdl_stats: max_trees < 0");
    if (tree_mask) *tree_mask = (int64_t)h->b.F();
    if (buffer_count) *buffer_count = h->b.buf.live;
    if (live_counts)
        for (int i = 0; i < max_trees; i++) live_counts[i] = i < kMaxTrees ? h->b.tree[i].live : 0;
    return PG_OK;
}

void pg_bdl_free(pg_bdl* h) {
    if (!h) return;
    for (int i = 0; i < kMaxTrees; i++) free_tree(h->b.tree[i]);
    free_tree(h->b.buf);
    h->ws.release();
    delete h;
}

static pg_status b1_create(int32_t d, int32_t dtype, int32_t leaf, int split, pg_b1** out) {
    if (!out) return fail(PG_ERR_INVALID, "pg_b1_create: out is NULL");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_b1_create: d must be in [1, 8]");
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_b1_create: leaf must be in [1, 64]");
    if (dtype != PG_INT32 && dtype != PG_FLOAT32) return fail(PG_ERR_INVALID, "pg_b1_create: bad dtype");
    pg_b1* h = new (std::nothrow) pg_b1();
    if (!h) return fail(PG_ERR_NOMEM, "pg_b1_create: host allocation failed");
    h->b.shape.d = d;
    h->b.shape.dtype = dtype;
    h->b.shape.leaf = leaf;
    h->b.shape.split = split;
    *out = h;
    return PG_OK;
}

pg_status pg_b1_create(int32_t d, int32_t dtype, int32_t leaf, pg_b1** out) {
    return b1_create(d, dtype, leaf, 0, out);
}

pg_status pg_b1_create_spatial(int32_t d, int32_t dtype, int32_t leaf, pg_b1** out) {
    return b1_create(d, dtype, leaf, 1, out);
}

pg_status pg_b1_insert(pg_b1* h, const void* points, int64_t m, void* stream, int64_t* first_id) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b1_insert: handle is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b1_insert: m must be in [0, 2^31)");
    if (m > 0 && !points) return fail(PG_ERR_INVALID, "pg_b1_insert: points is NULL");
    B1& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    if (first_id) *first_id = B.next_id;
    if (m == 0) return PG_OK;
    if ((B.T.t ? B.T.live : 0) + m >= ((int64_t)1 << 31))
        return fail(PG_ERR_UNSUPPORTED, "B1: more than 2^31 - 1 points");
    PG_TRY(check_queries(points, m, B.shape.d, B.shape.dtype == PG_FLOAT32, s));
    DevBuf ids(s);
    PG_TRY(ids.alloc(sizeof(int64_t) * m));
    hipLaunchKernelGGL(iota64_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, ids.as<int64_t>(), m,
                       B.next_id);
    PG_LAUNCH_CHECK();
    Staged S;
    S.rows = (uint32_t*)points;
    S.ids = ids.as<int64_t>();
    S.count = m;
    PG_TRY(b1_rebuild(B, S, s));
    B.next_id += m;
    return PG_OK;
}

pg_status pg_b1_erase(pg_b1* h, const void* points, int64_t m, void* stream, int64_t* n_erased) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b1_erase: handle is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b1_erase: m must be in [0, 2^31)");
    if (m > 0 && !points) return fail(PG_ERR_INVALID, "pg_b1_erase: points is NULL");
    B1& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    if (n_erased) *n_erased = 0;
    if (m == 0 || !B.T.t || B.T.t->n == 0) return PG_OK;
    Forest f{};
    f.count = 1;
    f.s[0] = ForestSlot{B.T.t->view(), B.T.ids, B.T.alive, 1};
    CallWs c;
    PG_TRY(begin_call(h->ws, &f.s[0].tv, points, m, B.shape.d, B.shape.dtype == PG_FLOAT32, s, c));
    const int32_t* o = c.order;
    unsigned long long* e = c.cnt;
    const int tk = B.shape.split ? kTreeX : kTreeHeap;
    if (B.shape.dtype == PG_FLOAT32) PG_TRY(erase_any<float>(tk, f, points, o, m, B.shape.d, e, s));
    else PG_TRY(erase_any<int32_t>(tk, f, points, o, m, B.shape.d, e, s));
    unsigned long long host = 0;
    PG_HIP(hipMemcpyAsync(&host, e, sizeof(host), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    B.T.live -= (int64_t)host;
    if (n_erased) *n_erased = (int64_t)host;
    if (host == 0) return PG_OK;
    Staged none;
    return b1_rebuild(B, none, s);
}

pg_status pg_b1_knn(const pg_b1* h, const void* queries, int64_t m, int32_t k, int64_t* out_id,
                    void* out_dist, void* stream) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b1_knn: handle is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_b1_knn: k must be in [1, 64]");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b1_knn: m must be in [0, 2^31)");
    if (m > 0 && (!queries || !out_id || !out_dist)) return fail(PG_ERR_INVALID, "pg_b1_knn: NULL pointer");
    if (m == 0) return PG_OK;
    const B1& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    Forest f{};
    f.count = 0;
    if (B.T.t) f.s[f.count++] = ForestSlot{B.T.t->view(), B.T.ids, B.T.alive, 1};
    CallWs c;
    PG_TRY(begin_call(h->ws, f.count > 0 ? &f.s[0].tv : nullptr, queries, m, B.shape.d,
                      B.shape.dtype == PG_FLOAT32, s, c));
    const int tk = B.shape.split ? kTreeX : kTreeHeap;
    if (B.shape.dtype == PG_FLOAT32)
        return forest_knn_float(tk, f, queries, c.order, c.keys, m, B.shape.d, k, B.next_id, c.redo, c.nredo, out_id,
                                out_dist, s);
    return forest_knn_int(tk, f, queries, c.order, c.keys, m, B.shape.d, k, B.next_id, c.redo, c.nredo, out_id,
                          out_dist, s);
}

int64_t pg_b1_size(const pg_b1* h) { return h ? (h->b.T.t ? h->b.T.live : 0) : -1; }

void pg_b1_free(pg_b1* h) {
    if (!h) return;
    free_tree(h->b.T);
    h->ws.release();
    delete h;
}

static pg_status b2_create(const void* points, int64_t n, int32_t d, int32_t leaf, int32_t dtype,
                           int split, void* stream, pg_b2** out) {
    if (!out) return fail(PG_ERR_INVALID, "pg_b2_create: out is NULL");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_b2_create: d must be in [1, 8]");
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_b2_create: leaf must be in [1, 64]");
    if (dtype != PG_INT32 && dtype != PG_FLOAT32) return fail(PG_ERR_INVALID, "pg_b2_create: bad dtype");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b2_create: n must be in [0, 2^31)");
    if (n > 0 && !points) return fail(PG_ERR_INVALID, "pg_b2_create: points is NULL");
    hipStream_t s = (hipStream_t)stream;
    pg_b2* h = new (std::nothrow) pg_b2();
    if (!h) return fail(PG_ERR_NOMEM, "pg_b2_create: host allocation failed");
    B2& B = h->b;
    B.d = d;
    B.leaf = leaf;
    B.dtype = dtype;
    Bdl shape;
    shape.d = d;
    shape.leaf = leaf;
    shape.dtype = dtype;
    shape.split = split;
    DevBuf ids(s);
    pg_status st = ids.alloc(sizeof(int64_t) * (n > 0 ? n : 1));
    if (st == PG_OK && n > 0) {
        hipLaunchKernelGGL(iota64_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, ids.as<int64_t>(), n,
                           (int64_t)0);
        if (hipGetLastError() != hipSuccess) st = fail(PG_ERR_DEVICE, "pg_b2_create: launch failed");
    }
    Staged S;
    S.rows = (uint32_t*)points;
    S.ids = ids.as<int64_t>();
    S.count = n;
    if (st == PG_OK) st = build_bdl_tree(shape, S, s, B.T);
    const int64_t leaves = B.T.t ? ((int64_t)1 << B.T.t->L) : 0;
    // a spatial-median tree comes with its leaf offsets
    const bool closed = st == PG_OK && B.T.t->xn == nullptr && B.T.t->loff == nullptr;
    if (closed) st = dalloc(&B.T.t->loff, (size_t)leaves + 1, s);
    if (closed && st == PG_OK) {
        hipLaunchKernelGGL(closed_offsets_kernel, dim3(cdiv(leaves + 1, kNT)), dim3(kNT), 0, s, n,
                           B.T.t->L, B.T.t->loff);
        if (hipGetLastError() != hipSuccess) st = fail(PG_ERR_DEVICE, "pg_b2_create: launch failed");
    }
    if (st != PG_OK) {
        free_tree(B.T);
        delete h;
        return st;
    }
    B.next_id = n;
    *out = h;
    return PG_OK;
}

pg_status pg_b2_create(const void* points, int64_t n, int32_t d, int32_t leaf, int32_t dtype,
                       void* stream, pg_b2** out) {
    return b2_create(points, n, d, leaf, dtype, 0, stream, out);
}

pg_status pg_b2_create_spatial(const void* points, int64_t n, int32_t d, int32_t leaf, int32_t dtype,
                               void* stream, pg_b2** out) {
    return b2_create(points, n, d, leaf, dtype, 1, stream, out);
}

pg_status pg_b2_insert(pg_b2* h, const void* points, int64_t m, void* stream, int64_t* first_id) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b2_insert: handle is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b2_insert: m must be in [0, 2^31)");
    if (m > 0 && !points) return fail(PG_ERR_INVALID, "pg_b2_insert: points is NULL");
    B2& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    if (first_id) *first_id = B.next_id;
    if (m == 0) return PG_OK;
    PG_TRY(check_queries(points, m, B.d, B.dtype == PG_FLOAT32, s));
    PG_TRY(b2_insert(B, points, m, s));
    B.next_id += m;
    return PG_OK;
}

pg_status pg_b2_erase(pg_b2* h, const void* points, int64_t m, void* stream, int64_t* n_erased) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b2_erase: handle is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b2_erase: m must be in [0, 2^31)");
    if (m > 0 && !points) return fail(PG_ERR_INVALID, "pg_b2_erase: points is NULL");
    B2& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    if (n_erased) *n_erased = 0;
    if (m == 0 || !B.T.t || B.T.t->n == 0) return PG_OK;
    Forest f = b2_forest(B);
    CallWs c;
    PG_TRY(begin_call(h->ws, &f.s[0].tv, points, m, B.d, B.dtype == PG_FLOAT32, s, c));
    const int32_t* o = c.order;
    unsigned long long* e = c.cnt;
    const int tk = B.T.t->xn ? kTreeX : kTreeLoff;
    if (B.dtype == PG_FLOAT32) PG_TRY(erase_any<float>(tk, f, points, o, m, B.d, e, s));
    else PG_TRY(erase_any<int32_t>(tk, f, points, o, m, B.d, e, s));
    unsigned long long host = 0;
    PG_HIP(hipMemcpyAsync(&host, e, sizeof(host), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    B.T.live -= (int64_t)host;
    if (n_erased) *n_erased = (int64_t)host;
    return PG_OK;
}

pg_status pg_b2_knn(const pg_b2* h, const void* queries, int64_t m, int32_t k, int64_t* out_id,
                    void* out_dist, void* stream) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b2_knn: handle is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_b2_knn: k must be in [1, 64]");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_b2_knn: m must be in [0, 2^31)");
    if (m > 0 && (!queries || !out_id || !out_dist)) return fail(PG_ERR_INVALID, "pg_b2_knn: NULL pointer");
    if (m == 0) return PG_OK;
    const B2& B = h->b;
    hipStream_t s = (hipStream_t)stream;
    Forest f = b2_forest(B);
    CallWs c;
    PG_TRY(begin_call(h->ws, f.count > 0 ? &f.s[0].tv : nullptr, queries, m, B.d, B.dtype == PG_FLOAT32, s, c));
    const int tk = B.T.t && B.T.t->xn ? kTreeX : kTreeLoff;
    if (B.dtype == PG_FLOAT32)
        return forest_knn_float(tk, f, queries, c.order, c.keys, m, B.d, k, B.next_id, c.redo, c.nredo, out_id,
                                out_dist, s);
    return forest_knn_int(tk, f, queries, c.order, c.keys, m, B.d, k, B.next_id, c.redo, c.nredo, out_id, out_dist,
                          s);
}

int64_t pg_b2_size(const pg_b2* h) { return h ? h->b.T.live : -1; }

pg_status pg_b2_stats(const pg_b2* h, int64_t* stored, int32_t* levels) {
    if (!h) return fail(PG_ERR_INVALID, "pg_b2_stats: handle is NULL");
    if (stored) *stored = h->b.T.n();
    if (levels) *levels = h->b.T.t ? h->b.T.t->L : 0;
    return PG_OK;
}

void pg_b2_free(pg_b2* h) {
    if (!h) return;
    free_tree(h->b.T);
    h->ws.release();
    delete h;
}

}  // extern "C"
