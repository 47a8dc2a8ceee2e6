// Orthogonal range search over a static kd-tree: one query box per lane
// (the kd-tree range query of the paper's first module, timed in Table 1;
// queries are independent, as in Appendix C's data-parallel k-NN).
//
// Query: a closed axis-aligned box [lo, hi]; result: every point p with
// lo_c <= p_c <= hi_c in every dimension c (an empty box when lo_c > hi_c).
// Coordinates are compared as values, so -0.0 and +0.0 are equal.
//
// Traversal: depth-first over the implicit heap.  For one box: a node whose
// bounding box misses it is skipped, a node whose box lies inside it reports
// its whole leaf-order range (closed form floor(j n/2^l), or the leaf
// offsets of trees that have them) without touching its points, and a leaf
// that the box cuts tests each of its points.  The 64 boxes of a wave
// (neighbours in the tree's leaf order) share one walk over the union of the
// nodes they need (range_kernel).
//
// Two passes: counting, then (after a prefix sum of the counts) writing the
// input rows, in leaf order, from each box's offset.  pg_range_search keeps
// each box's first rows during the counting pass and only walks again the
// boxes that have more.
#include "range.hpp"
#include "knn.hpp"
#include "scan.hpp"
#include "xsearch.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;
// Boxes are taken in the tree's leaf order from this many on, so that the
// 64 boxes of a wave lie close together.
constexpr int64_t kRangeOrderMin = 256;

// Bounding box of heap node h (2d words: min[d], max[d]).
template <typename T, int MD>
__device__ inline void load_node_box(const TreeView& tv, uint32_t h, int d, T (&bl)[MD],
                                     T (&bh)[MD]) {
    using M = Metric<T>;
    if constexpr (MD == 2) {
        const uint4 r = reinterpret_cast<const uint4*>(tv.nbox)[h];
        bl[0] = M::load(r.x);
        bl[1] = M::load(r.y);
        bh[0] = M::load(r.z);
        bh[1] = M::load(r.w);
    } else if constexpr (MD == 3) {
        const uint2* b = reinterpret_cast<const uint2*>(tv.nbox) + (size_t)h * 3;
        const uint2 a0 = b[0], a1 = b[1], a2 = b[2];
        bl[0] = M::load(a0.x);
        bl[1] = M::load(a0.y);
        bl[2] = M::load(a1.x);
        bh[0] = M::load(a1.y);
        bh[1] = M::load(a2.x);
        bh[2] = M::load(a2.y);
    } else {
        const uint32_t* b = tv.nbox + (size_t)h * 2 * d;
#pragma unroll
        for (int c = 0; c < MD; c++) {
            bl[c] = (MD < 8 || c < d) ? M::load(b[c]) : T(0);
            bh[c] = (MD < 8 || c < d) ? M::load(b[d + c]) : T(0);
        }
    }
}

// Leaf-order position where node j of level l starts (explicit offsets when
// the tree has them, else the closed form).
__device__ inline int64_t node_begin(const TreeView& tv, int l, int64_t j) {
    return tv.loff ? tv.loff[j << (tv.L - l)] : node_start(tv.n, l, j);
}

// Walk modes of range_kernel, and the rows a box keeps in the stash.
constexpr int kCount = 0, kReport = 1, kStash = 2;
constexpr int kStashRows = 32;
// pg_range_search stashes rows for at most this many boxes (beyond, the
// reporting pass walks every box again).
constexpr int64_t kStashMaxBoxes = (int64_t)1 << 25;

// Leaf records and rows are read this many at a time.
constexpr int kGroup = kTreePad;

// A value that is the same in every lane, as a scalar (the builtin returns
// a signed int: widen without sign extension).
__device__ inline uint64_t scalar_u64(uint64_t w) {
    const uint32_t whi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(w >> 32));
    const uint32_t wlo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)w);
    return ((uint64_t)whi << 32) | wlo;
}

// Lane masks of the wave: boxes that miss node box [bl, bh] (disjoint) and
// boxes that contain it (and do not miss it: empty boxes only miss).
template <typename T, int MD>
__device__ inline void box_masks(const T (&bl)[MD], const T (&bh)[MD], const T (&lo)[MD],
                                 const T (&hi)[MD], int d, uint64_t& miss, uint64_t& inside) {
    miss = 0;
    inside = ~0ull;
#pragma unroll
    for (int c = 0; c < MD; c++) {
        if (MD < 8 || c < d) {
            miss |= __ballot(bh[c] < lo[c]) | __ballot(bl[c] > hi[c]);
            inside &= __ballot(lo[c] <= bl[c]) & __ballot(bh[c] <= hi[c]);
        }
    }
    inside &= ~miss;
}

// One box per lane, one walk per wave.  The wave enters an internal node
// when some lane's box cuts it (neither misses nor contains its bounding
// box); entering a node tests both children against every lane's box: a
// child inside a lane's box adds its whole leaf-order range to that lane, a
// cut leaf has its points tested, a cut internal child is entered (the left
// one first; the right sibling then waits, with the lanes that contain it,
// on a small per-wave stack of lane masks, one entry per level).  The node index, the masks and every tree
// load are the same across the wave: scalar loads and no divergence.
// kCount:  counts[i] = number of points in box i.
// kReport: rows of those points go to out_idx[offsets[i] ...]; a slot at or
//          beyond `capacity` is not written and raises *overflow.
// kStash:  counts as kCount, and the first kStashRows rows of the box walked
//          i0-th go to out_idx[i0 * kStashRows ...], with i0 in where[i] (a
//          later gather moves them; boxes with more rows are walked again by
//          kReport).
template <typename T, int MD, int MODE, bool XT>
__global__ void __launch_bounds__(kNT)
range_kernel(TreeView tv, const uint32_t* __restrict__ boxes, const int32_t* __restrict__ order,
             int64_t m, int32_t* __restrict__ counts, const int64_t* __restrict__ offsets,
             int32_t* __restrict__ out_idx, int64_t capacity, uint32_t* __restrict__ overflow,
             int32_t* __restrict__ where) {
    using M = Metric<T>;
    // per wave, by level: lanes that cut / contain a right child not yet visited
    __shared__ uint64_t pend[kNT / kWave][32][2];
    const int d = MD < 8 ? MD : tv.d;
    const int64_t i0 = xcd_block() * kNT + threadIdx.x;
    const bool valid = i0 < m;
    if (__ballot(valid) == 0) return;  // whole wave past the end
    uint64_t(*stk)[2] = pend[threadIdx.x / kWave];
    const uint64_t me = 1ull << lane_id();
    const int64_t i = valid ? (order ? (int64_t)order[i0] : i0) : 0;
    T lo[MD], hi[MD];
#pragma unroll
    for (int c = 0; c < MD; c++) {
        lo[c] = (valid && (MD < 8 || c < d)) ? M::load(boxes[i * 2 * d + c]) : T(0);
        hi[c] = (valid && (MD < 8 || c < d)) ? M::load(boxes[i * 2 * d + d + c]) : T(0);
    }
    constexpr bool WR = MODE != kCount;  // rows are written
    const int64_t base = !valid ? 0 : (MODE == kReport ? offsets[i] : (MODE == kStash ? i0 * kStashRows : 0));
    const int64_t limit = MODE == kReport ? capacity : base + kStashRows;
    bool over = false;
    int64_t cnt = 0;

    // every point of leaf-order range [s, e) is in the boxes of lanes `mask`
    auto take_range = [&](int64_t s, int64_t e, uint64_t mask) {
        if ((mask & me) == 0) return;
        if (WR) {
            // stashing stops at the box's kStashRows slots
            const int64_t pe = MODE == kStash ? min(e, s + max((int64_t)0, limit - base - cnt)) : e;
            for (int64_t p = s; p < pe; p += kGroup) {  // the row array is padded
                int32_t r[kGroup];
#pragma unroll
                for (int t = 0; t < kGroup; t++) r[t] = tv.pidx[p + t];
#pragma unroll
                for (int t = 0; t < kGroup; t++) {
                    const int64_t slot = base + cnt + (p - s) + t;
                    if (p + t < pe) {
                        if (slot < limit) out_idx[slot] = r[t];
                        else over = true;
                    }
                }
            }
        }
        cnt += e - s;
    };
    // test the points of leaf-order range [s, e) against the boxes of `mask`
    auto scan_leaf = [&](int64_t s, int64_t e, uint64_t mask) {
        const bool mine = (mask & me) != 0;
        for (int64_t p = s; p < e; p += kGroup) {  // the records are padded
            T pt[kGroup][MD];
            uint32_t idw[kGroup];
#pragma unroll
            for (int t = 0; t < kGroup; t++) load_point<T, MD>(tv, p + t, d, pt[t], idw[t]);
#pragma unroll
            for (int t = 0; t < kGroup; t++) {
                bool in = mine & (p + t < e);
#pragma unroll
                for (int c = 0; c < MD; c++)
                    if (MD < 8 || c < d) in = in & (lo[c] <= pt[t][c]) & (pt[t][c] <= hi[c]);
                if (in) {
                    if (WR) {
                        if (base + cnt < limit) out_idx[base + cnt] = (int32_t)idw[t];
                        else over = true;
                    }
                    cnt++;
                }
            }
        }
    };

    const uint64_t live = __ballot(valid);
    if constexpr (XT) {
        // Explicit-node tree: the same walk, stack-free.  Entering node h
        // (with act = the lanes whose box cuts it) tests its children in
        // order; back from a child, the lanes cutting h are recomputed from
        // h's box (node boxes nest, so they are the lanes active at h).
        auto range_of = [&](uint32_t u, int64_t& s0, int64_t& s1) {
            const uint2 sp = tv.xspan[u];
            s0 = tv.loff[sp.x];
            s1 = tv.loff[sp.y];
        };
        T bl[MD], bh[MD];
        load_node_box<T, MD>(tv, 0, d, bl, bh);
        uint64_t miss, inside;
        box_masks<T, MD>(bl, bh, lo, hi, d, miss, inside);
        const uint64_t take = live & inside;
        uint64_t act = live & ~miss & ~inside;
        if (take != 0) take_range(0, tv.n, take);
        uint4 r = tv.xn[0];
        if (r.w & kXLeaf) {
            if (act != 0) scan_leaf(0, tv.n, act);
            act = 0;
        }
        uint32_t h = 0, prev = kXNone;  // prev == parent: h was just entered
        while (act != 0 || h != 0 || prev != kXNone) {
            if (prev != r.z) {
                // back from child prev: the lanes cutting h
                load_node_box<T, MD>(tv, h, d, bl, bh);
                box_masks<T, MD>(bl, bh, lo, hi, d, miss, inside);
                act = live & ~miss & ~inside;
            }
            uint32_t side = prev == r.z ? 0u : prev - r.y + 1u;
            bool down = false;
            for (; side < 2u; side++) {
                const uint32_t c = r.y + side;
                load_node_box<T, MD>(tv, c, d, bl, bh);
                box_masks<T, MD>(bl, bh, lo, hi, d, miss, inside);
                const uint64_t tk = act & inside, ct = act & ~miss & ~inside;
                if ((tk | ct) == 0) continue;
                int64_t s0, s1;
                range_of(c, s0, s1);
                if (tk != 0) take_range(s0, s1, tk);
                if (ct != 0) {
                    if (r.w & (kXChildLeaf << side)) {
                        scan_leaf(s0, s1, ct);
                    } else {
                        prev = h;
                        h = c;
                        act = ct;
                        r = tv.xn[h];
                        down = true;
                        break;
                    }
                }
            }
            if (down) continue;
            if (r.z == kXNone) break;  // back at the root, both children done
            prev = h;
            h = r.z;
            r = tv.xn[h];
        }
    } else {
        uint64_t act;  // lanes whose box cuts the node the walk enters
        {
            T bl[MD], bh[MD];
            load_node_box<T, MD>(tv, 1, d, bl, bh);
            uint64_t miss, inside;
            box_masks<T, MD>(bl, bh, lo, hi, d, miss, inside);
            const uint64_t take = live & inside;
            act = live & ~miss & ~inside;
            if (take != 0) take_range(0, tv.n, take);
            if (tv.L == 0) {
                if (act != 0) scan_leaf(0, tv.n, act);
                act = 0;
            }
        }
        uint32_t h = 1;          // node entered (internal), level l
        int l = 0;
        uint32_t pending = 0;    // bit k: stk[k] holds the right child at level k+1
        while (act != 0) {
            T bl0[MD], bh0[MD], bl1[MD], bh1[MD];
            load_node_box<T, MD>(tv, 2u * h, d, bl0, bh0);
            load_node_box<T, MD>(tv, 2u * h + 1u, d, bl1, bh1);
            uint64_t miss0, in0, miss1, in1;
            box_masks<T, MD>(bl0, bh0, lo, hi, d, miss0, in0);
            box_masks<T, MD>(bl1, bh1, lo, hi, d, miss1, in1);
            const uint64_t take0 = act & in0, take1 = act & in1;
            const uint64_t cut0 = act & ~miss0 & ~in0, cut1 = act & ~miss1 & ~in1;
            // a lane's rows come out in leaf order: everything under the left
            // child before anything under the right one
            const int64_t j = 2 * ((int64_t)h - ((int64_t)1 << l));  // left child at level l+1
            if (l + 1 == tv.L) {
                if ((take0 | take1 | cut0 | cut1) != 0) {
                    const int64_t s0 = node_begin(tv, l + 1, j), s1 = node_begin(tv, l + 1, j + 1),
                                  s2 = node_begin(tv, l + 1, j + 2);
                    if (take0 != 0) take_range(s0, s1, take0);
                    if (cut0 != 0) scan_leaf(s0, s1, cut0);
                    if (take1 != 0) take_range(s1, s2, take1);
                    if (cut1 != 0) scan_leaf(s1, s2, cut1);
                }
                act = 0;
            } else {
                if (take0 != 0)
                    take_range(node_begin(tv, l + 1, j), node_begin(tv, l + 1, j + 1), take0);
                if (cut0 != 0) {
                    if ((cut1 | take1) != 0) {  // the right child waits (same value in every lane)
                        stk[l][0] = cut1;
                        stk[l][1] = take1;
                        pending |= 1u << l;
                    }
                    h = 2u * h;
                    l++;
                    act = cut0;
                    continue;
                }
                if (take1 != 0)
                    take_range(node_begin(tv, l + 1, j + 1), node_begin(tv, l + 1, j + 2), take1);
                if (cut1 != 0) {
                    h = 2u * h + 1u;
                    l++;
                    act = cut1;
                    continue;
                }
                act = 0;
            }
            // subtree done: the deepest waiting right child, its whole-range
            // lanes first; entered when some lane's box cuts it
            while (pending != 0) {
                const int k = 31 - __builtin_clz(pending);
                pending &= ~(1u << k);
                h = 2u * (h >> (l - k)) + 1u;
                l = k + 1;
                const uint64_t ct = scalar_u64(stk[k][0]), tk = scalar_u64(stk[k][1]);
                if (tk != 0) {
                    const int64_t jr = (int64_t)h - ((int64_t)1 << l);
                    take_range(node_begin(tv, l, jr), node_begin(tv, l, jr + 1), tk);
                }
                if (ct != 0) {
                    act = ct;
                    break;
                }
            }
        }
    }
    if (valid && MODE != kReport) counts[i] = (int32_t)cnt;
    if (valid && MODE == kStash) where[i] = (int32_t)i0;
    if (MODE == kReport && over) atomicOr(overflow, 1u);
}

template <typename T, int MD, bool XT>
pg_status launch_range_t(const pg_tree* t, const void* boxes, const int32_t* order, int64_t m,
                         int mode, int32_t* counts, const int64_t* offsets, int32_t* out_idx,
                         int64_t capacity, uint32_t* overflow, int32_t* where, hipStream_t s) {
    const dim3 grid(grid_for_xcd(cdiv(m, kNT)));
    if (mode == kReport)
        hipLaunchKernelGGL((range_kernel<T, MD, kReport, XT>), grid, dim3(kNT), 0, s, t->view(),
                           (const uint32_t*)boxes, order, m, nullptr, offsets, out_idx, capacity,
                           overflow, nullptr);
    else if (mode == kStash)
        hipLaunchKernelGGL((range_kernel<T, MD, kStash, XT>), grid, dim3(kNT), 0, s, t->view(),
                           (const uint32_t*)boxes, order, m, counts, nullptr, out_idx, 0, nullptr,
                           where);
    else
        hipLaunchKernelGGL((range_kernel<T, MD, kCount, XT>), grid, dim3(kNT), 0, s, t->view(),
                           (const uint32_t*)boxes, order, m, counts, nullptr, nullptr, 0,
                           nullptr, nullptr);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

template <typename T, int MD>
pg_status launch_range(const pg_tree* t, const void* boxes, const int32_t* order, int64_t m,
                       int mode, int32_t* counts, const int64_t* offsets, int32_t* out_idx,
                       int64_t capacity, uint32_t* overflow, int32_t* where, hipStream_t s) {
    if (t->xn)
        return launch_range_t<T, MD, true>(t, boxes, order, m, mode, counts, offsets, out_idx,
                                           capacity, overflow, where, s);
    return launch_range_t<T, MD, false>(t, boxes, order, m, mode, counts, offsets, out_idx, capacity,
                                        overflow, where, s);
}

template <typename T>
pg_status dispatch_range(const pg_tree* t, const void* boxes, const int32_t* order, int64_t m,
                         int mode, int32_t* counts, const int64_t* offsets, int32_t* out_idx,
                         int64_t capacity, uint32_t* overflow, int32_t* where, hipStream_t s) {
    switch (t->d) {
        case 2: return launch_range<T, 2>(t, boxes, order, m, mode, counts, offsets, out_idx, capacity, overflow, where, s);
        case 3: return launch_range<T, 3>(t, boxes, order, m, mode, counts, offsets, out_idx, capacity, overflow, where, s);
        case 5: return launch_range<T, 5>(t, boxes, order, m, mode, counts, offsets, out_idx, capacity, overflow, where, s);
        default: return launch_range<T, 8>(t, boxes, order, m, mode, counts, offsets, out_idx, capacity, overflow, where, s);
    }
}

// Stashed rows to their final slots, one thread per box in box order.  A
// wave's boxes own one contiguous stretch of the output, so when none of
// them was flagged the rows are staged in LDS and written out as whole
// 64-lane runs; stash rows are read 16 bytes at a time.  Boxes with more
// than kStashRows rows are flagged, by walking position, for the reporting
// pass (their waves write per lane and leave those boxes' slots alone).
__global__ void __launch_bounds__(kNT)
range_gather_kernel(int64_t m, const int32_t* __restrict__ counts,
                    const int64_t* __restrict__ offsets, const int32_t* __restrict__ where,
                    const int32_t* __restrict__ stash, int32_t* __restrict__ out_idx,
                    int64_t capacity, uint32_t* __restrict__ redo_flag,
                    uint32_t* __restrict__ overflow) {
    __shared__ int32_t stage[kNT / kWave][kWave * kStashRows];
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const bool valid = i < m;
    if (__ballot(valid) == 0) return;
    int32_t* st = stage[threadIdx.x / kWave];
    const int32_t c = valid ? counts[i] : 0;
    const int64_t i0 = valid ? where[i] : 0;
    const int64_t o = valid ? offsets[i] : 0;
    const bool redo = c > kStashRows;
    if (redo) redo_flag[i0] = 1u;
    const int lane = lane_id();
    bool over = false;
    if (__ballot(redo) == 0) {
        const int64_t w0 = __shfl(o, 0, kWave);
        const uint64_t live = __ballot(valid);
        const int last = 63 - __builtin_clzll(live);
        const int64_t w1 = __shfl(o + c, last, kWave);  // end of the wave's stretch
        const int rel = (int)(o - w0);
        const int4* src = reinterpret_cast<const int4*>(stash + i0 * kStashRows);
        for (int q = 0; q < (c + 3) / 4; q++) {
            const int4 v = src[q];
            const int r = rel + 4 * q;
            if (4 * q + 0 < c) st[r + 0] = v.x;
            if (4 * q + 1 < c) st[r + 1] = v.y;
            if (4 * q + 2 < c) st[r + 2] = v.z;
            if (4 * q + 3 < c) st[r + 3] = v.w;
        }
        wave_lds_sync();
        const int total = (int)(w1 - w0);
        for (int e = lane; e < total; e += kWave) {
            if (w0 + e < capacity) out_idx[w0 + e] = st[e];
            else over = true;
        }
    } else if (valid && !redo) {
        for (int t = 0; t < c; t++) {
            if (o + t < capacity) out_idx[o + t] = stash[i0 * kStashRows + t];
            else over = true;
        }
    }
    if (over) atomicOr(overflow, 1u);
}

// The flagged boxes, in walking order (pos: exclusive prefix sum of flags).
__global__ void range_redo_list_kernel(const int32_t* __restrict__ order, int64_t m,
                                       const uint32_t* __restrict__ flag,
                                       const uint32_t* __restrict__ pos, int32_t* __restrict__ redo) {
    const int64_t i0 = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i0 < m && flag[i0]) redo[pos[i0]] = order ? order[i0] : (int32_t)i0;
}

// The order in which the boxes are walked (the tree's leaf order of their
// centres), or none for few boxes.
pg_status range_order(const pg_tree* t, const void* boxes, int64_t m, hipStream_t s,
                      DevBuf& order, const int32_t** o) {
    *o = nullptr;
    if (m >= kRangeOrderMin) {
        PG_TRY(order_queries(t->view(), t->dtype == PG_FLOAT32, boxes, m, s, order, true));
        *o = order.as<int32_t>();
    }
    return PG_OK;
}

pg_status range_pass(const pg_tree* t, const void* boxes, const int32_t* o, int64_t m, int mode,
                     int32_t* counts, const int64_t* offsets, int32_t* out_idx, int64_t capacity,
                     uint32_t* overflow, hipStream_t s, int32_t* where = nullptr) {
    if (t->dtype == PG_FLOAT32)
        return dispatch_range<float>(t, boxes, o, m, mode, counts, offsets, out_idx, capacity, overflow, where, s);
    return dispatch_range<int32_t>(t, boxes, o, m, mode, counts, offsets, out_idx, capacity, overflow, where, s);
}

// Counting pass into counts (caller's), the prefix sum into offsets when
// given.
pg_status count_pass(const pg_tree* t, const void* boxes, const int32_t* o, int64_t m,
                     int32_t* counts, int64_t* offsets, hipStream_t s) {
    if (m > 0) {
        if (t->n == 0) PG_HIP(hipMemsetAsync(counts, 0, sizeof(int32_t) * m, s));
        else PG_TRY(range_pass(t, boxes, o, m, kCount, counts, nullptr, nullptr, 0, nullptr, s));
    }
    if (offsets) {
        if (m > 0) PG_TRY(exclusive_scan_i32_i64(counts, offsets, m, offsets + m, s));
        else PG_HIP(hipMemsetAsync(offsets, 0, sizeof(int64_t), s));
    }
    return PG_OK;
}

// Reporting pass; PG_ERR_INVALID when a slot at or beyond capacity was
// needed.  Synchronises.
pg_status report_pass(const pg_tree* t, const void* boxes, const int32_t* o, int64_t m,
                      const int64_t* offsets, int32_t* out_idx, int64_t capacity, hipStream_t s) {
    if (m == 0 || t->n == 0) return PG_OK;
    DevBuf flag(s);
    PG_TRY(flag.alloc(sizeof(uint32_t)));
    PG_HIP(hipMemsetAsync(flag.p, 0, sizeof(uint32_t), s));
    PG_TRY(range_pass(t, boxes, o, m, kReport, nullptr, offsets, out_idx, capacity,
                      flag.as<uint32_t>(), s));
    uint32_t h = 0;
    PG_HIP(hipMemcpyAsync(&h, flag.p, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h) return fail(PG_ERR_INVALID, "range report: a result slot lies at or beyond `capacity` (offsets do not match the counts)");
    return PG_OK;
}

}  // namespace

pg_status range_count(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                      int64_t* offsets, int64_t* total_host, hipStream_t s) {
    DevBuf order(s), tmp(s);
    const int32_t* o = nullptr;
    if (t->n > 0) PG_TRY(range_order(t, boxes, m, s, order, &o));
    int64_t* off = offsets;
    if (!off && total_host) {
        PG_TRY(tmp.alloc(sizeof(int64_t) * (m + 1)));
        off = tmp.as<int64_t>();
    }
    PG_TRY(count_pass(t, boxes, o, m, counts, off, s));
    if (total_host) {
        PG_HIP(hipMemcpyAsync(total_host, off + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    }
    return PG_OK;
}

pg_status range_report(const pg_tree* t, const void* boxes, int64_t m, const int64_t* offsets,
                       int32_t* out_idx, int64_t capacity, hipStream_t s) {
    if (m == 0 || t->n == 0) return PG_OK;
    DevBuf order(s);
    const int32_t* o = nullptr;
    PG_TRY(range_order(t, boxes, m, s, order, &o));
    return report_pass(t, boxes, o, m, offsets, out_idx, capacity, s);
}

pg_status range_search(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                       int64_t* offsets, int32_t* out_idx, int64_t capacity, int64_t* total_host,
                       hipStream_t s) {
    DevBuf order(s), work(s);
    const int32_t* o = nullptr;
    if (t->n > 0) PG_TRY(range_order(t, boxes, m, s, order, &o));
    // counting pass; with few enough boxes it also keeps each box's first
    // kStashRows rows, so the reporting pass only walks the boxes with more
    const bool stashing = t->n > 0 && m > 0 && m <= kStashMaxBoxes;
    // one temporary, carved: stash [m][kStashRows], counts (when the caller
    // gives none), where, flags, flag positions, redo list [m], and two words
    const size_t mm = (size_t)(m > 0 ? m : 1);
    const size_t stash_w = stashing ? mm * kStashRows : 0;
    PG_TRY(work.alloc(sizeof(int32_t) * (stash_w + (stashing ? 5 * mm : mm) + 2)));
    int32_t* stash = work.as<int32_t>();
    int32_t* cnts = stash + stash_w;
    if (!counts) counts = cnts;
    int32_t* where = cnts + mm;
    uint32_t* flag = (uint32_t*)(where + mm);
    uint32_t* pos = flag + mm;
    int32_t* redo = (int32_t*)(pos + mm);
    uint32_t* aux = stashing ? (uint32_t*)(redo + mm) : (uint32_t*)(cnts + mm);  // overflow, redo count
    if (stashing) {
        PG_TRY(range_pass(t, boxes, o, m, kStash, counts, nullptr, stash, 0, nullptr, s, where));
        PG_TRY(exclusive_scan_i32_i64(counts, offsets, m, offsets + m, s));
    } else {
        PG_TRY(count_pass(t, boxes, o, m, counts, offsets, s));
    }
    int64_t total = 0;
    PG_HIP(hipMemcpyAsync(&total, offsets + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (total_host) *total_host = total;
    if (total > capacity)
        return fail(PG_ERR_INVALID, "pg_range_search: " + std::to_string(total) +
                                        " results exceed capacity " + std::to_string(capacity) +
                                        " (counts, offsets and the total are written)");
    if (!stashing) return report_pass(t, boxes, o, m, offsets, out_idx, capacity, s);
    uint32_t* over = aux;
    uint32_t* nredo = aux + 1;
    PG_HIP(hipMemsetAsync(aux, 0, sizeof(uint32_t) * 2, s));
    PG_HIP(hipMemsetAsync(flag, 0, sizeof(uint32_t) * m, s));
    hipLaunchKernelGGL(range_gather_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, m, counts, offsets,
                       where, stash, out_idx, capacity, flag, over);
    PG_LAUNCH_CHECK();
    PG_TRY(exclusive_scan_u32(flag, pos, m, nredo, s));
    uint32_t h[2] = {0, 0};
    PG_HIP(hipMemcpyAsync(h, aux, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h[1] > 0) {
        hipLaunchKernelGGL(range_redo_list_kernel, dim3(cdiv(m, kNT)), dim3(kNT), 0, s, o, m, flag,
                           pos, redo);
        PG_LAUNCH_CHECK();
        PG_TRY(range_pass(t, boxes, redo, h[1], kReport, nullptr, offsets, out_idx, capacity, over, s));
        PG_HIP(hipMemcpyAsync(h, aux, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    }
    if (h[0]) return fail(PG_ERR_INVALID, "pg_range_search: a result slot lies at or beyond `capacity`");
    return PG_OK;
}

}  // namespace pg
