// Orthogonal range search over a static kd-tree: one query box per lane
// (the kd-tree range query of the paper's first module, timed in Table 1;
// queries are independent, as in Appendix C's data-parallel k-NN).
//
// Query: a closed axis-aligned box [lo, hi]; result: every point p with
// lo_c <= p_c <= hi_c in every dimension c (an empty box when lo_c > hi_c).
// Coordinates are compared as values, so -0.0 and +0.0 are equal.
//
// Traversal: depth-first over the implicit heap without a stack.  A node
// whose bounding box misses the query is skipped, a node whose box lies
// inside it reports its whole leaf-order range [floor(j n/2^l),
// floor((j+1) n/2^l)) without touching its points, and a leaf that the box
// cuts tests each of its points.  After a node is done the walk moves to the
// right sibling of its lowest left-child ancestor-or-self, found in one step
// by stripping the heap index's trailing one bits.
//
// A query is run twice: a counting pass, then (after a prefix sum of the
// counts) a pass that writes the input rows, in leaf order, from the query's
// offset on.
#include "range.hpp"
#include "knn.hpp"
#include "scan.hpp"
#include "search.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;

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

// REPORT = false: counts[i] = number of points in box i.
// REPORT = true:  rows of those points go to out_idx[offsets[i] ...]; a slot
// at or beyond `capacity` is not written and raises *overflow.
template <typename T, int MD, bool REPORT>
__global__ void __launch_bounds__(kNT)
range_kernel(TreeView tv, const uint32_t* __restrict__ boxes, const int32_t* __restrict__ order,
             int64_t m, int32_t* __restrict__ counts, const int64_t* __restrict__ offsets,
             int32_t* __restrict__ out_idx, int64_t capacity, uint32_t* __restrict__ overflow) {
    using M = Metric<T>;
    const int d = MD < 8 ? MD : tv.d;
    const int64_t i0 = xcd_block() * kNT + threadIdx.x;
    if (i0 >= m) return;
    const int64_t i = order ? (int64_t)order[i0] : i0;
    T lo[MD], hi[MD];
#pragma unroll
    for (int c = 0; c < MD; c++) {
        lo[c] = (MD < 8 || c < d) ? M::load(boxes[i * 2 * d + c]) : T(0);
        hi[c] = (MD < 8 || c < d) ? M::load(boxes[i * 2 * d + d + c]) : T(0);
    }
    const int64_t base = REPORT ? offsets[i] : 0;
    bool over = false;
    int64_t cnt = 0;
    const uint32_t first_leaf = 1u << tv.L;
    uint32_t h = 1;
    int l = 0;
    for (;;) {
        T bl[MD], bh[MD];
        load_node_box<T, MD>(tv, h, d, bl, bh);
        bool miss = false, inside = true;
#pragma unroll
        for (int c = 0; c < MD; c++) {
            if (MD < 8 || c < d) {
                miss = miss || bh[c] < lo[c] || bl[c] > hi[c];
                inside = inside && lo[c] <= bl[c] && bh[c] <= hi[c];
            }
        }
        if (!miss && !inside && h < first_leaf) {
            h = 2u * h;
            l++;
            continue;
        }
        if (!miss) {
            const int64_t j = (int64_t)h - ((int64_t)1 << l);
            const int64_t s = node_start(tv.n, l, j), e = node_start(tv.n, l, j + 1);
            if (inside) {
                if (REPORT) {
                    for (int64_t p = s; p < e; p++) {
                        const int64_t slot = base + cnt + (p - s);
                        if (slot < capacity) out_idx[slot] = tv.pidx[p];
                        else over = true;
                    }
                }
                cnt += e - s;
            } else {
                for (int64_t p = s; p < e; p++) {
                    T pt[MD];
                    uint32_t idw;
                    load_point<T, MD>(tv, p, d, pt, idw);
                    bool in = true;
#pragma unroll
                    for (int c = 0; c < MD; c++)
                        if (MD < 8 || c < d) in = in && lo[c] <= pt[c] && pt[c] <= hi[c];
                    if (in) {
                        if (REPORT) {
                            if (base + cnt < capacity) out_idx[base + cnt] = (int32_t)idw;
                            else over = true;
                        }
                        cnt++;
                    }
                }
            }
        }
        // done with h: climb while h is a right child, then step to the
        // right sibling (the rightmost path, all ones, ends the walk)
        if (~h == 0u) break;
        const int up = __builtin_ctz(~h);
        h >>= up;
        l -= up;
        if (h == 0u) break;
        h += 1u;
    }
    if (!REPORT) counts[i] = (int32_t)cnt;
    if (REPORT && over) atomicOr(overflow, 1u);
}

template <typename T, int MD>
pg_status launch_range(const pg_tree* t, const void* boxes, const int32_t* order, int64_t m,
                       int32_t* counts, const int64_t* offsets, int32_t* out_idx,
                       int64_t capacity, uint32_t* overflow, hipStream_t s) {
    const dim3 grid(grid_for_xcd(cdiv(m, kNT)));
    if (offsets)
        hipLaunchKernelGGL((range_kernel<T, MD, true>), grid, dim3(kNT), 0, s, t->view(),
                           (const uint32_t*)boxes, order, m, nullptr, offsets, out_idx, capacity,
                           overflow);
    else
        hipLaunchKernelGGL((range_kernel<T, MD, false>), grid, dim3(kNT), 0, s, t->view(),
                           (const uint32_t*)boxes, order, m, counts, nullptr, nullptr, 0,
                           nullptr);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

template <typename T>
pg_status dispatch_range(const pg_tree* t, const void* boxes, const int32_t* order, int64_t m,
                         int32_t* counts, const int64_t* offsets, int32_t* out_idx,
                         int64_t capacity, uint32_t* overflow, hipStream_t s) {
    switch (t->d) {
        case 2: return launch_range<T, 2>(t, boxes, order, m, counts, offsets, out_idx, capacity, overflow, s);
        case 3: return launch_range<T, 3>(t, boxes, order, m, counts, offsets, out_idx, capacity, overflow, s);
        case 5: return launch_range<T, 5>(t, boxes, order, m, counts, offsets, out_idx, capacity, overflow, s);
        default: return launch_range<T, 8>(t, boxes, order, m, counts, offsets, out_idx, capacity, overflow, s);
    }
}

pg_status range_pass(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                     const int64_t* offsets, int32_t* out_idx, int64_t capacity,
                     uint32_t* overflow, hipStream_t s) {
    DevBuf order(s);
    const int32_t* o = nullptr;
    if (m >= kOrderMin) {
        PG_TRY(order_queries(t->view(), t->dtype == PG_FLOAT32, boxes, m, s, order, true));
        o = order.as<int32_t>();
    }
    if (t->dtype == PG_FLOAT32)
        return dispatch_range<float>(t, boxes, o, m, counts, offsets, out_idx, capacity, overflow, s);
    return dispatch_range<int32_t>(t, boxes, o, m, counts, offsets, out_idx, capacity, overflow, s);
}

}  // namespace

pg_status range_count(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                      int64_t* offsets, int64_t* total_host, hipStream_t s) {
    if (m > 0) {
        if (t->n == 0) PG_HIP(hipMemsetAsync(counts, 0, sizeof(int32_t) * m, s));
        else PG_TRY(range_pass(t, boxes, m, counts, nullptr, nullptr, 0, nullptr, s));
    }
    if (offsets) {
        if (m > 0) PG_TRY(exclusive_scan_i32_i64(counts, offsets, m, offsets + m, s));
        else PG_HIP(hipMemsetAsync(offsets, 0, sizeof(int64_t), s));
    }
    if (total_host) {
        *total_host = 0;
        if (offsets) {
            PG_HIP(hipMemcpyAsync(total_host, offsets + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            PG_HIP(hipStreamSynchronize(s));
        } else if (m > 0) {
            DevBuf tmp(s);
            PG_TRY(tmp.alloc(sizeof(int64_t) * (m + 1)));
            PG_TRY(exclusive_scan_i32_i64(counts, tmp.as<int64_t>(), m, tmp.as<int64_t>() + m, s));
            PG_HIP(hipMemcpyAsync(total_host, tmp.as<int64_t>() + m, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s));
            PG_HIP(hipStreamSynchronize(s));
        }
    }
    return PG_OK;
}

pg_status range_report(const pg_tree* t, const void* boxes, int64_t m, const int64_t* offsets,
                       int32_t* out_idx, int64_t capacity, hipStream_t s) {
    if (m == 0 || t->n == 0) return PG_OK;
    DevBuf flag(s);
    PG_TRY(flag.alloc(sizeof(uint32_t)));
    PG_HIP(hipMemsetAsync(flag.p, 0, sizeof(uint32_t), s));
    PG_TRY(range_pass(t, boxes, m, nullptr, offsets, out_idx, capacity, flag.as<uint32_t>(), s));
    uint32_t h = 0;
    PG_HIP(hipMemcpyAsync(&h, flag.p, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h) return fail(PG_ERR_INVALID, "pg_range_report: a result slot lies at or beyond `capacity` (offsets do not match the counts)");
    return PG_OK;
}

}  // namespace pg
