// Static kd-tree by spatial-median splits: the alternative to the object
// median that Section 6.3 measures (a node's space is cut in half along a
// dimension instead of at the median point).
//
// Readings (the paper gives the rule only in words): the space of the root
// is the bounding box of the points; node (l, j) cuts its cell at the cell's
// midpoint s along dimension l mod d (rule 0) or along the cell's widest side,
// the lowest dimension on ties (rule 1); its points with coordinate < s go
// left, the others right.  Midpoints: an int32 cell [lo, hi] is cut at
// floor((lo + hi + 1) / 2) into [lo, s - 1] and [s, hi]; a float32 cell at
// the float nearest (lo + hi) / 2 (sum in double) into [lo, s] and [s, hi].
// The tree keeps the object-median tree's depth L = min{L : ceil(n/2^L) <=
// leaf} and heap layout, so leaves hold varying numbers of points and their
// ranges are explicit offsets.
//
// Point-box form (rule bit 1): a node cuts the bounding box of its own
// points instead of its cell, with the same midpoint and side rules; a node
// without points takes split 0 and dimension l mod d (0 under the widest
// rule).
//
// GPU form: since every cut depends only on the cell, the leaf of a point
// follows from its own coordinates (L comparisons against midpoints computed
// on the fly), so the build is one pass for leaf keys, a counting sort by
// leaf and a scatter, instead of one partition pass per level.  A point box
// depends on the node's members, so that form goes level by level, but moves
// no points until the end: every point carries its node, each level reduces
// the nodes' boxes (LDS-private while the level's boxes fit, then global
// atomics), cuts them, and steps every point to its child.  The order of
// points inside a leaf is the order the counting sort's atomics give (leaf
// membership, splits and offsets are deterministic; results do not depend on
// the order inside a leaf).
#include "build.hpp"
#include "scan.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;

// Midpoint of cell [lo, hi] (coordinate values as doubles) and the cells of
// the two halves.
__device__ inline double cell_mid(double lo, double hi, bool fl) {
    if (!fl) {
        const int64_t t = (int64_t)lo + (int64_t)hi + 1;
        return (double)(t >= 0 ? t / 2 : -((-t + 1) / 2));
    }
    return (double)(float)(0.5 * (lo + hi));
}

__device__ inline double coord_value(uint32_t bits, bool fl) {
    return fl ? (double)__uint_as_float(bits) : (double)(int32_t)bits;
}

// Root cell: min / max key per dimension (box[c], box[d + c]).
__global__ void __launch_bounds__(kNT)
key_box_kernel(const uint32_t* __restrict__ keys, int64_t n, int d, uint32_t* __restrict__ box) {
    for (int c = 0; c < d; c++) {
        uint32_t mn = 0xffffffffu, mx = 0u;
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT) {
            const uint32_t k = keys[(int64_t)c * n + i];
            mn = k < mn ? k : mn;
            mx = k > mx ? k : mx;
        }
        mn = wave_min_u32(mn);
        mx = wave_max_u32(mx);
        if (lane_id() == 0) {
            atomicMin(&box[c], mn);
            atomicMax(&box[d + c], mx);
        }
    }
}

// Cell of the root from the key box, as coordinate values.
__device__ inline void root_cell(const uint32_t* box, int d, bool fl, double (&lo)[8], double (&hi)[8]) {
#pragma unroll
    for (int c = 0; c < 8; c++) {
        lo[c] = c < d ? coord_value(key_to_coord(box[c], fl), fl) : 0.0;
        hi[c] = c < d ? coord_value(key_to_coord(box[d + c], fl), fl) : 0.0;
    }
}

// Split dimension of a cell at level l: l mod d, or its widest side.
__device__ inline int cell_dim(const double (&lo)[8], const double (&hi)[8], int d, int l, int rule) {
    if (rule == 0) return l % d;
    int c = 0;
    double best = hi[0] - lo[0];
#pragma unroll
    for (int cc = 1; cc < 8; cc++) {
        if (cc < d && hi[cc] - lo[cc] > best) {
            best = hi[cc] - lo[cc];
            c = cc;
        }
    }
    return c;
}

// Halves cell dimension c (runtime) toward `right`; returns the cut.
__device__ inline double cut_cell(double (&lo)[8], double (&hi)[8], int c, bool right_of, bool fl,
                                  bool go_right) {
    double s = 0.0;
#pragma unroll
    for (int cc = 0; cc < 8; cc++) {
        if (cc == c) {
            s = cell_mid(lo[cc], hi[cc], fl);
            if (right_of) {
                if (go_right) lo[cc] = s;
                else hi[cc] = fl ? s : s - 1.0;
            }
        }
    }
    return s;
}

// Ranks of the points of one workgroup (one point per thread) among their
// leaves' points.  A leaf that holds one of kRankSlots LDS slots (tagged by
// leaf) counts locally and takes one global atomic per workgroup; its points
// get a local rank flagged by bit 31, finished by leaf_rank_fix_kernel from
// the base stored in bbase[block][slot].  Other points take a global rank
// directly.  A heavy leaf thus costs one global atomic per workgroup, not
// one per point.  Must be called by every thread of the workgroup.
constexpr int kRankSlots = 64;

__device__ inline void rank_in_leaf(bool valid, uint32_t j, int64_t i, uint32_t* __restrict__ rank,
                                    uint32_t* __restrict__ cnt, uint32_t* __restrict__ bbase) {
    __shared__ uint32_t tag[kRankSlots], lcnt[kRankSlots];
    if (threadIdx.x < kRankSlots) {
        tag[threadIdx.x] = 0xffffffffu;
        lcnt[threadIdx.x] = 0u;
    }
    __syncthreads();
    if (valid) {
        const int slot = (int)(j & (kRankSlots - 1));
        uint32_t held = tag[slot];
        if (held == 0xffffffffu) {
            const uint32_t prev = atomicCAS(&tag[slot], 0xffffffffu, j);
            held = prev == 0xffffffffu ? j : prev;
        }
        if (held == j) rank[i] = atomicAdd(&lcnt[slot], 1u) | 0x80000000u;
        else rank[i] = atomicAdd(&cnt[j], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kRankSlots) {
        const uint32_t t = tag[threadIdx.x];
        bbase[(int64_t)blockIdx.x * kRankSlots + threadIdx.x] =
            t != 0xffffffffu ? atomicAdd(&cnt[t], lcnt[threadIdx.x]) : 0u;
    }
}

// Local ranks (bit 31) plus their workgroup's base for the leaf.
__global__ void __launch_bounds__(kNT)
leaf_rank_fix_kernel(const uint32_t* __restrict__ leaf, int64_t n, const uint32_t* __restrict__ bbase,
                     uint32_t* __restrict__ rank) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    const uint32_t r = rank[i];
    if (r & 0x80000000u)
        rank[i] = bbase[(i / kNT) * kRankSlots + (leaf[i] & (kRankSlots - 1))] + (r & 0x7fffffffu);
}

// Leaf of every point (input order) and its rank among its leaf's points.
__global__ void __launch_bounds__(kNT)
spatial_leaf_kernel(const uint32_t* __restrict__ keys, int64_t n, int d, int L, int fl, int rule,
                    const uint32_t* __restrict__ box, uint32_t* __restrict__ leaf,
                    uint32_t* __restrict__ rank, uint32_t* __restrict__ cnt,
                    uint32_t* __restrict__ bbase) {
    const int64_t i0 = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const bool valid = i0 < n;
    const int64_t i = valid ? i0 : n - 1;  // an idle thread computes a real point's leaf
    double lo[8], hi[8], x[8];
    root_cell(box, d, fl != 0, lo, hi);
#pragma unroll
    for (int c = 0; c < 8; c++) x[c] = c < d ? coord_value(key_to_coord(keys[(int64_t)c * n + i], fl != 0), fl != 0) : 0.0;
    uint32_t j = 0;
    for (int l = 0; l < L; l++) {
        const int c = cell_dim(lo, hi, d, l, rule);
        double xc = x[0];
#pragma unroll
        for (int cc = 1; cc < 8; cc++) xc = cc == c ? x[cc] : xc;
        double s = 0.0;
#pragma unroll
        for (int cc = 0; cc < 8; cc++)
            if (cc == c) s = cell_mid(lo[cc], hi[cc], fl != 0);
        const bool right = xc >= s;
        cut_cell(lo, hi, c, true, fl != 0, right);
        j = 2u * j + (right ? 1u : 0u);
    }
    if (valid) leaf[i] = j;
    rank_in_leaf(valid, j, i, rank, cnt, bbase);
}

// Split (and dimension, when sdim is given) of internal node h: replay its
// path from the root, then cut.
__global__ void __launch_bounds__(kNT)
spatial_split_kernel(int d, int L, int fl, int rule, const uint32_t* __restrict__ box,
                     uint32_t* __restrict__ split, uint8_t* __restrict__ sdim) {
    const int64_t h = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (h >= ((int64_t)1 << L)) return;
    if (h == 0) {
        split[0] = 0u;
        if (sdim) sdim[0] = 0;
        return;
    }
    const int l = 63 - __builtin_clzll((unsigned long long)h);
    double lo[8], hi[8];
    root_cell(box, d, fl != 0, lo, hi);
    for (int t = 0; t < l; t++) {
        const bool right = ((h >> (l - 1 - t)) & 1) != 0;
        cut_cell(lo, hi, cell_dim(lo, hi, d, t, rule), true, fl != 0, right);
    }
    const int c = cell_dim(lo, hi, d, l, rule);
    const double s = cut_cell(lo, hi, c, false, fl != 0, false);
    split[h] = fl ? __float_as_uint((float)s) : (uint32_t)(int32_t)s;
    if (sdim) sdim[h] = (uint8_t)c;
}

// ---- point-box form ----

constexpr int kBoxSlots = 512;  // node boxes cached per workgroup (a power of two)

__global__ void pbox_fill_kernel(uint32_t* __restrict__ bmin, uint32_t* __restrict__ bmax, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < cnt) {
        bmin[i] = 0xffffffffu;
        bmax[i] = 0u;
    }
}

// Box (min / max key per dimension) of every node of the level, over the
// points' current nodes nid.  lds: reduce into 2 * J * d LDS words first.
__global__ void __launch_bounds__(kNT)
pbox_reduce_kernel(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ nid, int64_t n,
                   int d, int64_t J, int lds, uint32_t* __restrict__ bmin,
                   uint32_t* __restrict__ bmax) {
    extern __shared__ uint32_t sb[];
    const int64_t Jd = J * d;
    const int64_t stride = (int64_t)gridDim.x * kNT;
    if (lds) {
        for (int64_t t = threadIdx.x; t < Jd; t += kNT) {
            sb[t] = 0xffffffffu;
            sb[Jd + t] = 0u;
        }
        __syncthreads();
        if (J == 1) {  // one node: registers first, one LDS atomic per thread and dimension
            uint32_t mn[8], mx[8];
#pragma unroll
            for (int c = 0; c < 8; c++) {
                mn[c] = 0xffffffffu;
                mx[c] = 0u;
            }
            for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride) {
#pragma unroll
                for (int c = 0; c < 8; c++) {
                    if (c < d) {
                        const uint32_t k = keys[(int64_t)c * n + i];
                        mn[c] = k < mn[c] ? k : mn[c];
                        mx[c] = k > mx[c] ? k : mx[c];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 8; c++) {
                if (c < d) {
                    atomicMin(&sb[c], mn[c]);
                    atomicMax(&sb[Jd + c], mx[c]);
                }
            }
        } else {
            for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride) {
                const int64_t j = nid[i];
                for (int c = 0; c < d; c++) {
                    const uint32_t k = keys[(int64_t)c * n + i];
                    atomicMin(&sb[j * d + c], k);
                    atomicMax(&sb[Jd + j * d + c], k);
                }
            }
        }
        __syncthreads();
        for (int64_t t = threadIdx.x; t < Jd; t += kNT) {
            if (sb[t] <= sb[Jd + t]) {  // the node has points in this workgroup's share
                atomicMin(&bmin[t], sb[t]);
                atomicMax(&bmax[t], sb[Jd + t]);
            }
        }
        return;
    }
    // Many nodes: a direct-mapped LDS cache of node boxes (tag = node).  A
    // point whose node holds (or claims) its slot updates the slot; the
    // others go to global memory.  Heavy nodes, which would serialise their
    // global atomics, are the likeliest to hold a slot; each workgroup then
    // flushes its slots once.
    uint32_t* tag = sb;                   // [kBoxSlots]
    uint32_t* cmin = sb + kBoxSlots;      // [kBoxSlots][d]
    uint32_t* cmax = cmin + kBoxSlots * d;
    for (int t = threadIdx.x; t < kBoxSlots; t += kNT) tag[t] = 0xffffffffu;
    for (int t = threadIdx.x; t < kBoxSlots * d; t += kNT) {
        cmin[t] = 0xffffffffu;
        cmax[t] = 0u;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride) {
        const uint32_t j = nid[i];
        const int slot = (int)(j & (kBoxSlots - 1));
        uint32_t held = tag[slot];
        if (held == 0xffffffffu) {
            const uint32_t prev = atomicCAS(&tag[slot], 0xffffffffu, j);
            held = prev == 0xffffffffu ? j : prev;
        }
        if (held == j) {
            for (int c = 0; c < d; c++) {
                const uint32_t k = keys[(int64_t)c * n + i];
                atomicMin(&cmin[slot * d + c], k);
                atomicMax(&cmax[slot * d + c], k);
            }
        } else {
            for (int c = 0; c < d; c++) {
                const uint32_t k = keys[(int64_t)c * n + i];
                atomicMin(&bmin[(int64_t)j * d + c], k);
                atomicMax(&bmax[(int64_t)j * d + c], k);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kBoxSlots * d; t += kNT) {
        const uint32_t j = tag[t / d];
        if (j != 0xffffffffu && cmin[t] <= cmax[t]) {
            atomicMin(&bmin[(int64_t)j * d + t % d], cmin[t]);
            atomicMax(&bmax[(int64_t)j * d + t % d], cmax[t]);
        }
    }
}

// Split of every node of level l from its point box: dimension (l mod d, or
// the box's widest side, lowest on ties), cut at the box's midpoint.
__global__ void __launch_bounds__(kNT)
pbox_split_kernel(const uint32_t* __restrict__ bmin, const uint32_t* __restrict__ bmax, int64_t J,
                  int l, int d, int fl, int widest, uint32_t* __restrict__ split_level,
                  uint8_t* __restrict__ sdim_level, double* __restrict__ ns,
                  uint8_t* __restrict__ nd) {
    const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (j >= J) return;
    const bool empty = bmin[j * d] > bmax[j * d];
    int c = widest ? 0 : l % d;
    double s = 0.0;
    if (!empty) {
        double lo[8], hi[8];
#pragma unroll
        for (int cc = 0; cc < 8; cc++) {
            lo[cc] = cc < d ? coord_value(key_to_coord(bmin[j * d + cc], fl != 0), fl != 0) : 0.0;
            hi[cc] = cc < d ? coord_value(key_to_coord(bmax[j * d + cc], fl != 0), fl != 0) : 0.0;
        }
        c = cell_dim(lo, hi, d, l, widest);
#pragma unroll
        for (int cc = 0; cc < 8; cc++)
            if (cc == c) s = cell_mid(lo[cc], hi[cc], fl != 0);
    }
    split_level[j] = fl ? __float_as_uint((float)s) : (uint32_t)(int32_t)s;
    if (sdim_level) sdim_level[j] = (uint8_t)c;
    ns[j] = s;
    nd[j] = (uint8_t)c;
}

// Every point steps to the child of its node: right when its coordinate
// along the node's dimension is at least the cut.
__global__ void __launch_bounds__(kNT)
pbox_step_kernel(const uint32_t* __restrict__ keys, uint32_t* __restrict__ nid, int64_t n, int fl,
                 const double* __restrict__ ns, const uint8_t* __restrict__ nd) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = nid[i];
    const int c = nd[j];
    const double x = coord_value(key_to_coord(keys[(int64_t)c * n + i], fl != 0), fl != 0);
    nid[i] = 2u * j + (x >= ns[j] ? 1u : 0u);
}

// Rank of every point among its leaf's points (the node after L steps).
__global__ void __launch_bounds__(kNT)
pbox_rank_kernel(const uint32_t* __restrict__ nid, int64_t n, uint32_t* __restrict__ rank,
                 uint32_t* __restrict__ cnt, uint32_t* __restrict__ bbase) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const bool valid = i < n;
    rank_in_leaf(valid, valid ? nid[i] : 0u, i, rank, cnt, bbase);
}

__global__ void spatial_offsets_kernel(const uint32_t* __restrict__ start, int64_t leaves, int64_t n,
                                       int64_t* __restrict__ loff) {
    const int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (j < leaves) loff[j] = start[j];
    else if (j == leaves) loff[j] = n;
}

// Point i to position start[leaf] + rank: coordinate planes, records, rows.
__global__ void __launch_bounds__(kNT)
spatial_scatter_kernel(const uint32_t* __restrict__ keys, const int32_t* __restrict__ idx, int64_t n,
                       int d, int rw, int fl, const uint32_t* __restrict__ leaf,
                       const uint32_t* __restrict__ rank, const uint32_t* __restrict__ start,
                       uint32_t* __restrict__ pts, uint32_t* __restrict__ rec,
                       int32_t* __restrict__ pidx) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    const int64_t p = (int64_t)start[leaf[i]] + rank[i];
    for (int w = 0; w < rw; w++) {
        uint32_t v = 0;
        if (w < d) {
            v = key_to_coord(keys[(int64_t)w * n + i], fl != 0);
            pts[(int64_t)w * n + p] = v;
        } else if (w == d) {
            v = (uint32_t)idx[i];
        }
        rec[p * rw + w] = v;
    }
    pidx[p] = idx[i];
}

}  // namespace

pg_status build_tree_spatial(const void* points, int64_t n, int d, int leaf, int dtype, int rule,
                             hipStream_t s, pg_tree* T) {
    const bool fl = dtype == PG_FLOAT32;
    const int widest = rule & 1;            // split dimension: the widest side
    const bool point_box = (rule & 2) != 0;  // cut each node's point box
    T->n = n;
    T->d = d;
    T->leaf = leaf;
    T->dtype = dtype;
    T->stream = s;
    T->L = tree_levels(n, leaf);
    const int L = T->L;
    const int64_t leaves = (int64_t)1 << L;
    const int64_t nn = n > 0 ? n : 1;
    const int rw = record_words(d);
    PG_TRY(dalloc(&T->pts, (size_t)d * nn, s));
    PG_TRY(dalloc(&T->pidx, (size_t)nn + kTreePad, s));
    PG_TRY(dalloc(&T->split, (size_t)leaves, s));
    PG_TRY(dalloc(&T->nbox, (size_t)leaves * 2 * 2 * d, s));
    T->bbox = T->nbox + (size_t)leaves * 2 * d;
    PG_TRY(dalloc(&T->rec, ((size_t)nn + kTreePad) * rw, s));
    PG_TRY(dalloc(&T->loff, (size_t)leaves + 1, s));
    if (widest) PG_TRY(dalloc(&T->sdim, (size_t)leaves, s));
    if (n == 0) {
        if (T->sdim) PG_HIP(hipMemsetAsync(T->sdim, 0, leaves, s));
        PG_HIP(hipMemsetAsync(T->loff, 0, sizeof(int64_t) * (leaves + 1), s));
        PG_HIP(hipMemsetAsync(T->split, 0, sizeof(uint32_t) * leaves, s));
        return offset_boxes(T, s);
    }
    DevBuf keys(s), idx(s), box(s), lf(s), rk(s), cnt(s), start(s), bbase(s);
    PG_TRY(keys.alloc(sizeof(uint32_t) * (size_t)d * n));
    PG_TRY(idx.alloc(sizeof(int32_t) * (size_t)n));
    uint32_t vary[8] = {0}, keybase[8] = {0};
    PG_TRY(ingest_points(points, n, d, fl, keys.as<uint32_t>(), idx.as<int32_t>(), vary, keybase, s));
    PG_TRY(lf.alloc(sizeof(uint32_t) * n));
    PG_TRY(rk.alloc(sizeof(uint32_t) * n));
    PG_TRY(cnt.alloc(sizeof(uint32_t) * leaves));
    PG_TRY(start.alloc(sizeof(uint32_t) * leaves));
    PG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t) * leaves, s));
    PG_TRY(bbase.alloc(sizeof(uint32_t) * (size_t)cdiv(n, kNT) * kRankSlots));
    if (!point_box) {
        PG_TRY(box.alloc(sizeof(uint32_t) * 2 * d));
        PG_HIP(hipMemsetAsync(box.p, 0xff, sizeof(uint32_t) * d, s));
        PG_HIP(hipMemsetAsync(box.as<uint32_t>() + d, 0, sizeof(uint32_t) * d, s));
        const unsigned grid = cdiv(n, kNT) < 1024u ? cdiv(n, kNT) : 1024u;
        hipLaunchKernelGGL(key_box_kernel, dim3(grid), dim3(kNT), 0, s, keys.as<uint32_t>(), n, d,
                           box.as<uint32_t>());
        PG_LAUNCH_CHECK();
        hipLaunchKernelGGL(spatial_leaf_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s,
                           keys.as<uint32_t>(), n, d, L, fl ? 1 : 0, widest, box.as<uint32_t>(),
                           lf.as<uint32_t>(), rk.as<uint32_t>(), cnt.as<uint32_t>(),
                           bbase.as<uint32_t>());
        PG_LAUNCH_CHECK();
    } else {
        // every point starts at the root; the level loop writes every split
        // (and dimension) of nodes 1 .. 2^L - 1, node 0 is unused
        uint32_t* nid = lf.as<uint32_t>();
        PG_HIP(hipMemsetAsync(nid, 0, sizeof(uint32_t) * n, s));
        PG_HIP(hipMemsetAsync(T->split, 0, sizeof(uint32_t) * leaves, s));
        if (T->sdim) PG_HIP(hipMemsetAsync(T->sdim, 0, leaves, s));
        const int64_t jmax = L > 0 ? leaves / 2 : 1;
        DevBuf bmin(s), bmax(s), ns(s), nd(s);
        PG_TRY(bmin.alloc(sizeof(uint32_t) * jmax * d));
        PG_TRY(bmax.alloc(sizeof(uint32_t) * jmax * d));
        PG_TRY(ns.alloc(sizeof(double) * jmax));
        PG_TRY(nd.alloc(sizeof(uint8_t) * jmax));
        constexpr int64_t kLdsBoxWords = 4096;  // J * d of a level reduced in LDS (32 KB)
        for (int l = 0; l < L; l++) {
            const int64_t J = (int64_t)1 << l;
            const int64_t Jd = J * d;
            hipLaunchKernelGGL(pbox_fill_kernel, dim3(cdiv(Jd, kNT)), dim3(kNT), 0, s,
                               bmin.as<uint32_t>(), bmax.as<uint32_t>(), Jd);
            PG_LAUNCH_CHECK();
            const int lds = Jd <= kLdsBoxWords ? 1 : 0;
            const unsigned cap = lds ? 512u : 1024u;
            const unsigned grid = cdiv(n, kNT) < cap ? cdiv(n, kNT) : cap;
            const size_t lds_bytes = lds ? sizeof(uint32_t) * 2 * (size_t)Jd
                                         : sizeof(uint32_t) * (size_t)kBoxSlots * (1 + 2 * d);
            hipLaunchKernelGGL(pbox_reduce_kernel, dim3(grid), dim3(kNT), lds_bytes, s,
                               keys.as<uint32_t>(),
                               nid, n, d, J, lds, bmin.as<uint32_t>(), bmax.as<uint32_t>());
            PG_LAUNCH_CHECK();
            hipLaunchKernelGGL(pbox_split_kernel, dim3(cdiv(J, kNT)), dim3(kNT), 0, s,
                               bmin.as<uint32_t>(), bmax.as<uint32_t>(), J, l, d, fl ? 1 : 0, widest,
                               T->split + J, T->sdim ? T->sdim + J : nullptr, ns.as<double>(),
                               nd.as<uint8_t>());
            PG_LAUNCH_CHECK();
            hipLaunchKernelGGL(pbox_step_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s,
                               keys.as<uint32_t>(), nid, n, fl ? 1 : 0, ns.as<double>(),
                               nd.as<uint8_t>());
            PG_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(pbox_rank_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, nid, n,
                           rk.as<uint32_t>(), cnt.as<uint32_t>(), bbase.as<uint32_t>());
        PG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(leaf_rank_fix_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s, lf.as<uint32_t>(),
                       n, bbase.as<uint32_t>(), rk.as<uint32_t>());
    PG_LAUNCH_CHECK();
    PG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), start.as<uint32_t>(), leaves, nullptr, s));
    hipLaunchKernelGGL(spatial_offsets_kernel, dim3(cdiv(leaves + 1, kNT)), dim3(kNT), 0, s,
                       start.as<uint32_t>(), leaves, n, T->loff);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(spatial_scatter_kernel, dim3(cdiv(n, kNT)), dim3(kNT), 0, s,
                       keys.as<uint32_t>(), idx.as<int32_t>(), n, d, rw, fl ? 1 : 0,
                       lf.as<uint32_t>(), rk.as<uint32_t>(), start.as<uint32_t>(), T->pts, T->rec,
                       T->pidx);
    PG_LAUNCH_CHECK();
    if (!point_box) {
        hipLaunchKernelGGL(spatial_split_kernel, dim3(cdiv(leaves, kNT)), dim3(kNT), 0, s, d, L,
                           fl ? 1 : 0, widest, box.as<uint32_t>(), T->split, T->sdim);
        PG_LAUNCH_CHECK();
    }
    return offset_boxes(T, s);
}

}  // namespace pg
