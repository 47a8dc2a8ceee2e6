// Static kd-tree by spatial-median splits: the alternative to the object
// median that Section 6.3 measures (a node's space is cut in half along a
// dimension instead of at the median point), split, as Section 5 defines a
// kd-tree, until a node holds a small constant number of points.
//
// Readings (the paper gives the rule only in words):
//  * a node holding at most `leaf` points, or only identical points (no cut
//    separates them), is a leaf;
//  * the root's space is the bounding box of the points; a node cuts its cell
//    (rule bit 1 clear) or the bounding box of its own points (bit 1 set);
//  * the cut dimension is depth mod d (rule bit 0 clear) or the space's
//    widest side hi - lo, the lowest dimension on ties (bit 0 set);
//  * spaces are closed intervals [lo, hi] of representable coordinates, and
//    the cut s of [lo, hi] with lo < hi lies in (lo, hi]: int32
//    floor((lo + hi + 1) / 2); float32 the float nearest (lo + hi) / 2 (sum
//    and halving in double), or the next float above lo when that nearest
//    float is lo itself; s = lo when lo == hi;
//  * points with coordinate < s go to the first child (cell [lo, s-], s- the
//    value just below s), the others to the second (cell [s, hi]), each side
//    keeping the parent's order.
// Nodes are numbered breadth-first: the root is 0, a level's nodes in leaf
// order, the children of a node consecutive.
//
// GPU form: level-synchronous over the nodes that still split.  The points
// of every node are one contiguous segment of a key-plane buffer; each level
// cuts the splitting nodes' segments into 256-point chunks (one wave each),
// counts the points going left per chunk, scans the counts, and partitions
// stably into the other buffer -- or, for a child that is already a leaf by
// its count, straight into the tree's leaf-order arrays.  The same pass
// reduces each child's bounding box (a wave-wide min/max, one atomic per
// chunk, child and bound), which gives the next level its point boxes, its
// identical-point test and the search its node boxes.  A child holding only
// identical points but more than `leaf` of them is copied to the leaf-order
// arrays by the next level's pass.  Points of finished nodes are never
// touched again.  Afterwards, level by level, subtree leaf counts (bottom-up)
// give every leaf its index in leaf order (top-down).
#include <algorithm>
#include <utility>
#include <vector>

#include "build.hpp"
#include "scan.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;
constexpr int kCH = 256;                 // points per chunk: one wave, four per lane
constexpr int kChunkGroups = kCH / kWave;
constexpr uint32_t kCopy = 1u << 8;      // entry mode bit: copy the segment (identical points)
constexpr uint64_t kFlagSplit = 1ull;
constexpr uint64_t kFlagCopy = 1ull << 32;

__device__ inline double coord_value(uint32_t bits, bool fl) {
    return fl ? (double)__uint_as_float(bits) : (double)(int32_t)bits;
}

// Coordinate bits of value v (representable as the coordinate type).
__device__ inline uint32_t value_bits(double v, bool fl) {
    return fl ? __float_as_uint((float)v) : (uint32_t)(int32_t)v;
}

// The next float above / below x (both zeros step to the smallest denormal).
__device__ inline float next_up(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) == 0) return __uint_as_float(1u);
    return __uint_as_float((b & 0x80000000u) ? b - 1u : b + 1u);
}
__device__ inline float next_down(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) == 0) return __uint_as_float(0x80000001u);
    return __uint_as_float((b & 0x80000000u) ? b + 1u : b - 1u);
}

// The cut of [lo, hi].
__device__ inline double space_cut(double lo, double hi, bool fl) {
    if (!(lo < hi)) return lo;
    if (!fl) {
        const int64_t t = (int64_t)lo + (int64_t)hi + 1;
        return (double)(t >= 0 ? t / 2 : -((-t + 1) / 2));
    }
    float s = (float)(0.5 * (lo + hi));
    if ((double)s <= lo) s = next_up((float)lo);
    return (double)s;
}

// The largest coordinate below s.
__device__ inline double value_below(double s, bool fl) {
    return fl ? (double)next_down((float)s) : s - 1.0;
}

// The cut dimension of space [lo, hi] at depth `depth`.
__device__ inline int space_dim(const double* lo, const double* hi, int d, int depth, int widest) {
    if (!widest) return depth % d;
    int c = 0;
    for (int e = 1; e < d; e++)
        if (hi[e] - lo[e] > hi[c] - lo[c]) c = e;
    return c;
}

// The list of nodes a level processes (SoA): splitting nodes first, then the
// identical-point nodes whose segment is copied.
struct Entries {
    uint32_t* node;   // node id
    uint32_t* par;    // its parent
    uint32_t* lo;     // segment start (leaf-order position)
    uint32_t* cnt;    // points
    uint32_t* cut;    // key of the cut
    uint32_t* dim;    // cut dimension | kCopy
    double* cell;     // [A][2d] cell (cell form): lo[d], hi[d]
};

// The counts of one level, kept in device memory so that levels are queued
// without the host reading them: splitting entries, copy entries, chunks,
// and the id of the level's first child node.
struct Level {
    uint32_t As, Ac, C, nbase;
};

struct Nodes {
    uint4* xn;        // records
    uint32_t* key;    // [N][2d] box keys: min[d], max[d]
    uint32_t* lo;     // segment start
    uint32_t* cnt;    // points
};

// Box keys of the root.
__global__ void __launch_bounds__(kNT)
root_box_kernel(const uint32_t* __restrict__ keys, int64_t n, int d, uint32_t* __restrict__ box) {
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

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t count, uint32_t lo_val,
                                uint32_t hi_val, int d) {
    // boxes: words [2d) per node, min then max
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < count) p[i] = (i % (2 * d)) < d ? lo_val : hi_val;
}

// Whether the box (keys) holds a single location.
__device__ inline bool box_single(const uint32_t* b, int d) {
    bool same = true;
    for (int c = 0; c < d; c++) same = same && b[c] == b[d + c];
    return same;
}

// Sets up the root: a leaf (copied when it holds points) or the first
// splitting node.  tot = {splitting entries, copy entries}; cstart = {0, chunks}.
__global__ void root_kernel(Nodes N, Entries E, int64_t n, int d, int leaf, int fl, int rule,
                            uint32_t* __restrict__ cstart, uint32_t* __restrict__ tot) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t* b = N.key;
    const bool isleaf = n <= leaf || box_single(b, d);
    N.lo[0] = 0;
    N.cnt[0] = (uint32_t)n;
    const uint32_t chunks = (uint32_t)((n + kCH - 1) / kCH);
    cstart[0] = 0;
    cstart[1] = chunks;
    if (isleaf) {
        N.xn[0] = make_uint4(0u, 0u, kXNone, kXLeaf | (n == 0 ? kXEmpty : 0u));
        tot[0] = 0;
        tot[1] = n > 0 ? 1u : 0u;
        if (n > 0) {
            E.node[0] = 0;
            E.par[0] = kXNone;
            E.lo[0] = 0;
            E.cnt[0] = (uint32_t)n;
            E.cut[0] = 0;
            E.dim[0] = kCopy;
        }
        return;
    }
    double lo[8], hi[8];
    for (int c = 0; c < d; c++) {
        lo[c] = coord_value(key_to_coord(b[c], fl != 0), fl != 0);
        hi[c] = coord_value(key_to_coord(b[d + c], fl != 0), fl != 0);
        if (!(rule & 2)) {
            E.cell[c] = lo[c];
            E.cell[d + c] = hi[c];
        }
    }
    const int c = space_dim(lo, hi, d, 0, rule & 1);
    const double s = space_cut(lo[c], hi[c], fl != 0);
    E.node[0] = 0;
    E.par[0] = kXNone;
    E.lo[0] = 0;
    E.cnt[0] = (uint32_t)n;
    E.cut[0] = coord_to_key(value_bits(s, fl != 0), fl != 0);
    E.dim[0] = (uint32_t)c;
    tot[0] = 1;
    tot[1] = 0;
}

// The first level's counts from the root's set-up.
__global__ void level_init_kernel(Level* __restrict__ L, const uint32_t* __restrict__ tot,
                                  const uint32_t* __restrict__ cstart) {
    if (threadIdx.x == 0 && blockIdx.x == 0) L[0] = Level{tot[0], tot[1], cstart[1], 1u};
}

// The next level's counts: the split and copy entries the scan of the
// children's flags counted, their chunks, and the node id after this
// level's children.  A level without splitting entries ends the build.
__global__ void level_advance_kernel(Level* __restrict__ L, const uint64_t* __restrict__ ftot,
                                     const uint32_t* __restrict__ cst_next) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const Level c = L[0];
    Level x{0u, 0u, 0u, c.nbase};
    if (c.As > 0) {
        const uint64_t f = *ftot;
        x.As = (uint32_t)f;
        x.Ac = (uint32_t)(f >> 32);
        x.C = cst_next[2u * c.As];
        x.nbase = c.nbase + 2u * c.As;
    }
    L[1] = x;
}

// Entry of chunk c (the same in every lane): the last a with cstart[a] <= c
// (every entry has a chunk).  A 64-way search: each step the lanes test 64
// evenly spaced candidates, so a level of 10^6 entries takes four loads.
__device__ inline uint32_t chunk_entry(const uint32_t* cstart, uint32_t A, uint32_t c) {
    uint32_t lo = 0, hi = A;  // cstart[lo] <= c < cstart[hi]
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + kWave - 1) / kWave;
        const uint32_t at = lo + (uint32_t)lane_id() * step;
        const uint64_t le = __ballot(at < hi && cstart[at] <= c);  // a prefix of the lanes
        const uint32_t last = 63u - (uint32_t)__clzll(le);
        lo = lo + last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Splitting entries of at least kRepChunks chunks reduce their children's
// boxes into kReplicas copies each (replica = chunk mod kReplicas): with one
// set of words per child, every chunk of a big node would update the same
// few words, and those atomics serialise.
constexpr uint32_t kRepChunks = 16;
constexpr int kReplicas = 64;
constexpr uint32_t kNoRep = 0xffffffffu;

// One chunk of chunk_count_kernel.
__device__ inline void chunk_count_one(const Entries& E, const uint32_t* __restrict__ cstart, uint32_t A,
                                       uint32_t c, const uint32_t* __restrict__ keys, int64_t n,
                                       uint32_t* __restrict__ c2e, uint32_t* __restrict__ lcnt, int d,
                                       uint32_t* __restrict__ rbase, uint32_t* __restrict__ rentry,
                                       uint32_t* __restrict__ rcount, uint32_t* __restrict__ rep) {
    const uint32_t a = chunk_entry(cstart, A, c);
    const uint32_t dm = E.dim[a];
    if (c == cstart[a]) {
        uint32_t b = kNoRep;
        if (!(dm & kCopy) && cstart[a + 1] - c >= kRepChunks) {
            if (lane_id() == 0) b = atomicAdd(rcount, 1u);
            b = __shfl(b, 0, kWave);
            uint32_t* blk = rep + (size_t)b * 2 * kReplicas * 2 * d;
            for (int w = lane_id(); w < 2 * kReplicas * 2 * d; w += kWave)
                blk[w] = (w % (2 * d)) < d ? 0xffffffffu : 0u;
            if (lane_id() == 0) rentry[b] = a;
        }
        if (lane_id() == 0) rbase[a] = b;
    }
    uint32_t left = 0;
    if (!(dm & kCopy)) {
        const uint32_t lo = E.lo[a], end = lo + E.cnt[a];
        const uint32_t base = lo + (c - cstart[a]) * kCH;
        const uint32_t cut = E.cut[a];
        const uint32_t* plane = keys + (int64_t)(dm & 15u) * n;
        uint32_t kv[kChunkGroups];
#pragma unroll
        for (int g = 0; g < kChunkGroups; g++) {
            const uint32_t p = base + g * kWave + lane_id();
            kv[g] = p < end ? plane[p] : 0xffffffffu;
        }
#pragma unroll
        for (int g = 0; g < kChunkGroups; g++) {
            const uint32_t p = base + g * kWave + lane_id();
            left += (uint32_t)__popcll(__ballot(p < end && kv[g] < cut));
        }
    }
    if (lane_id() == 0) {
        c2e[c] = a;
        lcnt[c] = left;
    }
}

// Per chunk (one wave, grid-stride): its entry, and the number of its
// points going left.  The first chunk of a splitting entry with kRepChunks
// or more chunks takes a replica block (rbase[a]; block b serves entry
// rentry[b]) and resets it.
__global__ void __launch_bounds__(kNT)
chunk_count_kernel(Entries E, const uint32_t* __restrict__ cstart, const Level* __restrict__ L,
                   const uint32_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ c2e,
                   uint32_t* __restrict__ lcnt, int d, uint32_t* __restrict__ rbase,
                   uint32_t* __restrict__ rentry, uint32_t* __restrict__ rcount,
                   uint32_t* __restrict__ rep) {
    const uint32_t A = L->As + L->Ac, C = L->C;
    if (blockIdx.x == 0 && threadIdx.x == 0) lcnt[C] = 0;
    for (uint32_t c = blockIdx.x * (kNT / kWave) + threadIdx.x / kWave; c < C;
         c += gridDim.x * (kNT / kWave))
        chunk_count_one(E, cstart, A, c, keys, n, c2e, lcnt, d, rbase, rentry, rcount, rep);
}
// Writes point (keys kv, row r) to leaf-order position p of the tree.
template <int MD>
__device__ inline void put_final(const uint32_t (&kv)[MD], int32_t r, int64_t p, int d, int rw, bool fl,
                                 int64_t n, uint32_t* __restrict__ pts, uint32_t* __restrict__ rec,
                                 int32_t* __restrict__ pidx) {
    uint32_t w[16];
#pragma unroll
    for (int e = 0; e < 16; e++) w[e] = 0u;
#pragma unroll
    for (int c = 0; c < MD; c++) {
        if (c < d) {
            const uint32_t v = key_to_coord(kv[c], fl);
            pts[(int64_t)c * n + p] = v;
            w[c] = v;
        }
    }
#pragma unroll
    for (int e = 0; e < 16; e++)
        if (e == d) w[e] = (uint32_t)r;
    uint4* dst = reinterpret_cast<uint4*>(rec + p * rw);
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (q < rw / 4) dst[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    pidx[p] = r;
}

// Per chunk (one wave): stable partition of the chunk's points (left: key
// of the cut dimension below the cut), into the other buffer or, for a child
// that is a leaf by its count, the tree's arrays; reduces each child's box.
// Copy entries write their points to the tree's arrays in place.
template <int MD>
__device__ inline void chunk_scatter_one(const Entries& E, const Nodes& N, const uint32_t* __restrict__ cstart,
                                         const uint32_t* __restrict__ lpre, const uint32_t* __restrict__ c2e,
                                         uint32_t c, uint32_t nbase, const uint32_t* __restrict__ rbase,
                                         uint32_t* __restrict__ rep, int leaf, int d, int rw, int fl,
                                         const uint32_t* __restrict__ keys, const int32_t* __restrict__ idx,
                                         uint32_t* __restrict__ okeys, int32_t* __restrict__ oidx, int64_t n,
                                         uint32_t* __restrict__ pts, uint32_t* __restrict__ rec,
                                         int32_t* __restrict__ pidx) {
    const uint32_t a = c2e[c];
    const uint32_t dm = E.dim[a];
    const uint32_t lo = E.lo[a], cnt = E.cnt[a], end = lo + cnt;
    const uint32_t off = (c - cstart[a]) * kCH;
    const int lane = lane_id();
    if (dm & kCopy) {
        for (int g = 0; g < kChunkGroups; g++) {
            const uint32_t p = lo + off + g * kWave + lane;
            if (p < end) {
                uint32_t kv[MD];
#pragma unroll
                for (int e = 0; e < MD; e++) kv[e] = e < d ? keys[(int64_t)e * n + p] : 0u;
                put_final<MD>(kv, idx[p], p, d, rw, fl != 0, n, pts, rec, pidx);
            }
        }
        return;
    }
    const int dim = (int)(dm & 15u);
    const uint32_t cut = E.cut[a];
    const uint32_t cs = cstart[a];
    uint32_t lb = lpre[c] - lpre[cs];  // left points before this chunk in the node
    const uint32_t nl = lpre[cstart[a + 1]] - lpre[cs];
    uint32_t rb = off - lb;
    const uint32_t nr = cnt - nl;
    const bool lfin = nl <= (uint32_t)leaf, rfin = nr <= (uint32_t)leaf;
    uint32_t bmin[2][MD], bmax[2][MD];
#pragma unroll
    for (int e = 0; e < MD; e++) {
        bmin[0][e] = bmin[1][e] = 0xffffffffu;
        bmax[0][e] = bmax[1][e] = 0u;
    }
    bool any0 = false, any1 = false;
    for (int g = 0; g < kChunkGroups; g++) {
        const uint32_t p = lo + off + g * kWave + lane;
        const bool valid = p < end;
        uint32_t kv[MD];
        int32_t r = 0;
#pragma unroll
        for (int e = 0; e < MD; e++) kv[e] = (valid && e < d) ? keys[(int64_t)e * n + p] : 0u;
        if (valid) r = idx[p];
        uint32_t kc = kv[0];
#pragma unroll
        for (int e = 1; e < MD; e++) kc = e == dim ? kv[e] : kc;
        const bool left = valid && kc < cut;
        const uint64_t bl = __ballot(left), br = __ballot(valid && !left);
        any0 = any0 || bl != 0;
        any1 = any1 || br != 0;
        if (valid) {
            const uint32_t dst = left ? lo + lb + lane_prefix(bl) : lo + nl + rb + lane_prefix(br);
            if (left ? lfin : rfin) {
                put_final<MD>(kv, r, dst, d, rw, fl != 0, n, pts, rec, pidx);
            } else {
#pragma unroll
                for (int e = 0; e < MD; e++)
                    if (e < d) okeys[(int64_t)e * n + dst] = kv[e];
                oidx[dst] = r;
            }
#pragma unroll
            for (int e = 0; e < MD; e++) {
                if (e < d) {
                    const int sd = left ? 0 : 1;
                    // select without dynamic register indexing
                    if (sd == 0) {
                        bmin[0][e] = kv[e] < bmin[0][e] ? kv[e] : bmin[0][e];
                        bmax[0][e] = kv[e] > bmax[0][e] ? kv[e] : bmax[0][e];
                    } else {
                        bmin[1][e] = kv[e] < bmin[1][e] ? kv[e] : bmin[1][e];
                        bmax[1][e] = kv[e] > bmax[1][e] ? kv[e] : bmax[1][e];
                    }
                }
            }
        }
        lb += (uint32_t)__popcll(bl);
        rb += (uint32_t)__popcll(br);
    }
    // the children's boxes, or (entries with a replica block) replica
    // c mod kReplicas of them
    const uint32_t c0 = nbase + 2u * a;
    const uint32_t rblk = rbase[a];
#pragma unroll
    for (int sd = 0; sd < 2; sd++) {
        if (sd == 0 ? !any0 : !any1) continue;
        uint32_t* bk = rblk != kNoRep
                           ? rep + (((size_t)rblk * 2 + sd) * kReplicas + (c - cs) % kReplicas) * 2 * d
                           : N.key + (size_t)(c0 + sd) * 2 * d;
#pragma unroll
        for (int e = 0; e < MD; e++) {
            if (e < d) {
                const uint32_t mn = wave_min_u32(bmin[sd][e]);
                const uint32_t mx = wave_max_u32(bmax[sd][e]);
                if (lane == 0) {
                    atomicMin(&bk[e], mn);
                    atomicMax(&bk[d + e], mx);
                }
            }
        }
    }
}

template <int MD>
__global__ void __launch_bounds__(kNT)
chunk_scatter_kernel(Entries E, Nodes N, const uint32_t* __restrict__ cstart,
                     const uint32_t* __restrict__ lpre, const uint32_t* __restrict__ c2e,
                     const Level* __restrict__ L, const uint32_t* __restrict__ rbase,
                     uint32_t* __restrict__ rep, int leaf, int d, int rw, int fl,
                     const uint32_t* __restrict__ keys, const int32_t* __restrict__ idx,
                     uint32_t* __restrict__ okeys, int32_t* __restrict__ oidx, int64_t n,
                     uint32_t* __restrict__ pts, uint32_t* __restrict__ rec,
                     int32_t* __restrict__ pidx) {
    const uint32_t C = L->C, nbase = L->nbase;
    for (uint32_t c = blockIdx.x * (kNT / kWave) + threadIdx.x / kWave; c < C;
         c += gridDim.x * (kNT / kWave))
        chunk_scatter_one<MD>(E, N, cstart, lpre, c2e, c, nbase, rbase, rep, leaf, d, rw, fl, keys, idx,
                              okeys, oidx, n, pts, rec, pidx);
}

// Boxes of the children of the entries with a replica block: one wave per
// (block, child), one replica per lane (grid-stride).
__global__ void __launch_bounds__(kNT)
merge_replicas_kernel(const uint32_t* __restrict__ rep, const uint32_t* __restrict__ rentry,
                      const uint32_t* __restrict__ rcount, const Level* __restrict__ L, int d,
                      uint32_t* __restrict__ key) {
    const uint32_t nbase = L->nbase, slots = 2u * *rcount;
    const int lane = lane_id();
    for (uint32_t t = blockIdx.x * (kNT / kWave) + threadIdx.x / kWave; t < slots;
         t += gridDim.x * (kNT / kWave)) {  // 2 block + child
        const uint32_t a = rentry[t >> 1];
        const uint32_t* r = rep + ((size_t)t * kReplicas + lane) * 2 * d;
        uint32_t* k = key + (size_t)(nbase + 2u * a + (t & 1u)) * 2 * d;
        for (int c = 0; c < d; c++) {
            const uint32_t mn = wave_min_u32(r[c]);
            const uint32_t mx = wave_max_u32(r[d + c]);
            if (lane == 0) {
                k[c] = mn;
                k[d + c] = mx;
            }
        }
    }
}

// One entry of split_nodes_kernel.
__device__ inline void split_node_one(const Entries& E, const Nodes& N, const uint32_t* __restrict__ cstart,
                                      const uint32_t* __restrict__ lpre, uint32_t a, uint32_t nbase,
                                      int leaf, int d, int fl, uint64_t* __restrict__ flags,
                                      uint32_t* __restrict__ nch_next) {
    const uint32_t u = E.node[a];
    const uint32_t lo = E.lo[a], cnt = E.cnt[a];
    const uint32_t nl = lpre[cstart[a + 1]] - lpre[cstart[a]];
    const uint32_t c0 = nbase + 2u * a;
    uint32_t meta = E.dim[a] & 15u;
    for (int s = 0; s < 2; s++) {
        const uint32_t cc = c0 + s;
        const uint32_t ccnt = s ? cnt - nl : nl;
        const bool small = ccnt <= (uint32_t)leaf;
        const bool same = !small && box_single(N.key + (size_t)cc * 2 * d, d);
        const bool isleaf = small || same;
        N.lo[cc] = s ? lo + nl : lo;
        N.cnt[cc] = ccnt;
        N.xn[cc] = make_uint4(0u, 0u, u, isleaf ? (kXLeaf | (ccnt == 0 ? kXEmpty : 0u)) : 0u);
        if (isleaf) meta |= kXChildLeaf << s;
        if (ccnt == 0) meta |= kXChildEmpty << s;
        flags[2 * a + s] = small ? 0ull : (same ? kFlagCopy : kFlagSplit);
        nch_next[2 * a + s] = 0u;
    }
    N.xn[u] = make_uint4(key_to_coord(E.cut[a], fl != 0), c0, E.par[a], meta);
}

// Per splitting entry (grid-stride): the node's record, its children's
// records, counts and segments, and the children's flags for the next level
// (split / copy / leaf).
__global__ void __launch_bounds__(kNT)
split_nodes_kernel(Entries E, Nodes N, const uint32_t* __restrict__ cstart,
                   const uint32_t* __restrict__ lpre, const Level* __restrict__ L, int leaf, int d,
                   int fl, uint64_t* __restrict__ flags, uint32_t* __restrict__ nch_next,
                   uint32_t* __restrict__ rcount) {
    const uint32_t As = L->As, nbase = L->nbase;
    if (blockIdx.x == 0 && threadIdx.x == 0) *rcount = 0;  // the replica blocks were merged
    for (uint32_t a = blockIdx.x * kNT + threadIdx.x; a < As; a += gridDim.x * kNT)
        split_node_one(E, N, cstart, lpre, a, nbase, leaf, d, fl, flags, nch_next);
}

// Per child slot t = 2a + s of the level's splitting entries: the next
// level's entry of a child that splits (its space, cut dimension and cut;
// the boxes of its future children reset) or is copied.
__device__ inline void emit_one(const Entries& E, const Entries& X, const Nodes& N,
                                const uint64_t* __restrict__ flags, const uint64_t* __restrict__ fpre,
                                const uint64_t* __restrict__ ftot, uint32_t t, uint32_t nbase,
                                uint32_t nbase_next, int depth, int d, int fl, int rule,
                                uint32_t* __restrict__ nch_next) {
    const uint64_t f = flags[t];
    if (f == 0) return;
    const uint32_t a = t >> 1, s = t & 1u;
    const uint32_t cc = nbase + t;
    const uint32_t lo = N.lo[cc], cnt = N.cnt[cc];
    const uint32_t chunks = (cnt + kCH - 1) / kCH;
    if (f == kFlagCopy) {
        const uint32_t e = (uint32_t)(*ftot) + (uint32_t)(fpre[t] >> 32);
        X.node[e] = cc;
        X.par[e] = E.node[a];
        X.lo[e] = lo;
        X.cnt[e] = cnt;
        X.cut[e] = 0;
        X.dim[e] = kCopy;
        nch_next[e] = chunks;
        return;
    }
    const uint32_t e = (uint32_t)fpre[t];
    const bool fb = fl != 0;
    double slo[8], shi[8];
    if (rule & 2) {
        const uint32_t* b = N.key + (size_t)cc * 2 * d;
        for (int c = 0; c < d; c++) {
            slo[c] = coord_value(key_to_coord(b[c], fb), fb);
            shi[c] = coord_value(key_to_coord(b[d + c], fb), fb);
        }
    } else {
        // the child's cell: the parent's cell, cut
        const double* pc = E.cell + (size_t)a * 2 * d;
        for (int c = 0; c < d; c++) {
            slo[c] = pc[c];
            shi[c] = pc[d + c];
        }
        const int pd = (int)(E.dim[a] & 15u);
        const double ps = coord_value(key_to_coord(E.cut[a], fb), fb);
        if (s == 0) shi[pd] = value_below(ps, fb);
        else slo[pd] = ps;
        double* xc = X.cell + (size_t)e * 2 * d;
        for (int c = 0; c < d; c++) {
            xc[c] = slo[c];
            xc[d + c] = shi[c];
        }
    }
    const int c = space_dim(slo, shi, d, depth, rule & 1);
    const double cut = space_cut(slo[c], shi[c], fb);
    X.node[e] = cc;
    X.par[e] = E.node[a];
    X.lo[e] = lo;
    X.cnt[e] = cnt;
    X.cut[e] = coord_to_key(value_bits(cut, fb), fb);
    X.dim[e] = (uint32_t)c;
    nch_next[e] = chunks;
    uint32_t* bk = N.key + (size_t)(nbase_next + 2u * e) * 2 * d;
    for (int w = 0; w < 2 * d; w++) {
        bk[w] = (w % (2 * d)) < d ? 0xffffffffu : 0u;
        bk[2 * d + w] = (w % (2 * d)) < d ? 0xffffffffu : 0u;
    }
}

// emit_one over the level's child slots (grid-stride).
__global__ void __launch_bounds__(kNT)
emit_kernel(Entries E, Entries X, Nodes N, const uint64_t* __restrict__ flags,
            const uint64_t* __restrict__ fpre, const uint64_t* __restrict__ ftot,
            const Level* __restrict__ L, int depth, int d, int fl, int rule,
            uint32_t* __restrict__ nch_next) {
    const uint32_t As = L->As, nbase = L->nbase;
    const uint32_t nbase_next = nbase + 2u * As;
    for (uint32_t t = blockIdx.x * kNT + threadIdx.x; t < 2u * As; t += gridDim.x * kNT)
        emit_one(E, X, N, flags, fpre, ftot, t, nbase, nbase_next, depth, d, fl, rule, nch_next);
}

// Leaves below each node of one level (bottom-up, deepest level first).
__global__ void leaf_count_kernel(const uint4* __restrict__ xn, uint32_t first, uint32_t count,
                                  uint32_t* __restrict__ nlv) {
    const uint32_t i = blockIdx.x * kNT + threadIdx.x;
    if (i >= count) return;
    const uint32_t u = first + i;
    const uint4 r = xn[u];
    nlv[u] = (r.w & kXLeaf) ? 1u : nlv[r.y] + nlv[r.y + 1];
}

// Leaf-index spans of one level's nodes (top-down; jlo[u] is set by the
// parent's level, the root's is 0): children's spans, and for a leaf its
// index, offset and node.
__global__ void leaf_index_kernel(uint4* __restrict__ xn, uint32_t first, uint32_t count,
                                  const uint32_t* __restrict__ nlv, uint32_t* __restrict__ jlo,
                                  const uint32_t* __restrict__ nlo, uint2* __restrict__ xspan,
                                  int64_t* __restrict__ loff, uint32_t* __restrict__ lnode) {
    const uint32_t i = blockIdx.x * kNT + threadIdx.x;
    if (i >= count) return;
    const uint32_t u = first + i;
    const uint32_t j = u == 0 ? 0u : jlo[u];
    const uint4 r = xn[u];
    xspan[u] = make_uint2(j, j + nlv[u]);
    if (r.w & kXLeaf) {
        xn[u].x = j;
        loff[j] = nlo[u];
        lnode[j] = u;
    } else {
        jlo[r.y] = j;
        jlo[r.y + 1] = j + nlv[r.y];
    }
}

// Node boxes as coordinates (an empty node: the empty box, which every box
// query misses).
__global__ void node_box_kernel(const uint32_t* __restrict__ key, const uint32_t* __restrict__ cnt,
                                int64_t N, int d, int fl, uint32_t* __restrict__ nbox) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= N * 2 * d) return;
    const int64_t u = i / (2 * d);
    const int w = (int)(i % (2 * d));
    const uint32_t k = cnt[u] == 0 ? (w < d ? empty_min_key(fl != 0) : empty_max_key(fl != 0)) : key[i];
    nbox[i] = key_to_coord(k, fl != 0);
}

__global__ void set_i64_kernel(int64_t* __restrict__ p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// A device array that grows by copying (node arrays of unknown final size).
template <typename T>
struct Grow {
    T* p = nullptr;
    size_t cap = 0;
    hipStream_t s = nullptr;
    ~Grow() { if (p) dfree(p, s); }
    pg_status reserve(size_t need, size_t used) {
        if (need <= cap) return PG_OK;
        size_t nc = cap ? cap : 1024;
        while (nc < need) nc *= 2;
        T* q = nullptr;
        PG_TRY(dalloc(&q, nc, s));
        if (used) PG_HIP(hipMemcpyAsync(q, p, sizeof(T) * used, hipMemcpyDeviceToDevice, s));
        if (p) dfree(p, s);
        p = q;
        cap = nc;
        return PG_OK;
    }
    T* release() { T* q = p; p = nullptr; cap = 0; return q; }
};

template <int MD>
void launch_scatter(unsigned grid, hipStream_t s, const Entries& E, const Nodes& N,
                    const uint32_t* cstart, const uint32_t* lpre, const uint32_t* c2e, const Level* L,
                    const uint32_t* rbase, uint32_t* rep, int leaf, int d, int rw, int fl,
                    const uint32_t* keys, const int32_t* idx, uint32_t* okeys, int32_t* oidx, int64_t n,
                    pg_tree* T) {
    hipLaunchKernelGGL((chunk_scatter_kernel<MD>), dim3(grid), dim3(kNT), 0, s, E, N, cstart, lpre,
                       c2e, L, rbase, rep, leaf, d, rw, fl, keys, idx, okeys, oidx, n, T->pts, T->rec,
                       T->pidx);
}

// Leaf boxes (keys) of an explicit-node tree from its points: one lane per
// leaf-order position, a segmented min/max over the lanes of each leaf, one
// atomic per (leaf, dimension) and wave.
__global__ void __launch_bounds__(kNT)
xleaf_box_kernel(TreeView tv, int fl, uint32_t* __restrict__ lkey) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const bool valid = p < tv.n;
    if (__ballot(valid) == 0) return;
    uint32_t j = 0xffffffffu;
    if (valid) {
        uint32_t lo = 0, hi = (uint32_t)tv.nleaves;  // loff[lo] <= p < loff[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tv.loff[mid] <= p) lo = mid;
            else hi = mid;
        }
        j = lo;
    }
    const int lane = lane_id();
    const uint32_t jprev = __shfl_up(j, 1, kWave);
    const bool head = valid && (lane == 0 || jprev != j);
    const int d = tv.d;
    for (int c = 0; c < d; c++) {
        const uint32_t k = valid ? coord_to_key(tv.pts[(int64_t)c * tv.n + p], fl != 0) : 0u;
        uint32_t mn = valid ? k : 0xffffffffu, mx = k;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t omn = __shfl_down(mn, off, kWave), omx = __shfl_down(mx, off, kWave);
            const uint32_t oj = __shfl_down(j, off, kWave);
            if (lane + off < kWave && oj == j) {
                mn = omn < mn ? omn : mn;
                mx = omx > mx ? omx : mx;
            }
        }
        if (head) {
            atomicMin(&lkey[(int64_t)j * 2 * d + c], mn);
            atomicMax(&lkey[(int64_t)j * 2 * d + d + c], mx);
        }
    }
}

// One level of an explicit-node tree, bottom-up: a leaf's box from its
// points and its empty flag from its range; an internal node's box as the
// union of its children's, and its child flags from theirs.
__global__ void xrefresh_kernel(uint4* __restrict__ xn, uint32_t first, uint32_t count, int d, int fl,
                                const uint32_t* __restrict__ lkey, const int64_t* __restrict__ loff,
                                uint32_t* __restrict__ nkey, uint32_t* __restrict__ ncnt,
                                uint32_t* __restrict__ nbox) {
    const uint32_t i = blockIdx.x * kNT + threadIdx.x;
    if (i >= count) return;
    const uint32_t u = first + i;
    uint4 r = xn[u];
    uint32_t* bk = nkey + (size_t)u * 2 * d;
    if (r.w & kXLeaf) {
        const uint32_t c = (uint32_t)(loff[r.x + 1] - loff[r.x]);
        for (int w = 0; w < 2 * d; w++) bk[w] = lkey[(size_t)r.x * 2 * d + w];
        ncnt[u] = c;
        r.w = (r.w & ~kXEmpty) | (c == 0 ? kXEmpty : 0u);
    } else {
        const uint32_t* b0 = nkey + (size_t)r.y * 2 * d;
        const uint32_t* b1 = b0 + 2 * d;
        for (int c = 0; c < d; c++) {
            bk[c] = b0[c] < b1[c] ? b0[c] : b1[c];
            bk[d + c] = b0[d + c] > b1[d + c] ? b0[d + c] : b1[d + c];
        }
        const uint32_t c0 = ncnt[r.y], c1 = ncnt[r.y + 1];
        ncnt[u] = c0 + c1;
        r.w &= ~(3u * kXChildEmpty);
        r.w |= (c0 == 0 ? kXChildEmpty : 0u) | (c1 == 0 ? kXChildEmpty << 1 : 0u);
    }
    xn[u] = r;
    const uint32_t cu = ncnt[u];
    for (int w = 0; w < 2 * d; w++) {
        const uint32_t k = cu == 0 ? (w < d ? empty_min_key(fl != 0) : empty_max_key(fl != 0)) : bk[w];
        nbox[(size_t)u * 2 * d + w] = key_to_coord(k, fl != 0);
    }
}

}  // namespace

pg_status xtree_boxes(pg_tree* T, hipStream_t s) {
    const int d = T->d;
    const int fl = T->dtype == PG_FLOAT32 ? 1 : 0;
    const int64_t leaves = T->nleaves, nodes = T->nnodes;
    DevBuf lk(s), nk(s), nc(s);
    PG_TRY(lk.alloc(sizeof(uint32_t) * (size_t)leaves * 2 * d));
    PG_TRY(nk.alloc(sizeof(uint32_t) * (size_t)nodes * 2 * d));
    PG_TRY(nc.alloc(sizeof(uint32_t) * (size_t)nodes));
    hipLaunchKernelGGL(fill_u32_kernel, dim3(cdiv(leaves * 2 * d, kNT)), dim3(kNT), 0, s,
                       lk.as<uint32_t>(), leaves * 2 * d, 0xffffffffu, 0u, d);
    PG_LAUNCH_CHECK();
    if (T->n > 0) {
        hipLaunchKernelGGL(xleaf_box_kernel, dim3(cdiv(T->n, kNT)), dim3(kNT), 0, s, T->view(), fl,
                           lk.as<uint32_t>());
        PG_LAUNCH_CHECK();
    }
    for (int l = (int)T->lvl.size() - 2; l >= 0; l--) {
        const uint32_t first = (uint32_t)T->lvl[l], count = (uint32_t)(T->lvl[l + 1] - T->lvl[l]);
        hipLaunchKernelGGL(xrefresh_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s, T->xn, first,
                           count, d, fl, lk.as<uint32_t>(), T->loff, nk.as<uint32_t>(),
                           nc.as<uint32_t>(), T->nbox);
        PG_LAUNCH_CHECK();
    }
    return PG_OK;
}

pg_status build_tree_spatial(const void* points, int64_t n, int d, int leaf, int dtype, int rule,
                             hipStream_t s, pg_tree* T) {
    const bool fl = dtype == PG_FLOAT32;
    const int ifl = fl ? 1 : 0;
    T->n = n;
    T->d = d;
    T->leaf = leaf;
    T->dtype = dtype;
    T->stream = s;
    T->rule = rule;
    const int64_t nn = n > 0 ? n : 1;
    const int rw = record_words(d);
    PG_TRY(dalloc(&T->pts, (size_t)d * nn, s));
    PG_TRY(dalloc(&T->pidx, (size_t)nn + kTreePad, s));
    PG_TRY(dalloc(&T->rec, ((size_t)nn + kTreePad) * rw, s));

    // key planes (ping-pong), node arrays, per-level entries
    DevBuf ka(s), ia(s), kb(s), ib(s), aux(s);
    PG_TRY(ka.alloc(sizeof(uint32_t) * (size_t)d * nn));
    PG_TRY(ia.alloc(sizeof(int32_t) * (size_t)nn));
    uint32_t vary[8] = {0}, keybase[8] = {0};
    if (n > 0)
        PG_TRY(ingest_points(points, n, d, fl, ka.as<uint32_t>(), ia.as<int32_t>(), vary, keybase, s));
    PG_TRY(kb.alloc(sizeof(uint32_t) * (size_t)d * nn));
    PG_TRY(ib.alloc(sizeof(int32_t) * (size_t)nn));

    Grow<uint4> gxn;
    Grow<uint32_t> gkey, glo, gcnt;
    gxn.s = gkey.s = glo.s = gcnt.s = s;
    const size_t guess = (size_t)(4 * (nn / leaf) + 64);
    PG_TRY(gxn.reserve(guess, 0));
    PG_TRY(gkey.reserve(guess * 2 * d, 0));
    PG_TRY(glo.reserve(guess, 0));
    PG_TRY(gcnt.reserve(guess, 0));

    // entries: at most one per (leaf + 1) points, per level; two sets
    const size_t amax = (size_t)(nn / (leaf + 1) + 2);
    const size_t cmax = (size_t)(nn / kCH + amax + 2);  // chunks
    DevBuf ebuf[2] = {DevBuf(s), DevBuf(s)};
    Entries ent[2];
    for (int b = 0; b < 2; b++) {
        const size_t cellw = (rule & 2) ? 0 : amax * 2 * d;
        PG_TRY(ebuf[b].alloc(sizeof(double) * cellw + sizeof(uint32_t) * amax * 6));
        ent[b].cell = ebuf[b].as<double>();
        uint32_t* w = reinterpret_cast<uint32_t*>(ent[b].cell + cellw);
        ent[b].node = w;
        ent[b].par = w + amax;
        ent[b].lo = w + 2 * amax;
        ent[b].cnt = w + 3 * amax;
        ent[b].cut = w + 4 * amax;
        ent[b].dim = w + 5 * amax;
    }
    // chunk starts x 2 (current / next; the next level's are first indexed
    // by child slot, [2 amax + 1]), c2e [cmax], lcnt [cmax + 1], flags and
    // their prefix [2 amax] u64, totals
    DevBuf cbuf(s), fbuf(s), rbuf(s), rmeta(s);
    // replica blocks: one per entry of kRepChunks or more chunks, which holds
    // more than kCH (kRepChunks - 1) points
    const size_t rmax = (size_t)(nn / (kCH * (kRepChunks - 1)) + 2);
    PG_TRY(rbuf.alloc(sizeof(uint32_t) * rmax * 2 * kReplicas * 2 * d));
    PG_TRY(rmeta.alloc(sizeof(uint32_t) * (amax + rmax + 1)));
    uint32_t* rbase = rmeta.as<uint32_t>();  // [amax] per entry
    uint32_t* rentry = rbase + amax;         // [rmax] per block
    uint32_t* rcount = rentry + rmax;        // blocks taken this level
    PG_HIP(hipMemsetAsync(rcount, 0, sizeof(uint32_t), s));
    PG_TRY(cbuf.alloc(sizeof(uint32_t) * (2 * (2 * amax + 1) + cmax + cmax + 1 + 8)));
    uint32_t* cst[2] = {cbuf.as<uint32_t>(), cbuf.as<uint32_t>() + 2 * amax + 1};
    uint32_t* c2e = cst[1] + 2 * amax + 1;
    uint32_t* lcnt = c2e + cmax;
    uint32_t* tot32 = lcnt + cmax + 1;  // [0] root splitting entries, [1] root copies
    PG_TRY(fbuf.alloc(sizeof(uint64_t) * (4 * amax + 2)));
    uint64_t* flags = fbuf.as<uint64_t>();
    uint64_t* fpre = flags + 2 * amax;
    uint64_t* ftot = fpre + 2 * amax;

    Nodes N{gxn.p, gkey.p, glo.p, gcnt.p};
    // root box
    PG_HIP(hipMemsetAsync(gkey.p, 0xff, sizeof(uint32_t) * d, s));
    PG_HIP(hipMemsetAsync(gkey.p + d, 0, sizeof(uint32_t) * d, s));
    if (n > 0) {
        const unsigned grid = cdiv(n, kNT) < 1024u ? cdiv(n, kNT) : 1024u;
        hipLaunchKernelGGL(root_box_kernel, dim3(grid), dim3(kNT), 0, s, ka.as<uint32_t>(), n, d,
                           gkey.p);
        PG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(root_kernel, dim3(1), dim3(1), 0, s, N, ent[0], n, d, leaf, ifl, rule, cst[0],
                       tot32);
    PG_LAUNCH_CHECK();
    // the root's children's boxes start empty
    if (n > 0) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(cdiv(4 * d, kNT)), dim3(kNT), 0, s, gkey.p + 2 * d,
                           (int64_t)4 * d, 0xffffffffu, 0u, d);
        PG_LAUNCH_CHECK();
    }
    // Levels are queued in batches without the host reading their counts:
    // each level's kernels read them from L[j] and the last one writes
    // L[j + 1]; grids are sized for bounds on them (a level has at most
    // twice the splitting entries of the one above), and the node arrays
    // are reserved for the batch's worst case.  The host reads the counts
    // back once per batch.
    constexpr int kBatch = 16;
    DevBuf lbuf(s), sbuf(s);
    PG_TRY(lbuf.alloc(sizeof(Level) * (kBatch + 1)));
    Level* Ld = lbuf.as<Level>();
    const int64_t smax = std::max<int64_t>((int64_t)cmax + 1, 2 * (int64_t)amax);
    PG_TRY(sbuf.alloc(sizeof(uint64_t) * (size_t)scan_partials(smax)));
    uint32_t* sums32 = sbuf.as<uint32_t>();
    uint64_t* sums64 = sbuf.as<uint64_t>();
    hipLaunchKernelGGL(level_init_kernel, dim3(1), dim3(64), 0, s, Ld, tot32, cst[0]);
    PG_LAUNCH_CHECK();
    auto grid_cap = [](uint64_t blocks, uint64_t cap) {
        return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks, cap));
    };
    const unsigned mgrid = grid_cap(cdiv((int64_t)(2 * rmax), kNT / kWave), 512);

    uint32_t* kcur = ka.as<uint32_t>();
    int32_t* icur = ia.as<int32_t>();
    uint32_t* knext = kb.as<uint32_t>();
    int32_t* inext = ib.as<int32_t>();
    int64_t nodes = 1, leaves = 0;
    T->lvl.assign(1, 0);
    T->lvl.push_back(1);
    int depth = 0;  // depth of the current entries' nodes
    int cur = 0;
    // bounds on the batch's first level: its splitting entries, all entries
    uint64_t a0 = n > 0 ? 1 : 0, e0 = n > 0 ? 1 : 0;
    bool first = true, done = false;
    std::vector<Level> hl(kBatch + 1);
    while (!done) {
        // level j of a batch adds its 2 As_j children and resets the boxes
        // of up to 4 As_j children of the next level
        auto need_upto = [&](int B) {
            size_t nd = (size_t)nodes, a = (size_t)a0, need = 0;
            for (int j = 0; j < B; j++) {
                need = std::max(need, nd + 6 * a + 2);
                nd += 2 * a;
                a = std::min(2 * a, amax);
            }
            return need;
        };
        const size_t need1 = need_upto(1);
        PG_TRY(gxn.reserve(need1, nodes));
        PG_TRY(gkey.reserve(need1 * 2 * d, (nodes + 2 * (size_t)a0) * 2 * d));
        PG_TRY(glo.reserve(need1, nodes));
        PG_TRY(gcnt.reserve(need1, nodes));
        const size_t cap = std::min(std::min(gxn.cap, gkey.cap / (2 * (size_t)d)), std::min(glo.cap, gcnt.cap));
        int B = 1;
        while (B < kBatch && need_upto(B + 1) <= cap) B++;
        N = Nodes{gxn.p, gkey.p, glo.p, gcnt.p};
        uint64_t a = a0, e = e0;
        int c = cur;
        uint32_t *kc = kcur, *kn = knext;
        int32_t *ic = icur, *in = inext;
        for (int j = 0; j < B; j++) {
            const Level* Lj = Ld + j;
            const Entries& E = ent[c];
            const Entries& X = ent[c ^ 1];
            const uint64_t cb = std::min<uint64_t>(cmax, (uint64_t)(nn / kCH) + e + 1);
            const unsigned cgrid = grid_cap(cdiv((int64_t)cb, kNT / kWave), 4096);
            hipLaunchKernelGGL(chunk_count_kernel, dim3(cgrid), dim3(kNT), 0, s, E, cst[c], Lj, kc, n, c2e,
                               lcnt, d, rbase, rentry, rcount, rbuf.as<uint32_t>());
            PG_LAUNCH_CHECK();
            PG_TRY(exclusive_scan_u32_dev(lcnt, lcnt, &Lj->C, 1, 1, (int64_t)cb + 1, nullptr, false, sums32, s));
            uint32_t* rep = rbuf.as<uint32_t>();
            switch (d) {
                case 1: launch_scatter<1>(cgrid, s, E, N, cst[c], lcnt, c2e, Lj, rbase, rep, leaf, d, rw, ifl, kc, ic, kn, in, n, T); break;
                case 2: launch_scatter<2>(cgrid, s, E, N, cst[c], lcnt, c2e, Lj, rbase, rep, leaf, d, rw, ifl, kc, ic, kn, in, n, T); break;
                case 3: launch_scatter<3>(cgrid, s, E, N, cst[c], lcnt, c2e, Lj, rbase, rep, leaf, d, rw, ifl, kc, ic, kn, in, n, T); break;
                case 4: launch_scatter<4>(cgrid, s, E, N, cst[c], lcnt, c2e, Lj, rbase, rep, leaf, d, rw, ifl, kc, ic, kn, in, n, T); break;
                case 5: launch_scatter<5>(cgrid, s, E, N, cst[c], lcnt, c2e, Lj, rbase, rep, leaf, d, rw, ifl, kc, ic, kn, in, n, T); break;
                default: launch_scatter<8>(cgrid, s, E, N, cst[c], lcnt, c2e, Lj, rbase, rep, leaf, d, rw, ifl, kc, ic, kn, in, n, T); break;
            }
            PG_LAUNCH_CHECK();
            hipLaunchKernelGGL(merge_replicas_kernel, dim3(mgrid), dim3(kNT), 0, s, rep, rentry, rcount, Lj, d,
                               gkey.p);
            PG_LAUNCH_CHECK();
            const unsigned agrid = grid_cap(cdiv((int64_t)a, kNT), 2048);
            const unsigned a2grid = grid_cap(cdiv(2 * (int64_t)a, kNT), 2048);
            hipLaunchKernelGGL(split_nodes_kernel, dim3(agrid), dim3(kNT), 0, s, E, N, cst[c], lcnt, Lj, leaf,
                               d, ifl, flags, cst[c ^ 1], rcount);
            PG_LAUNCH_CHECK();
            PG_TRY(exclusive_scan_u64_dev(flags, fpre, &Lj->As, 2, 0, 2 * (int64_t)a, ftot, false, sums64, s));
            hipLaunchKernelGGL(emit_kernel, dim3(a2grid), dim3(kNT), 0, s, E, X, N, flags, fpre, ftot, Lj,
                               depth + j + 1, d, ifl, rule, cst[c ^ 1]);
            PG_LAUNCH_CHECK();
            // chunk starts of the next level (entries past its count hold 0)
            PG_TRY(exclusive_scan_u32_dev(cst[c ^ 1], cst[c ^ 1], &Lj->As, 2, 0, 2 * (int64_t)a, nullptr, true,
                                          sums32, s));
            hipLaunchKernelGGL(level_advance_kernel, dim3(1), dim3(64), 0, s, Ld + j, ftot, cst[c ^ 1]);
            PG_LAUNCH_CHECK();
            e = std::min<uint64_t>(2 * a, amax);
            a = e;
            c ^= 1;
            std::swap(kc, kn);
            std::swap(ic, in);
        }
        PG_HIP(hipMemcpyAsync(hl.data(), Ld, sizeof(Level) * (B + 1), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        if (first) {
            leaves = hl[0].As == 0 ? 1 : 0;
            first = false;
        }
        if (depth > (1 << 16))
            return fail(PG_ERR_DEVICE, "spatial-median build: no end after 65536 levels");
        for (int j = 0; j < B && !done; j++) {
            const Level& L0 = hl[j];
            if (L0.As == 0) {
                done = true;  // nothing splits (a copy-only level did its copies)
                break;
            }
            nodes += 2 * (int64_t)L0.As;
            leaves += 2 * (int64_t)L0.As - hl[j + 1].As;
            T->lvl.push_back(nodes);
            depth++;
            cur ^= 1;
            std::swap(kcur, knext);
            std::swap(icur, inext);
        }
        if (!done) {
            a0 = hl[B].As;
            e0 = (uint64_t)hl[B].As + hl[B].Ac;
            if (e0 == 0) done = true;
            else PG_HIP(hipMemcpyAsync(Ld, Ld + B, sizeof(Level), hipMemcpyDeviceToDevice, s));
        }
    }
    const int levels = (int)T->lvl.size() - 1;
    T->L = levels;
    T->nnodes = nodes;
    T->nleaves = leaves;

    // leaf order: subtree leaf counts bottom-up, then spans top-down
    DevBuf lv(s);
    PG_TRY(lv.alloc(sizeof(uint32_t) * 2 * (size_t)nodes));
    uint32_t* nlv = lv.as<uint32_t>();
    uint32_t* jlo = nlv + nodes;
    for (int l = levels - 1; l >= 0; l--) {
        const uint32_t first = (uint32_t)T->lvl[l], count = (uint32_t)(T->lvl[l + 1] - T->lvl[l]);
        hipLaunchKernelGGL(leaf_count_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s, gxn.p, first,
                           count, nlv);
        PG_LAUNCH_CHECK();
    }
    PG_TRY(dalloc(&T->xspan, (size_t)nodes, s));
    PG_TRY(dalloc(&T->loff, (size_t)leaves + 1, s));
    PG_TRY(dalloc(&T->lnode, (size_t)leaves, s));
    for (int l = 0; l < levels; l++) {
        const uint32_t first = (uint32_t)T->lvl[l], count = (uint32_t)(T->lvl[l + 1] - T->lvl[l]);
        hipLaunchKernelGGL(leaf_index_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s, gxn.p, first,
                           count, nlv, jlo, glo.p, T->xspan, T->loff, T->lnode);
        PG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, s, T->loff + leaves, n);
    PG_LAUNCH_CHECK();
    PG_TRY(dalloc(&T->nbox, (size_t)nodes * 2 * d, s));
    hipLaunchKernelGGL(node_box_kernel, dim3(cdiv(nodes * 2 * d, kNT)), dim3(kNT), 0, s, gkey.p,
                       gcnt.p, nodes, d, ifl, T->nbox);
    PG_LAUNCH_CHECK();
    T->xn = gxn.release();
    return PG_OK;
}

}  // namespace pg
