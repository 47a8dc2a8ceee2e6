// Batched uneven point clouds: thousands of independent float32 clouds are
// built and queried (all-points k-NN within each cloud) in ONE persistent
// launch driven by an atomic work queue, plus a small reset launch before it.
// Both launches allocate nothing and read nothing back, so a caller may
// capture them in a HIP graph.
//
//   items [0, C)        build cloud order[t] (largest first) with one
//                       workgroup: top levels by workgroup radix select +
//                       stable partition in global memory (L2-resident),
//                       bottom subtrees in LDS (the same device functions as
//                       the static build); then publish ready[c] (release);
//   items [C, C + Q)    (cloud, block of 256 of its points): wait for
//                       ready[c] (acquire), one point per lane, the static
//                       search (search.hpp) over the cloud's own tree.
//
// Build items precede every query item in the queue, so a workgroup that
// waits for a cloud waits for a workgroup that is already running: the wait
// always ends.  It is bounded anyway and reports a timeout in the workspace.
//
// The autotuner times leaf sizes {8, 16, 32} x workgroups per compute unit
// {2, 4} x queries per lane and item {1, 4} (64 or 256 queries per wave) x
// k-list placement {registers, LDS} on the caller's data and keeps the
// fastest per workload key; every choice returns identical results (the k-NN
// result depends neither on the tree nor on where the list lives).
#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "build.hpp"
#include "build_dev.hpp"
#include "knn.hpp"
#include "scan.hpp"
#include "search.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = kBuildNT;   // 256
constexpr int kQB = kNT;        // queries per query item
constexpr uint32_t kSpinLimit = 1u << 26;

struct CloudDesc {
    int64_t row;    // first global row of the cloud
    int64_t pts;    // element offset of its coordinate planes [d][n] (and key scratch)
    int64_t split;  // offset of its split array [2^L]
    int64_t bbox;   // offset of its leaf boxes [2^L][2d]
    int32_t n, L, ls, pad;
};

struct BatchParams {
    const uint32_t* points;  // [N][d] float32 bits
    int32_t* out_idx;        // [N][k]
    float* out_d2;           // [N][k]
    uint32_t* queue;         // [0] next item, [1] error flags
    uint32_t* ready;         // [C]
    const int32_t* order;    // [C] clouds by descending size
    const int64_t* qstart;   // [C+1] first query item of order[t]
    const CloudDesc* desc;   // [C]
    uint32_t* pts;           // coordinate planes pool
    uint32_t* keys;          // key scratch pool (same layout)
    int32_t* pidx;           // [N] leaf order -> local row
    int32_t* pidx2;          // [N] scratch
    uint32_t* split;         // split pool
    uint32_t* bbox;          // box pool
    uint32_t* rec;           // [N][rw] packed leaf records
    int64_t total_items;
    int32_t C, d, k, S;
    int32_t lq;  // queries each lane searches per query item
    // separate query sets (null queries: every point queries its own cloud)
    const uint32_t* queries;  // [M][d] float32 bits
    const int64_t* qoff;      // [C+1] cloud c's queries are rows [qoff[c], qoff[c+1])
    const int64_t* qitems;    // [C+1] first query item of order[t]
};

__global__ void batch_reset_kernel(uint32_t* queue, uint32_t* ready, int C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) queue[i] = 0;
    for (int c = i; c < C; c += gridDim.x * blockDim.x) ready[c] = 0;
}

__device__ inline void build_cloud(const BatchParams& P, int c, uint32_t* sm) {
    const CloudDesc D = P.desc[c];
    const int64_t n = D.n;
    const int d = P.d;
    uint32_t* outp = P.pts + D.pts;
    uint32_t* scr = P.keys + D.pts;
    int32_t* oidx = P.pidx + D.row;
    int32_t* sidx = P.pidx2 + D.row;
    uint32_t* split = P.split + D.split;
    uint32_t* bbox = P.bbox + D.bbox;
    if (n > 0) {
        // ingest: rows -> key planes (in the output planes), -0.0 -> +0.0
        for (int64_t e = threadIdx.x; e < n; e += kNT) {
            for (int cc = 0; cc < d; cc++) {
                uint32_t b = P.points[(D.row + e) * d + cc];
                if (b == 0x80000000u) b = 0;
                outp[(int64_t)cc * n + e] = coord_to_key(b, true);
            }
            oidx[e] = (int32_t)e;
        }
        __syncthreads();
        uint32_t* cur = outp;
        int32_t* cur_i = oidx;
        uint32_t* oth = scr;
        int32_t* oth_i = sidx;
        for (int l = 0; l < D.ls; l++) {
            const int cdim = l % d;
            for (int64_t j = 0; j < ((int64_t)1 << l); j++) {
                const int64_t lo = node_start(n, l, j), hi = node_start(n, l, j + 1);
                const int64_t mid = node_start(n, l + 1, 2 * j + 1);
                uint32_t mn, mx;
                block_minmax(cur + (int64_t)cdim * n, lo, hi, sm, &mn, &mx);
                const int sb = mn == mx ? 0 : 32 - __clz(mn ^ mx);
                const uint32_t low = sb >= 32 ? 0xffffffffu : ((1u << sb) - 1u);
                block_node_split(cur, cur_i, oth, oth_i, d, cdim, n, lo, hi, mid, mn & ~low, sb,
                                 &split[((int64_t)1 << l) + j], true, sm);
                __syncthreads();
            }
            uint32_t* t = cur; cur = oth; oth = t;
            int32_t* ti = cur_i; cur_i = oth_i; oth_i = ti;
        }
        for (int64_t j0 = 0; j0 < ((int64_t)1 << D.ls); j0++)
            block_subtree(cur, cur_i, n, d, D.L, D.ls, j0, P.S, true, outp, oidx, split, bbox,
                          P.rec + D.row * record_words(d), sm);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&P.ready[c], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// One query item: the cloud's points [blk * kQB * lq, ...), lane t taking
// points t, t + kQB, ... (lq of them); with separate query sets, the cloud's
// queries in the same way.  LDSL: the k-list lives in LDS (sm).
template <int MD, int KT, bool EX, bool LDSL>
__device__ inline void query_item(const BatchParams& P, int64_t q, int* s_ok, uint32_t* sm) {
    // item -> position t in the size order (binary search over the item starts)
    const int64_t* qs = P.queries ? P.qitems : P.qstart;
    int lo = 0, hi = P.C;  // qs[lo] <= q < qs[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (qs[mid] <= q) lo = mid;
        else hi = mid;
    }
    const int c = P.order[lo];
    const int64_t blk = q - qs[lo];
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        int ok = 1;
        while (__hip_atomic_load(&P.ready[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            __builtin_amdgcn_s_sleep(8);
            if (++spins > kSpinLimit) {
                atomicOr(&P.queue[1], 1u);
                ok = 0;
                break;
            }
        }
        *s_ok = ok;
    }
    __syncthreads();
    const int ok = *s_ok;
    __syncthreads();
    if (!ok) return;
    (void)__hip_atomic_load(&P.ready[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const CloudDesc D = P.desc[c];
    const int d = P.d, k = P.k;
    const TreeView tv{D.n, d, D.L, record_words(d), P.pts + D.pts, P.pidx + D.row,
                      P.split + D.split, P.bbox + D.bbox, P.rec + D.row * record_words(d)};
    using M = Metric<float>;
    const bool sep = P.queries != nullptr;
    const int64_t mq = sep ? P.qoff[c + 1] - P.qoff[c] : D.n;
    for (int r = 0; r < P.lq; r++) {
        const int64_t i = (blk * P.lq + r) * kQB + threadIdx.x;
        if (i >= mq) break;
        float q_[MD];
        uint32_t start;
        int64_t row;
        if (sep) {
            row = P.qoff[c] + i;
#pragma unroll
            for (int cc = 0; cc < MD; cc++) q_[cc] = cc < d ? M::load(P.queries[row * d + cc]) : 0.0f;
            start = 0;  // from the root
        } else {
#pragma unroll
            for (int cc = 0; cc < MD; cc++) q_[cc] = cc < d ? M::load(tv.pts[(int64_t)cc * D.n + i]) : 0.0f;
            start = (1u << D.L) + leaf_of(D.n, D.L, i);
            row = D.row + tv.pidx[i];
        }
        if constexpr (LDSL) {
            LdsList<KT, EX> kl;
            kl.init(reinterpret_cast<uint64_t*>(sm) + threadIdx.x, kNT);
            kd_search<float, MD>(tv, PlainIds{}, q_, d, kl, k, start);
            for (int s = 0; s < (EX ? KT : k); s++) {
                const uint64_t x = kl.at(s);
                const int32_t id = kl.id_of(x);
                P.out_idx[row * k + s] = id < 0 ? -1 : (int32_t)(D.row + id);
                P.out_d2[row * k + s] = kl.dist_of(x);
            }
        } else {
            PackedList<float, KT, EX> kl;
            kl.init(32);
            kd_search<float, MD>(tv, PlainIds{}, q_, d, kl, k, start);
#pragma unroll
            for (int s = 0; s < KT; s++) {
                if (EX || s < k) {
                    const int32_t id = kl.id_of(kl.key[s]);
                    P.out_idx[row * k + s] = id < 0 ? -1 : (int32_t)(D.row + id);
                    P.out_d2[row * k + s] = kl.dist_of(kl.key[s]);
                }
            }
        }
    }
}

template <int MD, int KT, bool EX, bool LDSL>
__global__ void __launch_bounds__(kNT) batch_kernel(BatchParams P) {
    extern __shared__ __align__(16) uint32_t sm[];
    __shared__ int s_item;
    __shared__ int s_ok;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&P.queue[0], 1u);
        __syncthreads();
        const int64_t it = s_item;
        __syncthreads();
        if (it >= P.total_items) break;
        if (it < P.C) build_cloud(P, P.order[it], sm);
        else query_item<MD, KT, EX, LDSL>(P, it - P.C, &s_ok, sm);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Backward of L = sum_{i,r} g[i,r] D(q_i, x_{idx[i,r]}) with fixed neighbours.
// ---------------------------------------------------------------------------
__global__ void grad_q_kernel(const float* __restrict__ q, const float* __restrict__ x,
                              int64_t m, int64_t n, int d, int k, const int32_t* __restrict__ idx,
                              const float* __restrict__ g, float* __restrict__ gq) {
    const int64_t t = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (t >= m * d) return;
    const int64_t i = t / d;
    const int c = (int)(t % d);
    const float qc = q[i * d + c];
    float acc = 0.0f;
    for (int r = 0; r < k; r++) {
        const int32_t j = idx[i * k + r];
        if (j < 0 || j >= n) continue;
        acc += 2.0f * g[i * k + r] * (qc - x[(int64_t)j * d + c]);
    }
    gq[t] = acc;
}

// Atomic form: every pair subtracts its term from grad_p[j] with a float
// atomic (the order of the adds, hence the rounding, varies between runs).
__global__ void grad_x_atomic_kernel(const float* __restrict__ q, const float* __restrict__ x,
                                     int64_t P, int64_t n, int d, int k,
                                     const int32_t* __restrict__ idx, const float* __restrict__ g,
                                     float* __restrict__ gx) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= P) return;
    const int32_t j = idx[p];
    if (j < 0 || j >= n) return;
    const int64_t i = p / k;
    const float w = 2.0f * g[p];
    for (int c = 0; c < d; c++)
        atomicAdd(&gx[(int64_t)j * d + c], -w * (q[i * d + c] - x[(int64_t)j * d + c]));
}

__global__ void zero_f32_kernel(float* __restrict__ a, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (t < count) a[t] = 0.0f;
}

__global__ void pair_count_kernel(const int32_t* __restrict__ idx, int64_t P, int64_t n,
                                  uint32_t* __restrict__ cnt) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p < P && idx[p] >= 0 && idx[p] < n) atomicAdd(&cnt[idx[p]], 1u);
}

__global__ void pair_fill_kernel(const int32_t* __restrict__ idx, int64_t P, int64_t n,
                                 const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                                 uint32_t* __restrict__ list) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= P) return;
    const int32_t j = idx[p];
    if (j < 0 || j >= n) return;
    list[start[j] + atomicAdd(&cursor[j], 1u)] = (uint32_t)p;
}

// Puts each point's pair list in ascending pair order (rank by counting), so
// the sums below add in a fixed order.
__global__ void pair_order_kernel(const uint32_t* __restrict__ list,
                                  const uint32_t* __restrict__ total,
                                  const int32_t* __restrict__ idx,
                                  const uint32_t* __restrict__ start,
                                  const uint32_t* __restrict__ cnt, uint32_t* __restrict__ ordered) {
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (s >= (int64_t)*total) return;  // only the filled entries
    const uint32_t p = list[s];
    const int32_t j = idx[p];
    const uint32_t b = start[j], e = b + cnt[j];
    uint32_t rank = 0;
    for (uint32_t t = b; t < e; t++) rank += list[t] < p;
    ordered[b + rank] = p;
}

__global__ void grad_x_kernel(const float* __restrict__ q, const float* __restrict__ x,
                              int64_t n, int d, int k, const float* __restrict__ g,
                              const uint32_t* __restrict__ start, const uint32_t* __restrict__ cnt,
                              const uint32_t* __restrict__ ordered, int accumulate,
                              float* __restrict__ gx) {
    const int64_t t = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (t >= n * d) return;
    const int64_t j = t / d;
    const int c = (int)(t % d);
    const float xc = x[t];
    const uint32_t b = start[j], e = b + cnt[j];
    float acc = 0.0f;
    for (uint32_t s = b; s < e; s++) {
        const uint32_t p = ordered[s];
        const int64_t i = p / (uint32_t)k;
        acc += 2.0f * g[p] * (q[i * d + c] - xc);
    }
    gx[t] = accumulate ? gx[t] - acc : -acc;
}

// ---------------------------------------------------------------------------
// Batched backward in leaf order.  The queries of a cloud are taken in the
// order of its tree's leaves (work items of kBwdItem positions), so the
// neighbours of an item's queries lie mostly in the window of positions
// [p0 - kBwdMargin, p0 + kBwdItem + kBwdMargin): their terms are summed in
// LDS and the window is stored whole to the item's slot (plain stores); the
// few pairs whose neighbour lies outside it are listed in LDS and their terms
// go to global row accumulators after the loop (a global atomic inside the
// loop would make every later load of the wave wait for it).  A finishing pass adds,
// for each position, its own item's window entry and the one neighbouring
// item's window that also covers it.  All sums are integer (int64 fixed
// point, each term rounded once), so they do not depend on the order of the
// adds: the result is deterministic.  Scale: every term is at most
// T = 2 max|g| sqrt(max D) in magnitude (with the forward's D); terms are
// multiplied by 2^(30 - ceil(log2 T)) and rounded to int32, so a sum of up
// to 2^32 of them fits in int64.
// ---------------------------------------------------------------------------
constexpr int kBwdItem = 1024;                    // leaf positions per backward work item
constexpr int kBwdMargin = 448;                   // window margin on each side (<= kBwdItem / 2)
static_assert(2 * kBwdMargin <= kBwdItem, "a position lies in at most one neighbour's window");
constexpr int kBwdWin = kBwdItem + 2 * kBwdMargin;  // window positions
constexpr int kBwdSpill = 1536;                   // out-of-window pairs deferred per item
// the spilled pairs' records ((d + 1) words each) reuse the window's LDS
static_assert(kBwdSpill * 2 * 4 <= kBwdWin * 8, "spill records must fit the window (d = 1)");

__device__ inline int cloud_of_item(const int64_t* __restrict__ start, int C, int64_t it) {
    int lo = 0, hi = C;  // start[lo] <= it < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= it) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Work items are dealt to the XCDs in contiguous eighths (xcd_block), so the
// items of a cloud run on one XCD and its points stay in that XCD's L2.
__device__ inline int64_t bwd_item() { return xcd_block(); }

// inv[row] = global leaf position of the row (its cloud's first row plus its
// position in the cloud's leaf order).  With rrec (d <= 3): rrec[row] = {the
// row's coordinates, its global leaf position}, so that the main pass
// gathers a neighbour's coordinates and window slot with one 16-byte load.
__global__ void bwd_inv_kernel(const CloudDesc* __restrict__ desc, const int64_t* __restrict__ start,
                               int C, int64_t items, const int32_t* __restrict__ pidx,
                               const float* __restrict__ x, int d, int32_t* __restrict__ inv,
                               uint4* __restrict__ rrec) {
    const int64_t it = bwd_item();
    if (it >= items) return;
    const int c = cloud_of_item(start, C, it);
    const CloudDesc D = desc[c];
    const int64_t p0 = (it - start[c]) * kBwdItem;
    for (int e = threadIdx.x; e < kBwdItem; e += kNT) {
        const int64_t pos = p0 + e;
        if (pos >= D.n) break;
        const int64_t row = D.row + pidx[D.row + pos];
        if (rrec) {
            uint32_t w[3] = {0u, 0u, 0u};
            for (int cc = 0; cc < d; cc++) w[cc] = __float_as_uint(x[row * d + cc]);
            rrec[row] = make_uint4(w[0], w[1], w[2], (uint32_t)(D.row + pos));
        } else {
            inv[row] = (int32_t)(D.row + pos);
        }
    }
}

// Per cloud: maxes[2c] = max |g|, maxes[2c+1] = max D over the cloud's pairs
// with a neighbour (the padding of a cloud smaller than k has D = +inf); as
// float bits: non-negative floats order like their bits, and a NaN |g|
// orders above every finite value.  One workgroup per backward item (its
// rows' pairs are contiguous).
__global__ void __launch_bounds__(kNT)
bwd_scale_kernel(const CloudDesc* __restrict__ desc, const int64_t* __restrict__ start, int C,
                 int64_t items, int k, const float* __restrict__ g, const float* __restrict__ d2,
                 uint32_t* __restrict__ maxes) {
    __shared__ uint32_t red[2][kNT / kWave];
    const int64_t it = bwd_item();
    if (it >= items) return;
    const int c = cloud_of_item(start, C, it);
    const CloudDesc D = desc[c];
    const int64_t p0 = (it - start[c]) * kBwdItem;
    const int64_t r1 = D.row + (p0 + kBwdItem < D.n ? p0 + kBwdItem : (int64_t)D.n);
    uint32_t mg = 0, md = 0;
    for (int64_t p = (D.row + p0) * k + threadIdx.x; p < r1 * k; p += kNT) {
        const float dp = d2[p];
        if (!(dp < __builtin_huge_valf())) continue;
        const uint32_t a = __float_as_uint(fabsf(g[p])), b = __float_as_uint(dp);
        mg = a > mg ? a : mg;
        md = b > md ? b : md;
    }
    mg = wave_max_u32(mg);
    md = wave_max_u32(md);
    if (lane_id() == 0) {
        red[0][threadIdx.x / kWave] = mg;
        red[1][threadIdx.x / kWave] = md;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kNT / kWave; w++) {
            mg = red[0][w] > mg ? red[0][w] : mg;
            md = red[1][w] > md ? red[1][w] : md;
        }
        mg = red[0][0] > mg ? red[0][0] : mg;
        md = red[1][0] > md ? red[1][0] : md;
        atomicMax(&maxes[2 * c], mg);
        atomicMax(&maxes[2 * c + 1], md);
    }
}

// Power-of-two scale of cloud c's terms (see above); 1 when every term is 0;
// 0 when the bound is not a finite float (NaN or infinite gradients, or
// terms beyond 3e38): that cloud's neighbour sums are then NaN.
__device__ inline float bwd_scale(const uint32_t* maxes, int c) {
    const float t = 2.0f * __uint_as_float(maxes[2 * c]) * sqrtf(__uint_as_float(maxes[2 * c + 1]));
    if (!(t <= 3.0e38f)) return 0.0f;
    if (!(t > 0.0f)) return 1.0f;
    int e = 0;
    (void)frexpf(t, &e);  // t < 2^e
    return ldexpf(1.0f, 30 - e);
}

// One work item: kBwdItem leaf positions of one cloud.  Lane queries i (in
// leaf order) accumulate their own gradient in registers (fixed order) and
// write it to gl at their global leaf position; the neighbour terms go to the
// LDS window, or the pair to the spill list; the window is then stored to the
// item's slot of wbuf and the spilled pairs' terms are added to acc (indexed
// by global leaf position).
template <int MD>
__global__ void __launch_bounds__(kNT)
bwd_main_kernel(const CloudDesc* __restrict__ desc, const int64_t* __restrict__ start, int C,
                int64_t items, const int32_t* __restrict__ pidx, const int32_t* __restrict__ inv,
                const uint4* __restrict__ rrec, const float* __restrict__ x, int d_, int k,
                const int32_t* __restrict__ idx,
                const float* __restrict__ g, const uint32_t* __restrict__ maxes,
                unsigned long long* __restrict__ acc, unsigned long long* __restrict__ wbuf,
                float* __restrict__ gl) {
    extern __shared__ __align__(16) unsigned long long win[];  // [kBwdWin][d]
    __shared__ uint32_t spill[kBwdSpill];
    __shared__ uint32_t nspill;
    const int d = MD < 8 ? MD : d_;
    const int64_t it = bwd_item();
    if (it >= items) return;
    const int c = cloud_of_item(start, C, it);
    const CloudDesc D = desc[c];
    const int64_t p0 = (it - start[c]) * kBwdItem;
    const int64_t org = p0 - kBwdMargin;  // position of window entry 0
    for (int e = threadIdx.x; e < kBwdWin * d; e += kNT) win[e] = 0ull;
    if (threadIdx.x == 0) nspill = 0;
    __syncthreads();
    const float scale = bwd_scale(maxes, c);  // 0: the terms are not rounded (the sums become NaN)
    for (int e = threadIdx.x; e < kBwdItem; e += kNT) {
        const int64_t pos = p0 + e;
        if (pos >= D.n) break;
        const int64_t i = D.row + pidx[D.row + pos];
        float xi[MD], gq[MD];
#pragma unroll
        for (int cc = 0; cc < MD; cc++) {
            xi[cc] = (MD < 8 || cc < d) ? x[i * d + cc] : 0.0f;
            gq[cc] = 0.0f;
        }
        // the row's neighbours four at a time: 16-byte loads of the index and
        // gradient rows (each row is read once, not word by word across the
        // loop), then the four neighbours' coordinates and leaf positions
        for (int r0 = 0; r0 < k; r0 += 4) {
            int32_t jj[4];
            float gg[4];
            if ((k & 3) == 0) {
                const int4 jv = *reinterpret_cast<const int4*>(idx + i * k + r0);
                const float4 gv = *reinterpret_cast<const float4*>(g + i * k + r0);
                jj[0] = jv.x; jj[1] = jv.y; jj[2] = jv.z; jj[3] = jv.w;
                gg[0] = gv.x; gg[1] = gv.y; gg[2] = gv.z; gg[3] = gv.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    jj[u] = r0 + u < k ? idx[i * k + r0 + u] : -1;
                    gg[u] = r0 + u < k ? g[i * k + r0 + u] : 0.0f;
                }
            }
            float xj[4][MD];
            int64_t w[4], pg[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int32_t j = jj[u] >= 0 ? jj[u] : (int32_t)i;  // a safe row for the loads
                int64_t pj;
                if constexpr (MD <= 3) {
                    const uint4 r = rrec[j];
                    const uint32_t rw[3] = {r.x, r.y, r.z};
#pragma unroll
                    for (int cc = 0; cc < MD; cc++) xj[u][cc] = __uint_as_float(rw[cc]);
                    pj = (int64_t)r.w;
                } else {
#pragma unroll
                    for (int cc = 0; cc < MD; cc++)
                        xj[u][cc] = (MD < 8 || cc < d) ? x[(int64_t)j * d + cc] : 0.0f;
                    pj = (uint32_t)inv[j];
                }
                // a neighbour of the same cloud inside the window sums in LDS
                const bool same = jj[u] >= 0 && j >= D.row && j < D.row + D.n;
                w[u] = same ? pj - D.row - org : -1;
                pg[u] = pj;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (jj[u] < 0) continue;
                const float gr = gg[u];
                if (scale == 0.0f) {  // the cloud's neighbour sums are NaN (bwd_finish_kernel)
#pragma unroll
                    for (int cc = 0; cc < MD; cc++) gq[cc] += 2.0f * gr * (xi[cc] - xj[u][cc]);
                    continue;
                }
                const bool in_win = w[u] >= 0 && w[u] < kBwdWin;
                int32_t t[MD];
#pragma unroll
                for (int cc = 0; cc < MD; cc++) {
                    const float diff = xi[cc] - xj[u][cc];
                    gq[cc] += 2.0f * gr * diff;
                    t[cc] = (int32_t)rintf(-2.0f * gr * diff * scale);
                }
                if (in_win) {
#pragma unroll
                    for (int cc = 0; cc < MD; cc++)
                        if (MD < 8 || cc < d)
                            atomicAdd(&win[w[u] * d + cc], (unsigned long long)(long long)t[cc]);
                } else {
                    const uint32_t sl = atomicAdd(&nspill, 1u);
                    if (sl < (uint32_t)kBwdSpill) {
                        spill[sl] = (uint32_t)(i * k + r0 + u);
                    } else {  // list full (only with pathological data): directly
#pragma unroll
                        for (int cc = 0; cc < MD; cc++)
                            if (MD < 8 || cc < d)
                                atomicAdd(&acc[pg[u] * d + cc], (unsigned long long)(long long)t[cc]);
                    }
                }
            }
        }
#pragma unroll
        for (int cc = 0; cc < MD; cc++)
            if (MD < 8 || cc < d) gl[(D.row + pos) * d + cc] = gq[cc];
    }
    __syncthreads();
    unsigned long long* slot = wbuf + it * kBwdWin * d;
    for (int e = threadIdx.x; e < kBwdWin * d; e += kNT) slot[e] = win[e];
    __syncthreads();
    // spilled pairs: terms into the (now free) window space, then the atomics
    const int ns = nspill < (uint32_t)kBwdSpill ? (int)nspill : kBwdSpill;
    int32_t* rec = reinterpret_cast<int32_t*>(win);  // [ns][d + 1]: j's global leaf position, terms
    for (int e = threadIdx.x; e < ns; e += kNT) {
        const uint32_t pp = spill[e];
        const int64_t i = pp / (uint32_t)k;
        const int32_t j = idx[pp];
        const float gr = g[pp];
        rec[e * (d + 1)] = (int32_t)(MD <= 3 ? rrec[j].w : (uint32_t)inv[j]);
        for (int cc = 0; cc < d; cc++) {
            const float diff = x[i * d + cc] - x[(int64_t)j * d + cc];
            rec[e * (d + 1) + 1 + cc] = (int32_t)rintf(-2.0f * gr * diff * scale);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ns * d; e += kNT) {
        const int q = e / d, cc = e - q * d;
        const int64_t pj = (uint32_t)rec[q * (d + 1)];
        atomicAdd(&acc[pj * d + cc], (unsigned long long)(long long)rec[q * (d + 1) + 1 + cc]);
    }
}

// Per item: each of its positions takes its own window entry, the entry of
// the neighbouring item of the same cloud whose window also covers it, if any
// (the previous item's below p0 + kBwdMargin, the next item's from
// p0 + kBwdItem - kBwdMargin on), and its accumulator (all in leaf order);
// gout[row] = its own gradient (gl, leaf order) + that sum / scale (NaN, and
// bit 1 of *flags, for a cloud whose scale is 0): one store per row.
__global__ void __launch_bounds__(kNT)
bwd_finish_kernel(const CloudDesc* __restrict__ desc, const int64_t* __restrict__ start, int C,
                  int64_t items, const int32_t* __restrict__ pidx, int d,
                  const unsigned long long* __restrict__ wbuf,
                  const unsigned long long* __restrict__ acc, const uint32_t* __restrict__ maxes,
                  const float* __restrict__ gl, uint32_t* __restrict__ flags, float* __restrict__ gout) {
    const int64_t b = bwd_item();
    if (b >= items) return;
    const int c = cloud_of_item(start, C, b);
    const CloudDesc D = desc[c];
    const int64_t b0 = start[c], b1 = start[c + 1];
    const int64_t p0 = (b - b0) * kBwdItem;
    const float scale = bwd_scale(maxes, c);
    const float inv_scale = scale > 0.0f ? 1.0f / scale : __builtin_nanf("");
    if (scale == 0.0f && threadIdx.x == 0) atomicOr(flags, 2u);
    const unsigned long long* own = wbuf + b * kBwdWin * d;
    for (int e = threadIdx.x; e < kBwdItem * d; e += kNT) {
        const int64_t pos = p0 + e / d;
        const int cc = e % d;
        if (pos >= D.n) break;
        const int64_t row = D.row + pidx[D.row + pos];
        long long v = (long long)own[(pos - (p0 - kBwdMargin)) * d + cc];
        if (pos < p0 + kBwdMargin) {
            if (b > b0) v += (long long)wbuf[(b - 1) * kBwdWin * d + (pos - (p0 - kBwdItem - kBwdMargin)) * d + cc];
        } else if (pos >= p0 + kBwdItem - kBwdMargin) {
            if (b + 1 < b1) v += (long long)wbuf[(b + 1) * kBwdWin * d + (pos - (p0 + kBwdItem - kBwdMargin)) * d + cc];
        }
        const int64_t gp = (D.row + pos) * d + cc;
        v += (long long)acc[gp];
        gout[row * d + cc] = gl[gp] + (float)((double)v * (double)inv_scale);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct BatchPlan {
    int C = 0, d = 0, leaf = 0, bpc = 0, S = 0, lq = 1, klist = PG_KLIST_VGPR;
    int64_t N = 0, total_items = 0;
    // workspace carve-up
    size_t bytes = 0;
    size_t o_queue = 0, o_ready = 0, o_order = 0, o_qstart = 0, o_desc = 0, o_pts = 0,
           o_keys = 0, o_pidx = 0, o_pidx2 = 0, o_split = 0, o_bbox = 0, o_rec = 0,
           o_qoff = 0, o_qitems = 0;
    // the query offsets last uploaded for pg_batch_knn, and their item count
    std::vector<int64_t> qoff;
    int64_t q_items = 0;
    std::vector<int32_t> order;
    std::vector<int64_t> qstart;
    std::vector<int64_t> bstart;  // first backward work item of cloud c (cloud order)
    std::vector<CloudDesc> desc;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static pg_status make_plan(const int64_t* offs, int C, int d, int leaf, int bpc, int lq, int klist,
                           BatchPlan& P) {
    P.C = C;
    P.d = d;
    P.leaf = leaf;
    P.bpc = bpc;
    P.lq = lq;
    P.klist = klist;
    P.S = subtree_capacity(d);
    P.desc.resize(C);
    int64_t pts = 0, split = 0, bbox = 0;
    for (int c = 0; c < C; c++) {
        const int64_t n = offs[c + 1] - offs[c];
        if (n < 0) return fail(PG_ERR_INVALID, "batch: offsets must be non-decreasing");
        if (n >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "batch: cloud too large");
        CloudDesc& D = P.desc[c];
        D.row = offs[c];
        D.n = (int32_t)n;
        D.L = tree_levels(n, leaf);
        int ls = 0;
        while (((n + ((int64_t)1 << ls) - 1) >> ls) > P.S) ls++;
        D.ls = ls;
        D.pad = 0;
        D.pts = pts;
        D.split = split;
        D.bbox = bbox;
        pts += (int64_t)d * n;
        split += (int64_t)1 << D.L;
        bbox += ((int64_t)1 << D.L) * 2 * d;
    }
    P.N = offs[C] - offs[0];
    if (offs[0] != 0) return fail(PG_ERR_INVALID, "batch: offsets[0] must be 0");
    if (P.N >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "batch: total points must be < 2^31");
    P.order.resize(C);
    std::iota(P.order.begin(), P.order.end(), 0);
    std::stable_sort(P.order.begin(), P.order.end(),
                     [&](int a, int b) { return P.desc[a].n > P.desc[b].n; });
    P.qstart.resize(C + 1);
    int64_t q = 0;
    for (int t = 0; t < C; t++) {
        P.qstart[t] = q;
        q += (P.desc[P.order[t]].n + (int64_t)kQB * lq - 1) / ((int64_t)kQB * lq);
    }
    P.qstart[C] = q;
    P.total_items = C + q;
    P.bstart.resize(C + 1);
    int64_t bi = 0;
    for (int c = 0; c < C; c++) {
        P.bstart[c] = bi;
        bi += (P.desc[c].n + kBwdItem - 1) / kBwdItem;
    }
    P.bstart[C] = bi;
    size_t o = 0;
    P.o_queue = o; o = align256(o + 16);
    P.o_ready = o; o = align256(o + 4 * (size_t)C);
    P.o_order = o; o = align256(o + 4 * (size_t)C);
    P.o_qstart = o; o = align256(o + 8 * (size_t)(C + 1));
    P.o_desc = o; o = align256(o + sizeof(CloudDesc) * (size_t)C);
    P.o_pts = o; o = align256(o + 4 * (size_t)(pts > 0 ? pts : 1));
    P.o_keys = o; o = align256(o + 4 * (size_t)(pts > 0 ? pts : 1));
    P.o_pidx = o; o = align256(o + 4 * (size_t)(P.N > 0 ? P.N : 1));
    P.o_pidx2 = o; o = align256(o + 4 * (size_t)(P.N > 0 ? P.N : 1));
    P.o_split = o; o = align256(o + 4 * (size_t)(split > 0 ? split : 1));
    P.o_bbox = o; o = align256(o + 4 * (size_t)(bbox > 0 ? bbox : 1));
    P.o_rec = o; o = align256(o + 4 * (size_t)record_words(d) * (size_t)(P.N > 0 ? P.N : 1));
    P.o_qoff = o; o = align256(o + 8 * (size_t)(C + 1));
    P.o_qitems = o; o = align256(o + 8 * (size_t)(C + 1));
    P.bytes = o;
    return PG_OK;
}

}  // namespace pg

struct pg_batch {
    pg::BatchPlan plan;
    uint8_t* ws = nullptr;
    bool owns = false;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    int64_t* bstart_dev = nullptr;  // plan.bstart on the device (first backward call)
};

namespace pg {
namespace {

template <int MD, int KT, bool EX>
pg_status launch_batch(pg_batch* b, const BatchParams& P, hipStream_t s) {
    const bool lds_list = b->plan.klist == PG_KLIST_LDS;
    size_t lds = subtree_lds_bytes(P.d, P.S);  // build items and LDS k-lists share it
    if (lds_list) lds = std::max(lds, sizeof(uint64_t) * KT * kNT);
    const unsigned grid = (unsigned)(b->num_cu * b->plan.bpc);
    hipLaunchKernelGGL(batch_reset_kernel, dim3(8), dim3(kNT), 0, s, P.queue, P.ready, P.C);
    PG_LAUNCH_CHECK();
    if (lds_list)
        hipLaunchKernelGGL((batch_kernel<MD, KT, EX, true>), dim3(grid), dim3(kNT), lds, s, P);
    else
        hipLaunchKernelGGL((batch_kernel<MD, KT, EX, false>), dim3(grid), dim3(kNT), lds, s, P);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

template <int MD>
pg_status batch_k(pg_batch* b, const BatchParams& P, hipStream_t s) {
    const int k = P.k;
    if (k == 5) return launch_batch<MD, 5, true>(b, P, s);
    if (k == 10) return launch_batch<MD, 10, true>(b, P, s);
    if (k == 16) return launch_batch<MD, 16, true>(b, P, s);
    if (k <= 2) return launch_batch<MD, 2, false>(b, P, s);
    if (k <= 4) return launch_batch<MD, 4, false>(b, P, s);
    if (k <= 8) return launch_batch<MD, 8, false>(b, P, s);
    if (k <= 16) return launch_batch<MD, 16, false>(b, P, s);
    if (k <= 32) return launch_batch<MD, 32, false>(b, P, s);
    return launch_batch<MD, 64, false>(b, P, s);
}

std::mutex g_tune_mu;
std::map<std::tuple<std::string, int64_t, int64_t, int, int>, pg_tune> g_tune_cache;

// The tuner's cache key: the device (its name and ISA), the cloud count and
// the point count each rounded up to a power of two, d and k.
using TuneKey = std::tuple<std::string, int64_t, int64_t, int, int>;

inline int64_t pow2_at_least(int64_t v) {
    int64_t b = 1;
    while (b < v) b <<= 1;
    return b;
}

std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string tag = std::string(prop.gcnArchName) + "/" + prop.name;
    for (char& ch : tag)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    return tag;
}

// PG_TUNE_CACHE names a text file that keeps the tuner's choices across
// processes: one line per key, "device clouds points d k leaf blocks_per_cu
// lane_queries klist" (the counts as their power-of-two buckets).  Lines
// that do not parse, or whose choice is out of range, are ignored; a new
// choice is appended.
bool tune_file_lookup(const char* path, const TuneKey& key, pg_tune* out) {
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string dev;
        int64_t c = 0, n = 0;
        int d = 0, k = 0;
        pg_tune t{};
        if (!(ls >> dev >> c >> n >> d >> k >> t.leaf >> t.blocks_per_cu >> t.lane_queries >> t.klist)) continue;
        if (t.leaf < 1 || t.leaf > 64 || t.blocks_per_cu < 1 || t.blocks_per_cu > 16 || t.lane_queries < 1 ||
            t.lane_queries > 8 || (t.klist != PG_KLIST_VGPR && t.klist != PG_KLIST_LDS))
            continue;
        if (TuneKey(dev, c, n, d, k) == key) {
            *out = t;  // the last matching line wins
            found = true;
        }
    }
    return found;
}

void tune_file_append(const char* path, const TuneKey& key, const pg_tune& t) {
    std::ofstream o(path, std::ios::app);
    if (!o) return;
    o << std::get<0>(key) << ' ' << std::get<1>(key) << ' ' << std::get<2>(key) << ' ' << std::get<3>(key) << ' '
      << std::get<4>(key) << ' ' << t.leaf << ' ' << t.blocks_per_cu << ' ' << t.lane_queries << ' ' << t.klist
      << '\n';
}

}  // namespace
}  // namespace pg

using namespace pg;

extern "C" {

pg_status pg_batch_workspace(const int64_t* offsets_host, int32_t n_clouds, int32_t d,
                             const pg_tune* tune, size_t* bytes) {
    if (!offsets_host || !bytes) return fail(PG_ERR_INVALID, "pg_batch_workspace: NULL pointer");
    if (n_clouds < 1) return fail(PG_ERR_INVALID, "pg_batch_workspace: n_clouds must be >= 1");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_batch_workspace: d must be in [1, 8]");
    const int leaf = tune && tune->leaf ? tune->leaf : 16;
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_batch_workspace: leaf must be in [1, 64]");
    BatchPlan P;
    PG_TRY(make_plan(offsets_host, n_clouds, d, leaf, 4, 1, PG_KLIST_VGPR, P));
    *bytes = P.bytes;
    return PG_OK;
}

pg_status pg_batch_create(const int64_t* offsets_host, int32_t n_clouds, int32_t d,
                          const pg_tune* tune, void* workspace, size_t workspace_bytes,
                          void* stream, pg_batch** out) {
    if (!offsets_host || !out) return fail(PG_ERR_INVALID, "pg_batch_create: NULL pointer");
    if (n_clouds < 1) return fail(PG_ERR_INVALID, "pg_batch_create: n_clouds must be >= 1");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_batch_create: d must be in [1, 8]");
    const int leaf = tune && tune->leaf ? tune->leaf : 16;
    const int bpc = tune && tune->blocks_per_cu ? tune->blocks_per_cu : 4;
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_batch_create: leaf must be in [1, 64]");
    const int lq = tune && tune->lane_queries ? tune->lane_queries : 1;
    const int kl = tune && tune->klist ? tune->klist : PG_KLIST_VGPR;
    if (bpc < 1 || bpc > 16) return fail(PG_ERR_INVALID, "pg_batch_create: blocks_per_cu must be in [1, 16]");
    if (lq < 1 || lq > 8) return fail(PG_ERR_INVALID, "pg_batch_create: lane_queries must be in [1, 8]");
    if (kl != PG_KLIST_VGPR && kl != PG_KLIST_LDS)
        return fail(PG_ERR_INVALID, "pg_batch_create: klist must be PG_KLIST_VGPR or PG_KLIST_LDS");
    pg_batch* b = new (std::nothrow) pg_batch();
    if (!b) return fail(PG_ERR_NOMEM, "pg_batch_create: host allocation failed");
    pg_status st = make_plan(offsets_host, n_clouds, d, leaf, bpc, lq, kl, b->plan);
    if (st != PG_OK) { delete b; return st; }
    hipStream_t s = (hipStream_t)stream;
    b->stream = s;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) { delete b; return fail(PG_ERR_DEVICE, "pg_batch_create: device query failed"); }
    if (workspace) {
        if (workspace_bytes < b->plan.bytes) {
            delete b;
            return fail(PG_ERR_INVALID, "pg_batch_create: workspace too small (see pg_batch_workspace)");
        }
        b->ws = (uint8_t*)workspace;
    } else {
        void* p = nullptr;
        st = dmalloc(&p, b->plan.bytes, s);
        if (st != PG_OK) { delete b; return st; }
        b->ws = (uint8_t*)p;
        b->owns = true;
    }
    const BatchPlan& P = b->plan;
    // Static plan tables (order, query starts, descriptors) go to the workspace
    // once, here; the launches only read them.
    hipError_t e1 = hipMemcpyAsync(b->ws + P.o_order, P.order.data(), 4 * (size_t)P.C, hipMemcpyHostToDevice, s);
    hipError_t e2 = hipMemcpyAsync(b->ws + P.o_qstart, P.qstart.data(), 8 * (size_t)(P.C + 1), hipMemcpyHostToDevice, s);
    hipError_t e3 = hipMemcpyAsync(b->ws + P.o_desc, P.desc.data(), sizeof(CloudDesc) * (size_t)P.C, hipMemcpyHostToDevice, s);
    hipError_t e4 = hipStreamSynchronize(s);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
        if (b->owns) dfree(b->ws, s);
        delete b;
        return fail(PG_ERR_DEVICE, "pg_batch_create: plan upload failed");
    }
    *out = b;
    return PG_OK;
}

static BatchParams batch_params(pg_batch* b, const float* points, int32_t k, int32_t* out_idx,
                                float* out_d2) {
    const BatchPlan& PL = b->plan;
    BatchParams P;
    P.points = (const uint32_t*)points;
    P.out_idx = out_idx;
    P.out_d2 = out_d2;
    P.queue = (uint32_t*)(b->ws + PL.o_queue);
    P.ready = (uint32_t*)(b->ws + PL.o_ready);
    P.order = (const int32_t*)(b->ws + PL.o_order);
    P.qstart = (const int64_t*)(b->ws + PL.o_qstart);
    P.desc = (const CloudDesc*)(b->ws + PL.o_desc);
    P.pts = (uint32_t*)(b->ws + PL.o_pts);
    P.keys = (uint32_t*)(b->ws + PL.o_keys);
    P.pidx = (int32_t*)(b->ws + PL.o_pidx);
    P.pidx2 = (int32_t*)(b->ws + PL.o_pidx2);
    P.split = (uint32_t*)(b->ws + PL.o_split);
    P.bbox = (uint32_t*)(b->ws + PL.o_bbox);
    P.rec = (uint32_t*)(b->ws + PL.o_rec);
    P.total_items = PL.total_items;
    P.C = PL.C;
    P.d = PL.d;
    P.k = k;
    P.S = PL.S;
    P.lq = PL.lq;
    P.queries = nullptr;
    P.qoff = nullptr;
    P.qitems = nullptr;
    return P;
}

static pg_status batch_launch(pg_batch* b, const BatchParams& P, hipStream_t s) {
    switch (b->plan.d) {
        case 2: return batch_k<2>(b, P, s);
        case 3: return batch_k<3>(b, P, s);
        case 5: return batch_k<5>(b, P, s);
        default: return batch_k<8>(b, P, s);
    }
}

pg_status pg_batch_knn_self(pg_batch* b, const float* points, int32_t k, int32_t* out_idx,
                            float* out_d2, void* stream) {
    if (!b) return fail(PG_ERR_INVALID, "pg_batch_knn_self: handle is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_batch_knn_self: k must be in [1, 64]");
    const BatchPlan& PL = b->plan;
    if (PL.N > 0 && (!points || !out_idx || !out_d2)) return fail(PG_ERR_INVALID, "pg_batch_knn_self: NULL pointer");
    return batch_launch(b, batch_params(b, points, k, out_idx, out_d2), (hipStream_t)stream);
}

pg_status pg_batch_knn(pg_batch* b, const float* points, const float* queries,
                       const int64_t* q_offsets_host, int32_t k, int32_t* out_idx, float* out_d2,
                       void* stream) {
    if (!b) return fail(PG_ERR_INVALID, "pg_batch_knn: handle is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_batch_knn: k must be in [1, 64]");
    if (!q_offsets_host) return fail(PG_ERR_INVALID, "pg_batch_knn: q_offsets_host is NULL");
    BatchPlan& PL = b->plan;
    const int C = PL.C;
    const int64_t M = q_offsets_host[C];
    if (PL.N > 0 && !points) return fail(PG_ERR_INVALID, "pg_batch_knn: points is NULL");
    if (M > 0 && (!queries || !out_idx || !out_d2)) return fail(PG_ERR_INVALID, "pg_batch_knn: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    const bool same = (int)PL.qoff.size() == C + 1 &&
                      std::equal(PL.qoff.begin(), PL.qoff.end(), q_offsets_host);
    if (!same) {
        // a new query layout: checked, its items planned in the clouds' size
        // order, uploaded (synchronises)
        if (q_offsets_host[0] != 0) return fail(PG_ERR_INVALID, "pg_batch_knn: q_offsets[0] must be 0");
        for (int c = 0; c < C; c++)
            if (q_offsets_host[c + 1] < q_offsets_host[c])
                return fail(PG_ERR_INVALID, "pg_batch_knn: q_offsets must be non-decreasing");
        if (M >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_batch_knn: total queries must be < 2^31");
        std::vector<int64_t> items(C + 1);
        int64_t q = 0;
        const int64_t per = (int64_t)kQB * PL.lq;
        for (int t = 0; t < C; t++) {
            items[t] = q;
            const int c = PL.order[t];
            q += (q_offsets_host[c + 1] - q_offsets_host[c] + per - 1) / per;
        }
        items[C] = q;
        PG_HIP(hipMemcpyAsync(b->ws + PL.o_qoff, q_offsets_host, sizeof(int64_t) * (C + 1),
                              hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(b->ws + PL.o_qitems, items.data(), sizeof(int64_t) * (C + 1),
                              hipMemcpyHostToDevice, s));
        PG_HIP(hipStreamSynchronize(s));
        PL.qoff.assign(q_offsets_host, q_offsets_host + C + 1);
        PL.q_items = q;
    }
    BatchParams P = batch_params(b, points, k, out_idx, out_d2);
    P.queries = (const uint32_t*)queries;
    P.qoff = (const int64_t*)(b->ws + PL.o_qoff);
    P.qitems = (const int64_t*)(b->ws + PL.o_qitems);
    P.total_items = C + PL.q_items;
    return batch_launch(b, P, s);
}

pg_status pg_batch_status(const pg_batch* b, void* stream, int32_t* flags) {
    if (!b) return fail(PG_ERR_INVALID, "pg_batch_status: handle is NULL");
    uint32_t h[2] = {0, 0};
    hipStream_t s = (hipStream_t)stream;
    PG_HIP(hipMemcpyAsync(h, b->ws + b->plan.o_queue, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (flags) *flags = (int32_t)(h[1] & 3u);
    return PG_OK;
}

pg_status pg_batch_check(const float* points, int64_t n, int32_t d, void* stream) {
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_batch_check: d must be in [1, 8]");
    if (n < 0) return fail(PG_ERR_INVALID, "pg_batch_check: n < 0");
    if (n > 0 && !points) return fail(PG_ERR_INVALID, "pg_batch_check: points is NULL");
    return check_queries(points, n, d, true, (hipStream_t)stream);
}

pg_status pg_batch_autotune(const float* points, const int64_t* offsets_host, int32_t n_clouds,
                            int32_t d, int32_t k, void* stream, pg_tune* best) {
    if (!best || !offsets_host) return fail(PG_ERR_INVALID, "pg_batch_autotune: NULL pointer");
    if (n_clouds < 1 || d < 1 || d > 8 || k < 1 || k > 64)
        return fail(PG_ERR_INVALID, "pg_batch_autotune: bad sizes");
    const int64_t N = offsets_host[n_clouds];
    const TuneKey key(device_tag(), pow2_at_least(n_clouds), pow2_at_least(N), d, k);
    const char* cache_path = std::getenv("PG_TUNE_CACHE");
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return PG_OK;
        }
        pg_tune t{};
        if (cache_path && *cache_path && tune_file_lookup(cache_path, key, &t)) {
            g_tune_cache[key] = t;
            *best = t;
            return PG_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    DevBuf oi(s), od(s);
    PG_TRY(oi.alloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1) * k));
    PG_TRY(od.alloc(sizeof(float) * (size_t)(N > 0 ? N : 1) * k));
    hipEvent_t e0, e1;
    PG_HIP(hipEventCreate(&e0));
    PG_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    pg_tune win{16, 4, 1, PG_KLIST_VGPR};
    const int leaves[3] = {8, 16, 32};
    const int bpcs[2] = {2, 4};
    const int lqs[2] = {1, 4};
    const int kls[2] = {PG_KLIST_VGPR, PG_KLIST_LDS};
    for (int ci = 0; ci < 24; ci++) {
        const int li = ci / 8, bi = (ci / 4) % 2, qi = (ci / 2) % 2, ki = ci % 2;
        pg_tune t{leaves[li], bpcs[bi], lqs[qi], kls[ki]};
        pg_batch* b = nullptr;
        PG_TRY(pg_batch_create(offsets_host, n_clouds, d, &t, nullptr, 0, stream, &b));
        pg_status st = pg_batch_knn_self(b, points, k, oi.as<int32_t>(), od.as<float>(), stream);
        float ms = 0.0f;
        if (st == PG_OK) {
            (void)hipEventRecord(e0, s);
            st = pg_batch_knn_self(b, points, k, oi.as<int32_t>(), od.as<float>(), stream);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
        }
        pg_batch_free(b);
        if (st != PG_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return st;
        }
        if (ms < best_ms) {
            best_ms = ms;
            win = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = win;
        if (cache_path && *cache_path) tune_file_append(cache_path, key, win);
    }
    *best = win;
    return PG_OK;
}

void pg_batch_free(pg_batch* b) {
    if (!b) return;
    if (b->owns) dfree(b->ws, b->stream);
    if (b->bstart_dev) dfree(b->bstart_dev, b->stream);
    delete b;
}

pg_status pg_batch_backward(pg_batch* b, const float* points, int32_t k, const int32_t* idx,
                            const float* d2, const float* grad_d2, float* grad_points,
                            void* stream) {
    if (!b) return fail(PG_ERR_INVALID, "pg_batch_backward: handle is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_batch_backward: k must be in [1, 64]");
    const BatchPlan& PL = b->plan;
    const int64_t N = PL.N;
    if (N == 0) return PG_OK;
    if (!points || !idx || !d2 || !grad_d2 || !grad_points)
        return fail(PG_ERR_INVALID, "pg_batch_backward: NULL pointer");
    if (N * (int64_t)k >= ((int64_t)1 << 32)) return fail(PG_ERR_INVALID, "pg_batch_backward: N * k too large");
    hipStream_t s = (hipStream_t)stream;
    const int C = PL.C, d = PL.d;
    if (!b->bstart_dev) {
        PG_TRY(dalloc(&b->bstart_dev, (size_t)(C + 1), s));
        PG_HIP(hipMemcpyAsync(b->bstart_dev, PL.bstart.data(), sizeof(int64_t) * (C + 1),
                              hipMemcpyHostToDevice, s));
    }
    const int64_t items = PL.bstart[C];
    const CloudDesc* desc = (const CloudDesc*)(b->ws + PL.o_desc);
    const int32_t* pidx = (const int32_t*)(b->ws + PL.o_pidx);
    DevBuf inv(s), acc(s), maxes(s), wbuf(s), gl(s);
    const bool recs = d <= 3;  // row records {x, leaf position} instead of inv
    PG_TRY(inv.alloc(recs ? sizeof(uint4) * (size_t)N : sizeof(int32_t) * (size_t)N));
    PG_TRY(acc.alloc(sizeof(unsigned long long) * (size_t)N * d));
    PG_TRY(maxes.alloc(sizeof(uint32_t) * 2 * (size_t)C));
    PG_TRY(gl.alloc(sizeof(float) * (size_t)N * d));
    PG_TRY(wbuf.alloc(sizeof(unsigned long long) * (size_t)items * kBwdWin * d));
    PG_HIP(hipMemsetAsync(acc.p, 0, sizeof(unsigned long long) * (size_t)N * d, s));
    PG_HIP(hipMemsetAsync(maxes.p, 0, sizeof(uint32_t) * 2 * (size_t)C, s));
    const unsigned grid = grid_for_xcd(items);
    hipLaunchKernelGGL(bwd_inv_kernel, dim3(grid), dim3(kNT), 0, s, desc, (const int64_t*)b->bstart_dev,
                       C, items, pidx, points, d, inv.as<int32_t>(), recs ? inv.as<uint4>() : nullptr);
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(bwd_scale_kernel, dim3(grid), dim3(kNT), 0, s, desc, (const int64_t*)b->bstart_dev,
                       C, items, k, grad_d2, d2, maxes.as<uint32_t>());
    PG_LAUNCH_CHECK();
    const size_t lds = sizeof(unsigned long long) * (size_t)kBwdWin * d;
    auto main_kernel = d == 2 ? bwd_main_kernel<2>
                     : d == 3 ? bwd_main_kernel<3>
                     : d == 5 ? bwd_main_kernel<5> : bwd_main_kernel<8>;
    hipLaunchKernelGGL(main_kernel, dim3(grid), dim3(kNT), lds, s, desc, (const int64_t*)b->bstart_dev, C,
                       items, pidx, inv.as<int32_t>(), recs ? inv.as<uint4>() : nullptr, points, d, k, idx,
                       grad_d2, maxes.as<uint32_t>(), acc.as<unsigned long long>(),
                       wbuf.as<unsigned long long>(), gl.as<float>());
    PG_LAUNCH_CHECK();
    hipLaunchKernelGGL(bwd_finish_kernel, dim3(grid), dim3(kNT), 0, s, desc,
                       (const int64_t*)b->bstart_dev, C, items, pidx, d, wbuf.as<unsigned long long>(),
                       acc.as<unsigned long long>(), maxes.as<uint32_t>(), gl.as<float>(),
                       (uint32_t*)(b->ws + PL.o_queue) + 1, grad_points);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

pg_status pg_knn_backward_atomic(const float* queries, const float* points, int64_t m, int64_t n,
                               int32_t d, int32_t k, const int32_t* idx, const float* grad_d2,
                               float* grad_q, float* grad_p, void* stream) {
    if (d < 1 || d > 8 || k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_knn_backward_atomic: bad d or k");
    if (m < 0 || n < 0 || m * (int64_t)k >= ((int64_t)1 << 32) || n >= ((int64_t)1 << 31))
        return fail(PG_ERR_INVALID, "pg_knn_backward_atomic: bad sizes");
    if ((m > 0 && (!queries || !idx || !grad_d2 || !grad_q)) || (n > 0 && (!points || !grad_p)))
        return fail(PG_ERR_INVALID, "pg_knn_backward_atomic: NULL pointer");
    const bool alias = grad_q == grad_p;
    if (alias && (queries != points || m != n))
        return fail(PG_ERR_INVALID, "pg_knn_backward_atomic: grad_q may alias grad_p only when queries == points");
    hipStream_t s = (hipStream_t)stream;
    if (m > 0) {
        hipLaunchKernelGGL(grad_q_kernel, dim3(cdiv(m * d, kNT)), dim3(kNT), 0, s, queries, points,
                           m, n, d, k, idx, grad_d2, grad_q);
        PG_LAUNCH_CHECK();
    }
    if (n == 0) return PG_OK;
    if (!alias) {  // aliased: grad_q already overwrote every row
        hipLaunchKernelGGL(zero_f32_kernel, dim3(cdiv(n * d, kNT)), dim3(kNT), 0, s, grad_p, n * d);
        PG_LAUNCH_CHECK();
    }
    const int64_t P = m * k;
    if (P > 0) {
        hipLaunchKernelGGL(grad_x_atomic_kernel, dim3(cdiv(P, kNT)), dim3(kNT), 0, s, queries,
                           points, P, n, d, k, idx, grad_d2, grad_p);
        PG_LAUNCH_CHECK();
    }
    return PG_OK;
}

pg_status pg_knn_backward(const float* queries, const float* points, int64_t m, int64_t n,
                          int32_t d, int32_t k, const int32_t* idx, const float* grad_d2,
                          float* grad_q, float* grad_p, void* stream) {
    if (d < 1 || d > 8 || k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_knn_backward: bad d or k");
    if (m < 0 || n < 0 || m * (int64_t)k >= ((int64_t)1 << 32) || n >= ((int64_t)1 << 31))
        return fail(PG_ERR_INVALID, "pg_knn_backward: bad sizes");
    if ((m > 0 && (!queries || !idx || !grad_d2 || !grad_q)) || (n > 0 && (!points || !grad_p)))
        return fail(PG_ERR_INVALID, "pg_knn_backward: NULL pointer");
    const bool alias = grad_q == grad_p;
    if (alias && (queries != points || m != n))
        return fail(PG_ERR_INVALID, "pg_knn_backward: grad_q may alias grad_p only when queries == points");
    hipStream_t s = (hipStream_t)stream;
    const int64_t P = m * k;
    if (m > 0) {
        hipLaunchKernelGGL(grad_q_kernel, dim3(cdiv(m * d, kNT)), dim3(kNT), 0, s, queries, points,
                           m, n, d, k, idx, grad_d2, grad_q);
        PG_LAUNCH_CHECK();
    }
    if (n == 0) return PG_OK;
    DevBuf cnt(s), start(s), cursor(s), list(s), ordered(s), total(s);
    PG_TRY(total.alloc(sizeof(uint32_t)));
    PG_TRY(cnt.alloc(sizeof(uint32_t) * n));
    PG_TRY(start.alloc(sizeof(uint32_t) * n));
    PG_TRY(cursor.alloc(sizeof(uint32_t) * n));
    PG_TRY(list.alloc(sizeof(uint32_t) * (P > 0 ? P : 1)));
    PG_TRY(ordered.alloc(sizeof(uint32_t) * (P > 0 ? P : 1)));
    PG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t) * n, s));
    PG_HIP(hipMemsetAsync(cursor.p, 0, sizeof(uint32_t) * n, s));
    if (P > 0) {
        hipLaunchKernelGGL(pair_count_kernel, dim3(cdiv(P, kNT)), dim3(kNT), 0, s, idx, P, n,
                           cnt.as<uint32_t>());
        PG_LAUNCH_CHECK();
    }
    PG_TRY(exclusive_scan_u32(cnt.as<uint32_t>(), start.as<uint32_t>(), n, total.as<uint32_t>(), s));
    if (P > 0) {
        hipLaunchKernelGGL(pair_fill_kernel, dim3(cdiv(P, kNT)), dim3(kNT), 0, s, idx, P, n,
                           start.as<uint32_t>(), cursor.as<uint32_t>(), list.as<uint32_t>());
        PG_LAUNCH_CHECK();
        hipLaunchKernelGGL(pair_order_kernel, dim3(cdiv(P, kNT)), dim3(kNT), 0, s,
                           list.as<uint32_t>(), total.as<uint32_t>(), idx, start.as<uint32_t>(),
                           cnt.as<uint32_t>(), ordered.as<uint32_t>());
        PG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(grad_x_kernel, dim3(cdiv(n * d, kNT)), dim3(kNT), 0, s, queries, points,
                       n, d, k, grad_d2, start.as<uint32_t>(), cnt.as<uint32_t>(),
                       ordered.as<uint32_t>(), alias ? 1 : 0, grad_p);
    PG_LAUNCH_CHECK();
    return PG_OK;
}

}  // extern "C"
