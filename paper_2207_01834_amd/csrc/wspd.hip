// Well-separated pair decomposition (WSPD) of a kd-tree's points: Section 2
// builds it from the kd-tree (second module), after Callahan and Kosaraju.
//
// Readings (the paper names the decomposition but does not define its test):
//  * the tree is the object-median tree with leaf size 1 (every leaf holds at
//    most one point), so the pairs cover every pair of distinct points
//    exactly once;
//  * a node's ball is centred at the centre of its bounding box, with the
//    half diagonal as radius; nodes a and b are well separated for s when
//    the distance of the centres is at least (s + 2) r, r the larger radius
//    (balls of radius r around each set, at least s r apart), tested on
//    squares: |c_a - c_b|^2 >= (s + 2)^2 r^2, in double, half side
//    (hi - lo) * 0.5, centre (lo + hi) * 0.5, sums over dimensions in order,
//    no contraction into fused multiply-adds;
//  * an unseparated pair is refined by splitting the node with the larger
//    radius (the first on ties; never a leaf); pairs with an empty node are
//    dropped; every internal node starts with the pair of its children.
//
// GPU form: instead of the recursion, rounds over a frontier of candidate
// pairs (one lane each): the first frontier is every internal node's pair of
// children; each round tests every candidate, emits the separated ones, and
// replaces each unseparated one by its two refinements.  A scan of packed
// (emitted, refined) flags gives every candidate its output slot and its
// slots in the next frontier, so the output order is deterministic (round by
// round, frontier order within a round).  A round moves one of the two nodes
// one level down, so there are at most 2L rounds.
#include "knn.hpp"
#include "scan.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = 256;
constexpr uint64_t kEmit = 1ull, kRefine = 1ull << 32;

// Points of heap node h (closed-form ranges).
__device__ inline int64_t heap_points(int64_t n, uint32_t h) {
    const int l = 31 - __clz(h);
    const int64_t j = (int64_t)h - ((int64_t)1 << l);
    return node_start(n, l, j + 1) - node_start(n, l, j);
}

// Squared radius and centre of node h's box.
template <typename T, int MD>
__device__ inline void node_ball(const TreeView& tv, uint32_t h, int d, double (&c)[MD], double& r2) {
#pragma clang fp contract(off)
    const uint32_t* b = tv.nbox + (size_t)h * 2 * d;
    r2 = 0.0;
#pragma unroll
    for (int e = 0; e < MD; e++) {
        if (MD < 8 || e < d) {
            const double lo = (double)Metric<T>::load(b[e]), hi = (double)Metric<T>::load(b[d + e]);
            const double t = (hi - lo) * 0.5;
            r2 = r2 + t * t;
            c[e] = (lo + hi) * 0.5;
        } else {
            c[e] = 0.0;
        }
    }
}

__global__ void wspd_init_kernel(int64_t count, uint2* __restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < count) {
        const uint32_t h = (uint32_t)(i + 1);
        F[i] = make_uint2(2u * h, 2u * h + 1u);
    }
}

// Decision per candidate: 0 drop (an empty node), 1 emit, 2 refine by
// splitting the first node, 3 the second; flags pack (emit, refine) counts.
template <typename T, int MD>
__device__ inline void wspd_decide(const TreeView& tv, uint2 p, int d, double s2, uint8_t& dc, uint64_t& fl) {
#pragma clang fp contract(off)
    dc = 0;
    fl = 0;
    if (heap_points(tv.n, p.x) > 0 && heap_points(tv.n, p.y) > 0) {
        double ca[MD], cb[MD], ra, rb;
        node_ball<T, MD>(tv, p.x, d, ca, ra);
        node_ball<T, MD>(tv, p.y, d, cb, rb);
        double g2 = 0.0;
#pragma unroll
        for (int e = 0; e < MD; e++) {
            if (MD < 8 || e < d) {
                const double t = ca[e] - cb[e];
                g2 = g2 + t * t;
            }
        }
        const double r2 = ra > rb ? ra : rb;
        if (g2 >= s2 * r2) {
            dc = 1;
            fl = kEmit;
        } else {
            const uint32_t first_leaf = 1u << tv.L;
            const bool split_a = (ra >= rb && p.x < first_leaf) || p.y >= first_leaf;
            dc = split_a ? 2 : 3;
            fl = kRefine;
        }
    }
}

template <typename T, int MD>
__global__ void __launch_bounds__(kNT)
wspd_step_kernel(TreeView tv, const uint2* __restrict__ F, int64_t nf, double s2,
                 uint8_t* __restrict__ dec, uint64_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= nf) return;
    uint8_t dc;
    uint64_t fl;
    wspd_decide<T, MD>(tv, F[i], MD < 8 ? MD : tv.d, s2, dc, fl);
    dec[i] = dc;
    flags[i] = fl;
}

// Emitted candidates to out[base + rank] (below capacity), refined ones to
// their two slots of the next frontier.
__global__ void __launch_bounds__(kNT)
wspd_scatter_kernel(const uint2* __restrict__ F, int64_t nf, const uint8_t* __restrict__ dec,
                    const uint64_t* __restrict__ pre, uint2* __restrict__ out, int64_t base,
                    int64_t capacity, uint2* __restrict__ next) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= nf) return;
    const uint8_t dc = dec[i];
    if (dc == 0) return;
    const uint2 p = F[i];
    if (dc == 1) {
        const int64_t o = base + (int64_t)(uint32_t)pre[i];
        if (o < capacity) out[o] = p;
        return;
    }
    const int64_t r = (int64_t)(pre[i] >> 32);
    if (dc == 2) {
        next[2 * r] = make_uint2(2u * p.x, p.y);
        next[2 * r + 1] = make_uint2(2u * p.x + 1u, p.y);
    } else {
        next[2 * r] = make_uint2(p.x, 2u * p.y);
        next[2 * r + 1] = make_uint2(p.x, 2u * p.y + 1u);
    }
}

// ---- Rounds driven from the device: the frontier size, the output base and
// an overflow flag live in device memory, so the host enqueues every round
// without reading anything back.  The passes are grid-stride loops over the
// current frontier; a frontier that would outgrow its buffers stops the
// rounds (the host then runs the rounds it drives itself, above).
struct Rounds {
    int64_t nf;         // current frontier size
    int64_t base;       // pairs emitted before this round
    uint64_t total;     // packed (emitted, refined) counts of this round
    uint32_t overflow;  // a frontier exceeded the capacity
};

constexpr unsigned kRoundGrid = 4096;      // workgroups of the grid-stride passes
constexpr int kScanItems = 8;
constexpr int kScanTile = kNT * kScanItems;  // flags per partial sum

// Decisions of the current frontier, in tiles of kScanTile candidates: each
// tile's packed (emit, refine) total goes to sums[tile].
template <typename T, int MD>
__global__ void __launch_bounds__(kNT)
wspd_step_dev_kernel(TreeView tv, const uint2* __restrict__ F, const Rounds* __restrict__ R, double s2,
                     uint8_t* __restrict__ dec, uint64_t* __restrict__ flags, uint64_t* __restrict__ sums) {
    __shared__ uint64_t red[kNT / kWave];
    const int64_t nf = R->nf;
    const int64_t tiles = (nf + kScanTile - 1) / kScanTile;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        uint64_t acc = 0;
        for (int i = 0; i < kScanItems; i++) {
            const int64_t e = t * kScanTile + (int64_t)i * kNT + threadIdx.x;
            if (e < nf) {
                uint8_t dc;
                uint64_t fl;
                wspd_decide<T, MD>(tv, F[e], MD < 8 ? MD : tv.d, s2, dc, fl);
                dec[e] = dc;
                flags[e] = fl;
                acc += fl;
            }
        }
        acc = wave_sum(acc);
        if (lane_id() == 0) red[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t a = 0;
            for (int w = 0; w < kNT / kWave; w++) a += red[w];
            sums[t] = a;
        }
        __syncthreads();
    }
}

// Exclusive scan of the tile totals (one workgroup); the round's total.
__global__ void __launch_bounds__(kNT)
wspd_sums_kernel(uint64_t* __restrict__ sums, Rounds* __restrict__ R) {
    __shared__ uint64_t lds[kNT / kWave + 1];
    const int64_t tiles = (R->nf + kScanTile - 1) / kScanTile;
    uint64_t run = 0;
    for (int64_t b = 0; b < tiles; b += kNT) {
        const int64_t e = b + threadIdx.x;
        const uint64_t v = e < tiles ? sums[e] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_excl_scan<kNT>(v, lds, &tot);
        if (e < tiles) sums[e] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) R->total = run;
}

// Per tile: the candidates' exclusive prefix of packed counts (the tile's
// scanned total plus a workgroup scan); emitted candidates to
// out[base + rank] (below capacity), refined ones to their two slots of the
// next frontier when it fits `cap` pairs.
__global__ void __launch_bounds__(kNT)
wspd_scatter_dev_kernel(const uint2* __restrict__ F, const Rounds* __restrict__ R,
                        const uint8_t* __restrict__ dec, const uint64_t* __restrict__ flags,
                        const uint64_t* __restrict__ sums, uint2* __restrict__ out, int64_t capacity,
                        uint2* __restrict__ next, int64_t cap) {
    __shared__ uint64_t lds[kNT / kWave + 1];
    const int64_t nf = R->nf, base = R->base;
    const bool fits = 2 * (int64_t)(R->total >> 32) <= cap;
    const int64_t tiles = (nf + kScanTile - 1) / kScanTile;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        uint64_t run = sums[t];
        for (int i = 0; i < kScanItems; i++) {
            const int64_t e = t * kScanTile + (int64_t)i * kNT + threadIdx.x;
            const uint64_t v = e < nf ? flags[e] : 0ull;
            uint64_t tot;
            const uint64_t pre = run + block_excl_scan<kNT>(v, lds, &tot);
            run += tot;
            if (e >= nf) continue;
            const uint8_t dc = dec[e];
            if (dc == 0) continue;
            const uint2 p = F[e];
            if (dc == 1) {
                const int64_t o = base + (int64_t)(uint32_t)pre;
                if (o < capacity) out[o] = p;
                continue;
            }
            if (!fits) continue;
            const int64_t r = (int64_t)(pre >> 32);
            if (dc == 2) {
                next[2 * r] = make_uint2(2u * p.x, p.y);
                next[2 * r + 1] = make_uint2(2u * p.x + 1u, p.y);
            } else {
                next[2 * r] = make_uint2(p.x, 2u * p.y);
                next[2 * r + 1] = make_uint2(p.x, 2u * p.y + 1u);
            }
        }
    }
}

// One thread: the next round's frontier size and output base.
__global__ void wspd_advance_kernel(Rounds* __restrict__ R, int64_t cap) {
    const int64_t emits = (int64_t)(uint32_t)R->total, refines = (int64_t)(R->total >> 32);
    R->base += emits;
    if (2 * refines > cap) {
        R->overflow = 1u;
        R->nf = 0;
    } else {
        R->nf = 2 * refines;
    }
    R->total = 0;
}

__global__ void wspd_rounds_init_kernel(Rounds* __restrict__ R, int64_t nf) {
    R->nf = nf;
    R->base = 0;
    R->total = 0;
    R->overflow = 0u;
}

template <typename T, int MD>
void launch_step_dev(const TreeView& tv, const uint2* F, const Rounds* R, double s2, uint8_t* dec,
                     uint64_t* flags, uint64_t* sums, hipStream_t s) {
    hipLaunchKernelGGL((wspd_step_dev_kernel<T, MD>), dim3(kRoundGrid), dim3(kNT), 0, s, tv, F, R, s2, dec,
                       flags, sums);
}

template <typename T>
void step_dev_d(const TreeView& tv, const uint2* F, const Rounds* R, double s2, uint8_t* dec,
                uint64_t* flags, uint64_t* sums, hipStream_t s) {
    switch (tv.d) {
        case 1: launch_step_dev<T, 1>(tv, F, R, s2, dec, flags, sums, s); break;
        case 2: launch_step_dev<T, 2>(tv, F, R, s2, dec, flags, sums, s); break;
        case 3: launch_step_dev<T, 3>(tv, F, R, s2, dec, flags, sums, s); break;
        case 5: launch_step_dev<T, 5>(tv, F, R, s2, dec, flags, sums, s); break;
        default: launch_step_dev<T, 8>(tv, F, R, s2, dec, flags, sums, s); break;
    }
}

template <typename T, int MD>
void launch_step(const TreeView& tv, const uint2* F, int64_t nf, double s2, uint8_t* dec,
                 uint64_t* flags, hipStream_t s) {
    hipLaunchKernelGGL((wspd_step_kernel<T, MD>), dim3(cdiv(nf, kNT)), dim3(kNT), 0, s, tv, F, nf, s2,
                       dec, flags);
}

template <typename T>
void step_d(const TreeView& tv, const uint2* F, int64_t nf, double s2, uint8_t* dec, uint64_t* flags,
            hipStream_t s) {
    switch (tv.d) {
        case 1: launch_step<T, 1>(tv, F, nf, s2, dec, flags, s); break;
        case 2: launch_step<T, 2>(tv, F, nf, s2, dec, flags, s); break;
        case 3: launch_step<T, 3>(tv, F, nf, s2, dec, flags, s); break;
        case 5: launch_step<T, 5>(tv, F, nf, s2, dec, flags, s); break;
        default: launch_step<T, 8>(tv, F, nf, s2, dec, flags, s); break;
    }
}

}  // namespace

namespace {

// The rounds enqueued at once, driven from the device (see Rounds).  Returns
// PG_OK with *done set when they finished within the frontier capacity.
pg_status wspd_device(const pg_tree* t, double s2, uint32_t* out_pairs, int64_t capacity, int64_t* count,
                      bool* done, hipStream_t s) {
    *done = false;
    const TreeView tv = t->view();
    const int64_t nf0 = ((int64_t)1 << t->L) - 1;
    const int64_t cap = 4 * nf0 + ((int64_t)1 << 20);  // pairs per frontier
    const int64_t tiles = (cap + kScanTile - 1) / kScanTile;
    const size_t bytes = sizeof(uint2) * 2 * (size_t)cap + (size_t)cap + sizeof(uint64_t) * (size_t)(cap + tiles) +
                         sizeof(Rounds) + 1024;
    if (bytes > ((size_t)16 << 30)) return PG_OK;  // too large to hold up front: the host drives the rounds
    DevBuf buf(s);
    PG_TRY(buf.alloc(bytes));
    uint8_t* b = buf.as<uint8_t>();
    uint2* fr[2] = {reinterpret_cast<uint2*>(b), reinterpret_cast<uint2*>(b) + cap};
    uint64_t* flags = reinterpret_cast<uint64_t*>(b + sizeof(uint2) * 2 * (size_t)cap);
    uint64_t* sums = flags + cap;
    Rounds* R = reinterpret_cast<Rounds*>(sums + tiles);
    uint8_t* dec = reinterpret_cast<uint8_t*>(R + 1);
    hipLaunchKernelGGL(wspd_init_kernel, dim3(cdiv(nf0, kNT)), dim3(kNT), 0, s, nf0, fr[0]);
    hipLaunchKernelGGL(wspd_rounds_init_kernel, dim3(1), dim3(1), 0, s, R, nf0);
    PG_LAUNCH_CHECK();
    // a round moves one node of a pair one level down: at most 2L rounds
    int cur = 0;
    for (int r = 0; r < 2 * t->L + 1; r++) {
        if (t->dtype == PG_FLOAT32) step_dev_d<float>(tv, fr[cur], R, s2, dec, flags, sums, s);
        else step_dev_d<int32_t>(tv, fr[cur], R, s2, dec, flags, sums, s);
        hipLaunchKernelGGL(wspd_sums_kernel, dim3(1), dim3(kNT), 0, s, sums, R);
        hipLaunchKernelGGL(wspd_scatter_dev_kernel, dim3(kRoundGrid), dim3(kNT), 0, s, fr[cur], R, dec, flags,
                           sums, reinterpret_cast<uint2*>(out_pairs), capacity, fr[cur ^ 1], cap);
        hipLaunchKernelGGL(wspd_advance_kernel, dim3(1), dim3(1), 0, s, R, cap);
        PG_LAUNCH_CHECK();
        cur ^= 1;
    }
    Rounds h{};
    PG_HIP(hipMemcpyAsync(&h, R, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (h.overflow || h.nf != 0) return PG_OK;  // not finished: the host drives the rounds
    *count = h.base;
    *done = true;
    return PG_OK;
}

}  // namespace

pg_status wspd(const pg_tree* t, double sep, uint32_t* out_pairs, int64_t capacity, int64_t* count,
               hipStream_t s) {
    const TreeView tv = t->view();
    const double s2 = (sep + 2.0) * (sep + 2.0);
    if (t->L > 0) {
        bool done = false;
        PG_TRY(wspd_device(t, s2, out_pairs, capacity, count, &done, s));
        if (done) {
            if (*count > capacity)
                return fail(PG_ERR_INVALID, "pg_wspd: " + std::to_string(*count) + " pairs exceed capacity " +
                                                std::to_string(capacity) + " (the first capacity pairs are written)");
            return PG_OK;
        }
    }
    // the rounds driven from the host, each reading its counts back (the
    // frontier grows without bound here)
    int64_t nf = t->L > 0 ? ((int64_t)1 << t->L) - 1 : 0;  // internal nodes
    int64_t total = 0;
    // two frontiers, decisions, flags scanned in place with the totals in
    // the entry after the last; grown by half again when too small, so that
    // a frontier growing over the rounds costs a few allocations, not one
    // per round (each had held the host for about 0.1 ms)
    DevBuf fr[2] = {DevBuf(s), DevBuf(s)}, dec(s), flg(s);
    size_t cap_fr[2] = {0, 0}, cap_dec = 0, cap_flg = 0;
    auto grow = [](DevBuf& b, size_t& cap, size_t bytes) -> pg_status {
        if (bytes > cap) {
            const size_t want = bytes + bytes / 2;
            PG_TRY(b.alloc(want));
            cap = want;
        }
        return PG_OK;
    };
    int cur = 0;
    if (nf > 0) {
        PG_TRY(grow(fr[0], cap_fr[0], sizeof(uint2) * nf));
        hipLaunchKernelGGL(wspd_init_kernel, dim3(cdiv(nf, kNT)), dim3(kNT), 0, s, nf, fr[0].as<uint2>());
        PG_LAUNCH_CHECK();
    }
    while (nf > 0) {
        PG_TRY(grow(dec, cap_dec, (size_t)nf));
        // flags [nf], their total, then the scan's partial sums
        PG_TRY(grow(flg, cap_flg, sizeof(uint64_t) * (nf + 1 + scan_partials(nf))));
        uint64_t* flags = flg.as<uint64_t>();
        if (t->dtype == PG_FLOAT32) step_d<float>(tv, fr[cur].as<uint2>(), nf, s2, dec.as<uint8_t>(), flags, s);
        else step_d<int32_t>(tv, fr[cur].as<uint2>(), nf, s2, dec.as<uint8_t>(), flags, s);
        PG_LAUNCH_CHECK();
        PG_TRY(exclusive_scan_u64_ws(flags, flags, nf, flags + nf, flags + nf + 1, s));
        uint64_t tot = 0;
        PG_HIP(hipMemcpyAsync(&tot, flags + nf, sizeof(tot), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        const int64_t emits = (int64_t)(uint32_t)tot, refines = (int64_t)(tot >> 32);
        PG_TRY(grow(fr[cur ^ 1], cap_fr[cur ^ 1], sizeof(uint2) * (size_t)(2 * refines > 0 ? 2 * refines : 1)));
        hipLaunchKernelGGL(wspd_scatter_kernel, dim3(cdiv(nf, kNT)), dim3(kNT), 0, s, fr[cur].as<uint2>(), nf,
                           dec.as<uint8_t>(), flags, reinterpret_cast<uint2*>(out_pairs), total, capacity,
                           fr[cur ^ 1].as<uint2>());
        PG_LAUNCH_CHECK();
        total += emits;
        nf = 2 * refines;
        cur ^= 1;
    }
    PG_HIP(hipStreamSynchronize(s));
    *count = total;
    if (total > capacity)
        return fail(PG_ERR_INVALID, "pg_wspd: " + std::to_string(total) + " pairs exceed capacity " +
                                        std::to_string(capacity) + " (the first capacity pairs are written)");
    return PG_OK;
}

}  // namespace pg

using namespace pg;

extern "C" pg_status pg_wspd(const pg_tree* t, double s, uint32_t* out_pairs, int64_t capacity,
                             int64_t* count_host, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_wspd: tree is NULL");
    if (!count_host) return fail(PG_ERR_INVALID, "pg_wspd: count_host is NULL");
    if (!(s > 0.0) || !(s < 1e300)) return fail(PG_ERR_INVALID, "pg_wspd: s must be positive and finite");
    if (capacity < 0 || (capacity > 0 && !out_pairs)) return fail(PG_ERR_INVALID, "pg_wspd: bad output buffer");
    if (t->xn || t->loff || t->leaf != 1)
        return fail(PG_ERR_UNSUPPORTED, "pg_wspd: needs a tree from pg_kdtree_build with leaf size 1");
    if (t->L > 31) return fail(PG_ERR_UNSUPPORTED, "pg_wspd: tree too deep");
    return wspd(t, s, out_pairs, capacity, count_host, (hipStream_t)stream);
}
