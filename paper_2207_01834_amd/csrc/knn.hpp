// k-NN search over static kd-trees: device-side pieces shared by the static,
// BDL and batched searches, and the host entry points of knn.hip.
#pragma once

#include <float.h>

#include "common.hpp"

namespace pg {

template <typename T> struct Metric;

// int32 coordinates: exact int64 squared distances (|diff| < 2^30).
template <> struct Metric<int32_t> {
    using D = int64_t;
    static __device__ __host__ inline D inf() { return INT64_MAX; }
    static __device__ inline int32_t load(uint32_t b) { return (int32_t)b; }
    static __device__ inline D sq(int32_t a, int32_t b) {
        const int32_t t = a - b;
        return (int64_t)t * (int64_t)t;
    }
    static __device__ inline D acc(D s, int32_t a, int32_t b) { return s + sq(a, b); }
    // distance from a to the interval [lo, hi] along one axis, squared, added to s
    static __device__ inline D acc_gap(D s, int32_t a, int32_t lo, int32_t hi) {
        const int32_t g = a < lo ? lo - a : (a > hi ? a - hi : 0);
        return s + (int64_t)g * (int64_t)g;
    }
};

// float32 coordinates: float32 squared distances accumulated with fused
// multiply-adds in dimension order.  The plane and box bounds use the same
// operations on smaller-or-equal magnitudes, and rounding is monotone, so a
// bound never exceeds the computed distance of a point it covers.
template <> struct Metric<float> {
    using D = float;
    static __device__ __host__ inline D inf() { return __builtin_huge_valf(); }
    static __device__ inline float load(uint32_t b) { return __uint_as_float(b); }
    static __device__ inline D sq(float a, float b) {
        const float t = a - b;
        return t * t;
    }
    static __device__ inline D acc(D s, float a, float b) {
        const float t = a - b;
        return __builtin_fmaf(t, t, s);
    }
    static __device__ inline D acc_gap(D s, float a, float lo, float hi) {
        const float g = a < lo ? lo - a : (a > hi ? a - hi : 0.0f);
        return __builtin_fmaf(g, g, s);
    }
};

// Sorted list of the k best (distance, id) keys held in registers.  KT is a
// compile-time capacity >= k; with EX the list length is exactly KT (= k),
// otherwise slots >= k are never touched (uniform guards).
template <typename DT, typename IT, int KT, bool EX>
struct KList {
    DT d[KT];
    IT id[KT];
    DT kd;   // distance of slot k-1 (the pruning radius, squared)
    IT kid;  // id of slot k-1

    __device__ inline void init(DT inf, IT none) {
#pragma unroll
        for (int s = 0; s < KT; s++) {
            d[s] = inf;
            id[s] = none;
        }
        kd = inf;
        kid = none;
    }
    __device__ static inline bool less(DT a, IT ai, DT b, IT bi) {
        return a < b || (a == b && ai < bi);
    }
    // True when (dd, ii) belongs in the list.
    __device__ inline bool admits(DT dd, IT ii) const { return less(dd, ii, kd, kid); }
    // Adds (dd, ii) when it belongs in the list.
    __device__ inline void offer(DT dd, IT ii, int k) {
        if (admits(dd, ii)) insert(dd, ii, k);
    }
    // Inserts (dd, ii); requires admits(dd, ii).
    // Slot s receives the old slot s-1 when the new key sorts before it, the
    // new key when it sorts before the old slot s but not before slot s-1,
    // and keeps its key otherwise.
    __device__ inline void insert(DT dd, IT ii, int k) {
        bool before_cur = true;  // new key sorts before the old key of slot s
#pragma unroll
        for (int s = KT - 1; s >= 0; --s) {
            if (EX || s < k) {
                const int p = s > 0 ? s - 1 : 0;
                const bool before_prev = s > 0 && less(dd, ii, d[p], id[p]);
                const DT nd = before_prev ? d[p] : (before_cur ? dd : d[s]);
                const IT ni = before_prev ? id[p] : (before_cur ? ii : id[s]);
                d[s] = nd;
                id[s] = ni;
                if (EX ? s == KT - 1 : s == k - 1) {
                    kd = nd;
                    kid = ni;
                }
                before_cur = before_prev;
            }
        }
    }
};

// Sorted list of the k best keys, each (squared distance, id) packed into one
// 64-bit word -- the distance in the high bits, the id (< 2^B) in the low B --
// so that one unsigned compare orders two (distance, id) pairs and moving an
// entry is one 64-bit select.  float32: the distance's bits (non-negative, so
// ordered as unsigned) over a 32-bit id: exact.  int32 coordinates: the
// int64 distance over B id bits, so only distances up to C = 2^(64-B) - 1
// fit; the radius starts at C and a point farther than the radius never
// enters, so every stored key is exact.  A search whose k-th key ends at C
// (or unfilled) may have missed points beyond C and is redone with KList;
// pruning with a radius of C only discards such points.
template <typename T, int KT, bool EX>
struct PackedList {
    using DT = typename Metric<T>::D;
    static constexpr bool kFloat = sizeof(DT) == 4;
    static constexpr uint64_t kEmpty = kFloat ? 0x7f800000ffffffffull : ~0ull;
    uint64_t key[KT];
    uint64_t kk;  // key of slot k-1
    DT kd;        // its distance: the pruning radius, squared
    int B;        // id bits

    __device__ inline void init(int idbits) {
        B = kFloat ? 32 : idbits;
#pragma unroll
        for (int s = 0; s < KT; s++) key[s] = kEmpty;
        kk = kEmpty;
        kd = dist_of(kEmpty);
    }
    __device__ inline DT dist_of(uint64_t x) const {
        if constexpr (kFloat) return __uint_as_float((uint32_t)(x >> 32));
        else return (DT)(x >> B);
    }
    __device__ inline int32_t id_of(uint64_t x) const {
        return (int32_t)(uint32_t)(x & (~0ull >> (64 - B)));
    }
    // True when the k-th distance is C or the list is not full (int32
    // coordinates only): the result may miss points beyond C.
    __device__ inline bool needs_redo() const {
        if constexpr (kFloat) return false;
        else return (kk >> B) == (~0ull >> B);
    }
    __device__ inline void offer(DT dd, int32_t ii, int k) {
        if constexpr (kFloat) {
            const uint64_t x = ((uint64_t)__float_as_uint(dd) << 32) | (uint32_t)ii;
            if (x < kk) insert(x, k);
        } else {
            // exact whenever dd <= kd, since kd <= 2^(64-B) - 1
            const uint64_t x = ((uint64_t)dd << B) | (uint32_t)ii;
            if (!(dd > kd) && x < kk) insert(x, k);
        }
    }
    __device__ inline void insert(uint64_t x, int k) {
        bool before_cur = true;
#pragma unroll
        for (int s = KT - 1; s >= 0; --s) {
            if (EX || s < k) {
                const int p = s > 0 ? s - 1 : 0;
                const bool before_prev = s > 0 && x < key[p];
                const uint64_t nk = before_prev ? key[p] : (before_cur ? x : key[s]);
                key[s] = nk;
                if (EX ? s == KT - 1 : s == k - 1) kk = nk;
                before_cur = before_prev;
            }
        }
        kd = dist_of(kk);
    }
};

// The float32 packed keys of PackedList held in LDS instead of registers:
// slot s of a lane at key[s * stride] (neighbouring lanes at neighbouring
// 8-byte words, so a slot access is conflict-free).  Frees 2*KT registers per
// lane (more waves per SIMD) and costs one LDS read and write per slot of an
// insertion; the batched launch's tuner picks the placement.
template <int KT, bool EX>
struct LdsList {
    using DT = float;
    static constexpr uint64_t kEmpty = 0x7f800000ffffffffull;
    uint64_t* key;  // this lane's slot 0
    int stride;     // words between a lane's slots
    uint64_t kk;    // key of slot k-1
    float kd;       // its distance: the pruning radius, squared

    __device__ inline void init(uint64_t* base, int stride_) {
        key = base;
        stride = stride_;
#pragma unroll
        for (int s = 0; s < KT; s++) key[s * stride] = kEmpty;
        kk = kEmpty;
        kd = dist_of(kEmpty);
    }
    __device__ static inline float dist_of(uint64_t x) { return __uint_as_float((uint32_t)(x >> 32)); }
    __device__ static inline int32_t id_of(uint64_t x) { return (int32_t)(uint32_t)x; }
    __device__ inline uint64_t at(int s) const { return key[s * stride]; }
    __device__ inline void offer(float dd, int32_t ii, int k) {
        const uint64_t x = ((uint64_t)__float_as_uint(dd) << 32) | (uint32_t)ii;
        if (x < kk) insert(x, k);
    }
    // As PackedList::insert, from the top slot down; the slot below is read
    // once and carried to the next step.
    __device__ inline void insert(uint64_t x, int k) {
        const int top = EX ? KT - 1 : k - 1;
        uint64_t cur = key[top * stride];
        for (int s = top; s >= 0; --s) {
            const uint64_t below = s > 0 ? key[(s - 1) * stride] : 0ull;
            const uint64_t nk = (s > 0 && x < below) ? below : (x < cur ? x : cur);
            key[s * stride] = nk;
            if (s == top) kk = nk;
            cur = below;
        }
        kd = dist_of(kk);
    }
};

// Id bits of the packed keys of a tree of n points (ids are rows < n).
inline int id_bits(int64_t n) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n) b++;
    return b;
}

// Host entry points.

// Queries below this count are searched in the caller's order.
constexpr int64_t kOrderMin = 4096;

// Device workspace of one separate-query k-NN call, for callers that bring
// their own memory (null members are allocated by the call).
struct KnnWs {
    int32_t* order;   // [m] query permutation
    uint32_t* work;   // [m + buckets] bucket keys, then bucket counts
    uint32_t* sums;   // [scan_partials(buckets)] partial sums of the bucket scan
    int32_t* redo;    // [m] queries searched again with exact pairs (int32 trees)
    uint32_t* nredo;  // [1] their count
};

// Where each separate query's descent in the tree that ordered the queries
// ended: key[i] is the level-`lev` node of a heap tree as an offset from
// 2^lev, or (lev < 0) the leaf index of an explicit-node tree.  key == null:
// not recorded.
struct QueryKeys {
    const uint32_t* key = nullptr;
    int lev = 0;
};

// Buckets the query ordering uses for m queries over tree tv.
int64_t order_buckets(const TreeView& tv, int64_t m);

// A permutation of the m queries that follows the leaf order of tree tv (a
// counting sort by the leaf each query's descent reaches); order receives
// m int32 query indices.  With `boxes` the queries are boxes [m][2][d]
// (lo, hi) and each descends by its centre.  keys (may be null): where each
// descent ended, valid while `order` is.
pg_status order_queries(const TreeView& tv, bool fl, const void* queries, int64_t m,
                        hipStream_t s, DevBuf& order, bool boxes = false, QueryKeys* keys = nullptr);
// The same into caller workspace (order [m], work [m + buckets], sums); the
// keys live in the first m words of work.
pg_status order_queries_ws(const TreeView& tv, bool fl, const void* queries, int64_t m,
                           hipStream_t s, int32_t* order, uint32_t* work, uint32_t* sums,
                           bool boxes = false, QueryKeys* keys = nullptr);
// no_self (all-points only): each point's own row is not a candidate.
pg_status knn_static(const pg_tree* t, const void* queries, int64_t m, int k, bool all_points,
                     int32_t* out_idx, void* out_dist, hipStream_t s, bool no_self = false,
                     const KnnWs* ws = nullptr);

// The static-tree k-NN launch for one coordinate type (order: the query
// permutation or null; qk: where the ordering's descents ended, or none;
// no_self: all-points without each point's own row).
pg_status knn_static_int(const pg_tree* t, const void* queries, const int32_t* order, QueryKeys qk,
                         int64_t m, int k, bool all, int32_t* out_idx, void* out_dist, hipStream_t s,
                         bool no_self, const KnnWs* ws);
pg_status knn_static_float(const pg_tree* t, const void* queries, const int32_t* order, QueryKeys qk,
                           int64_t m, int k, bool all, int32_t* out_idx, void* out_dist, hipStream_t s,
                           bool no_self, const KnnWs* ws);

// Validates query coordinates (range / finite); synchronises.
pg_status check_queries(const void* q, int64_t m, int d, bool fl, hipStream_t s);
// The same with a caller-provided device flag word.
pg_status check_queries_ws(const void* q, int64_t m, int d, bool fl, uint32_t* err, hipStream_t s);

}  // namespace pg
