// Wave-per-block k-NN over a static heap tree (Appendix C, "Data-Parallel
// k-NN", with the wave rather than the lane as the unit of traversal).
//
// The 64 lanes of a wave hold 64 queries that lie close together: in
// all-points mode 64 consecutive leaf-order points of the tree, otherwise 64
// consecutive queries of the leaf order the queries were sorted into.  The
// wave walks the tree once for all of them:
//   * the walk state (node, previous node) is uniform, so split values, node
//     boxes and leaf points are scalar loads shared by the 64 lanes, and the
//     walk itself costs scalar instructions instead of 64 divergent walks;
//   * a child is entered when it is within reach of any lane (the squared
//     distance from that lane's query to the child's box is at most its
//     current k-th distance); the child holding more of the wave's queries
//     goes first;
//   * at a leaf every lane measures every point of the leaf against its own
//     query (the points are broadcast from scalar registers); a point within
//     the lane's k-th distance goes to a small per-lane buffer, and the
//     buffers are merged into the sorted k-lists when one fills or the leaf
//     ends, so a merge round serves every lane that holds a candidate.
//
// Each lane ends with exactly the list of kd_search: every point within the
// final k-th distance of a query lies in a leaf whose box is within every
// earlier k-th distance of it, so it is offered, and the list keeps the k
// smallest (distance, id) keys whatever the order of the offers.
//
// Part of knn_static.hpp (included there after the per-lane kernels, whose
// load_query and block size it shares).
#pragma once

#include "search.hpp"
#include "wave.hpp"

namespace pg {
namespace knn_detail {

constexpr int kWaveBuf = 4;  // per-lane candidate buffer (packed keys)

template <typename T, typename KL>
struct WaveLane {
    KL kl;
    uint64_t buf[kWaveBuf];
    int cnt;

    // Merges the buffered keys into the list, in rounds over the wave.
    __device__ inline void flush(int k) {
        while (__ballot(cnt > 0) != 0) {
            if (cnt > 0) {
                cnt--;
                uint64_t x = buf[0];
#pragma unroll
                for (int b = 1; b < kWaveBuf; b++) x = cnt == b ? buf[b] : x;
                if (x < kl.kk) kl.insert(x, k);
            }
        }
    }
};

// Squared distance from q to the box {lo[d], hi[d]} at b (scalar words).
template <typename T, int MD>
__device__ inline typename Metric<T>::D wave_box_gap(const uint32_t* __restrict__ b, const T (&q)[MD],
                                                     int d) {
    using M = Metric<T>;
    typename M::D g = 0;
#pragma unroll
    for (int c = 0; c < MD; c++)
        if (MD < 8 || c < d) g = M::acc_gap(g, q[c], M::load(b[c]), M::load(b[d + c]));
    return g;
}

// MD <= 7 (records of 4 or 8 words); leaves of at most 64 points.
template <typename T, int MD, int KT, bool EX, bool NS>
__global__ void __launch_bounds__(kNT)
knn_wave_kernel(TreeView tv, const uint32_t* __restrict__ queries, const int32_t* __restrict__ order,
                int64_t m, int k, int all, int idbits, int32_t* __restrict__ out_idx,
                typename Metric<T>::D* __restrict__ out_dist, int32_t* __restrict__ redo,
                uint32_t* __restrict__ nredo, const uint32_t* __restrict__ split,
                const uint32_t* __restrict__ nbox, const uint32_t* __restrict__ rec) {
    using M = Metric<T>;
    using DT = typename M::D;
    using KL = PackedList<T, KT, EX>;
    const int d = MD < 8 ? MD : tv.d;
    const int64_t i0 = xcd_block() * kNT + threadIdx.x;
    const bool act = i0 < m;
    if (__ballot(act) == 0) return;  // the whole wave is past the end
    const int64_t i = act ? (order ? (int64_t)order[i0] : i0) : 0;
    T q[MD];
    if (act) {
        load_query<T, MD>(tv, queries, all, i, d, q);
    } else {
#pragma unroll
        for (int c = 0; c < MD; c++) q[c] = T(0);
    }
    WaveLane<T, KL> w;
    w.kl.init(idbits);
    w.cnt = 0;
    if (!act) w.kl.kd = DT(-1);  // reaches nothing, takes nothing
    const int64_t n = tv.n;
    const int L = tv.L;
    const uint32_t first_leaf = 1u << L;
    const int na = __popcll(__ballot(act));
    // the wave's leaf tile: one record per lane, read back by broadcast
    constexpr int kRecW = MD <= 3 ? 4 : 8;
    __shared__ uint4 tiles[kNT / kWave][kWave * kRecW / 4];
    uint4* tile = tiles[threadIdx.x / kWave];
    const int lane = lane_id();
    uint32_t cur = 1, prev = 0;
    while (cur != 0) {
        uint32_t next = cur >> 1;
        if (cur >= first_leaf) {
            const int64_t j = cur - first_leaf;
            const int64_t lo = node_start(n, L, j), hi = node_start(n, L, j + 1);
            wave_lds_sync();  // the previous leaf's reads are done
            if (lane < hi - lo) {
                const uint4* src = reinterpret_cast<const uint4*>(rec) + (lo + lane) * (kRecW / 4);
#pragma unroll
                for (int h = 0; h < kRecW / 4; h++) tile[lane * (kRecW / 4) + h] = src[h];
            }
            wave_lds_sync();
            for (int64_t p = lo; p < hi; p++) {
                uint32_t r[kRecW];
#pragma unroll
                for (int h = 0; h < kRecW / 4; h++) {
                    const uint4 v = tile[(p - lo) * (kRecW / 4) + h];
                    r[4 * h] = v.x;
                    r[4 * h + 1] = v.y;
                    r[4 * h + 2] = v.z;
                    r[4 * h + 3] = v.w;
                }
                DT dd = 0;
#pragma unroll
                for (int c = 0; c < MD; c++) dd = M::acc(dd, q[c], M::load(r[c]));
                const uint32_t idw = r[MD];
                bool cand = !(dd > w.kl.kd);
                if constexpr (NS) cand = cand && p != i;
                uint64_t x = 0;
                if constexpr (KL::kFloat) x = ((uint64_t)__float_as_uint(dd) << 32) | idw;
                else x = ((uint64_t)dd << w.kl.B) | idw;
                cand = cand && x < w.kl.kk;
                if (__ballot(cand) != 0) {
#pragma unroll
                    for (int b = 0; b < kWaveBuf; b++) w.buf[b] = (cand && w.cnt == b) ? x : w.buf[b];
                    w.cnt += cand ? 1 : 0;
                }
                // one merge site: a full buffer, or the leaf's last point
                if (p + 1 == hi || __ballot(w.cnt == kWaveBuf) != 0) w.flush(k);
            }
        } else {
            const int lvl = 31 - __clz(cur);
            const int dim = lvl % d;
            const T s = M::load(split[cur]);
            const int right = __popcll(__ballot(act && pick<MD>(q, dim) >= s));
            const uint32_t first = 2u * cur + (2 * right > na ? 1u : 0u);
            const uint32_t second = first ^ 1u;
            auto reach = [&](uint32_t c) {
                return __ballot(!(wave_box_gap<T, MD>(nbox + (size_t)c * 2 * d, q, d) > w.kl.kd)) != 0;
            };
            if (prev < cur) {
                if (reach(first)) next = first;
                else if (reach(second)) next = second;
            } else if (prev == first) {
                if (reach(second)) next = second;
            }
        }
        prev = cur;
        cur = next;
    }
    if (!act) return;
    if (w.kl.needs_redo()) {
        redo[atomicAdd(nredo, 1u)] = (int32_t)i;
        return;
    }
    const int64_t row = all ? (int64_t)tv.pidx[i] : i;
#pragma unroll
    for (int s = 0; s < KT; s++) {
        if (EX || s < k) {
            out_idx[row * k + s] = w.kl.id_of(w.kl.key[s]);
            out_dist[row * k + s] = w.kl.dist_of(w.kl.key[s]);
        }
    }
}

}  // namespace knn_detail
}  // namespace pg
