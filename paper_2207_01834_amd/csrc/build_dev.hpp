// Workgroup- and wave-level pieces of the kd-tree construction, shared by
// the static build (build.hip) and the batched persistent kernel (batch.hip).
// All node ranges follow the closed form of the construction: node j of
// level l owns positions [floor(j n/2^l), floor((j+1) n/2^l)) of its tree.
#pragma once

#include "common.hpp"
#include "wave.hpp"

namespace pg {

constexpr int kBuildNT = 256;  // threads of every build workgroup

// Stable partition of the elements [c0, c1) of a node [lo, end_node) whose
// left child ends at mid, around pivot key v (keys < v go left, then the
// first teq keys == v, the rest right); base_lt / base_eq count the node's
// keys < v / == v before c0.  The workgroup's waves each take one contiguous
// part of the chunk: they count it with ballots, exchange their totals
// through LDS (lds: >= 2 * waves words), then scatter their part in order,
// positions from ballot prefix counts.  Contains barriers.  wcnt (may be
// NULL): the waves' counts (lt | eq << 32), already taken over the same
// parts, so the counting pass is skipped.
__device__ inline void block_partition_range(const uint32_t* __restrict__ in,
                                             const int32_t* __restrict__ in_idx,
                                             uint32_t* __restrict__ out,
                                             int32_t* __restrict__ out_idx, int d, int c,
                                             int64_t n, int64_t c0, int64_t c1, int64_t lo,
                                             int64_t mid, int64_t end_node, uint32_t v,
                                             uint32_t teq, uint32_t base_lt, uint32_t base_eq,
                                             uint32_t* lds, const uint64_t* __restrict__ wcnt = nullptr) {
    constexpr int NW = kBuildNT / kWave;
    constexpr int PER = 4;  // 64-element groups per step: their loads are issued together
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t part = (c1 - c0 + NW - 1) / NW;
    const int64_t s0 = c0 + w * part < c1 ? c0 + w * part : c1;
    const int64_t s1 = s0 + part < c1 ? s0 + part : c1;
    const uint32_t* keys = in + (int64_t)c * n;
    uint32_t run_lt = base_lt, run_eq = base_eq;
    if (wcnt) {
        for (int i = 0; i < w; i++) {
            run_lt += (uint32_t)wcnt[i];
            run_eq += (uint32_t)(wcnt[i] >> 32);
        }
    } else {
        uint32_t nlt = 0, neq = 0;
        for (int64_t b0 = s0; b0 < s1; b0 += PER * kWave) {
            uint32_t k[PER];
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int64_t e = b0 + i * kWave + lane;
                k[i] = e < s1 ? keys[e] : 0u;
            }
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const bool valid = b0 + i * kWave + lane < s1;
                nlt += (uint32_t)__popcll(ballot(valid && k[i] < v));
                neq += (uint32_t)__popcll(ballot(valid && k[i] == v));
            }
        }
        if (lane == 0) {
            lds[w] = nlt;
            lds[NW + w] = neq;
        }
        __syncthreads();
        for (int i = 0; i < w; i++) {
            run_lt += lds[i];
            run_eq += lds[NW + i];
        }
        __syncthreads();
    }
    for (int64_t b0 = s0; b0 < s1; b0 += PER * kWave) {
        uint32_t k[PER];
        int32_t ix[PER];
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const int64_t e = b0 + i * kWave + lane;
            k[i] = e < s1 ? keys[e] : 0u;
            ix[i] = e < s1 ? in_idx[e] : 0;
        }
        // destinations, groups in element order so the running counts stay
        // in order
        int64_t dst[PER];
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const int64_t e = b0 + i * kWave + lane;
            const bool valid = e < s1;
            const bool lt = valid && k[i] < v;
            const bool eq = valid && k[i] == v;
            const uint64_t mlt = ballot(lt), meq = ballot(eq);
            const uint32_t ltb = run_lt + lane_prefix(mlt);
            const uint32_t eqb = run_eq + lane_prefix(meq);
            const uint32_t el = eqb < teq ? eqb : teq;
            int64_t dest;
            if (lt) dest = lo + ltb + el;
            else if (eq && eqb < teq) dest = lo + ltb + eqb;
            else dest = mid + (e - lo) - (int64_t)(ltb + el);
            // always inside the node for a consistent split
            dst[i] = valid && dest >= lo && dest < end_node ? dest : -1;
            run_lt += (uint32_t)__popcll(mlt);
            run_eq += (uint32_t)__popcll(meq);
        }
        // then plane by plane, the group's loads issued before its stores;
        // a step whose elements are all in the range stores without
        // per-lane branches, so the stores are not held up one by one
        if (b0 + PER * kWave <= s1) {
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int64_t e = b0 + i * kWave + lane;
                dst[i] = dst[i] >= 0 ? dst[i] : e;  // (an inconsistent split keeps the element)
            }
            for (int cc = 0; cc < d; cc++) {
                uint32_t val[PER];
#pragma unroll
                for (int i = 0; i < PER; i++)
                    val[i] = cc == c ? k[i] : in[(int64_t)cc * n + b0 + i * kWave + lane];
#pragma unroll
                for (int i = 0; i < PER; i++) out[(int64_t)cc * n + dst[i]] = val[i];
            }
#pragma unroll
            for (int i = 0; i < PER; i++) out_idx[dst[i]] = ix[i];
        } else {
            for (int cc = 0; cc < d; cc++) {
                uint32_t val[PER];
#pragma unroll
                for (int i = 0; i < PER; i++) {
                    const int64_t e = b0 + i * kWave + lane;
                    val[i] = cc == c ? k[i] : (dst[i] >= 0 ? in[(int64_t)cc * n + e] : 0u);
                }
#pragma unroll
                for (int i = 0; i < PER; i++)
                    if (dst[i] >= 0) out[(int64_t)cc * n + dst[i]] = val[i];
            }
#pragma unroll
            for (int i = 0; i < PER; i++)
                if (dst[i] >= 0) out_idx[dst[i]] = ix[i];
        }
    }
}

// wave_select_partition for a node of at most NS * 64 elements: lane t
// holds elements t, t + 64, ... (pin order); each element's rank under
// (key, position) is counted against every element, broadcast with
// readlane (a uniform loop); the left child takes the ranks below mid - lo,
// in order.  Returns the key of rank r.
template <int NS>
__device__ inline uint32_t wave_rank_partition(const uint32_t* keys, const uint16_t* pin,
                                               uint16_t* pout, int lo, int hi, int mid,
                                               uint32_t r) {
    const int lane = lane_id();
    const int m = hi - lo;
    const bool right_empty = mid >= hi;
    uint16_t p[NS];
    uint32_t k[NS], rank[NS];
#pragma unroll
    for (int u = 0; u < NS; u++) {
        const int e = u * kWave + lane;
        p[u] = e < m ? pin[lo + e] : (uint16_t)0;
        k[u] = e < m ? keys[p[u]] : 0u;
        rank[u] = 0;
    }
#pragma unroll
    for (int sv = 0; sv < NS; sv++) {
        const int cnt = m - sv * kWave < kWave ? m - sv * kWave : kWave;
        for (int j = 0; j < cnt; j++) {
            const uint32_t kj = __builtin_amdgcn_readlane(k[sv], j);
            const int pj = sv * kWave + j;
#pragma unroll
            for (int u = 0; u < NS; u++) {
                const int pi = u * kWave + lane;
                rank[u] += (kj < k[u] || (kj == k[u] && pj < pi)) ? 1u : 0u;
            }
        }
    }
    uint32_t v = 0;
    int nl = 0, nr = 0;  // left / right elements of the earlier slots
#pragma unroll
    for (int u = 0; u < NS; u++) {
        const bool valid = u * kWave + lane < m;
        const uint64_t hit = ballot(valid && rank[u] == r);
        if (hit != 0) v = __builtin_amdgcn_readlane(k[u], __ffsll((unsigned long long)hit) - 1);
        const bool left = right_empty || rank[u] < (uint32_t)(mid - lo);
        const uint64_t ml = ballot(valid && left), mr = ballot(valid && !left);
        if (valid) pout[left ? lo + nl + (int)lane_prefix(ml) : mid + nr + (int)lane_prefix(mr)] = p[u];
        nl += __popcll(ml);
        nr += __popcll(mr);
    }
    return v;
}

// One wave selects the rank-r key of node [lo, hi) (local positions, order
// given by pin) and writes the stable partition into pout.  Returns the
// split key.  mid == hi (right child empty) splits at the largest key and
// sends everything left.  Selection: a node of at most 64 elements ranks
// them directly (wave_rank_partition); a larger node's min and max fix
// the common high key bits and the bits below are resolved 8 at a time with
// a 256-bin LDS histogram private to the wave (whist).
__device__ inline uint32_t wave_select_partition(const uint32_t* keys, const uint16_t* pin,
                                                 uint16_t* pout, int lo, int hi, int mid,
                                                 uint32_t* whist) {
    const int lane = lane_id();
    const bool right_empty = mid >= hi;
    uint32_t r = (uint32_t)((right_empty ? hi - 1 : mid) - lo);
    if (hi - lo <= kWave) return wave_rank_partition<1>(keys, pin, pout, lo, hi, mid, r);
    uint32_t mn = 0xffffffffu, mx = 0;
    for (int e = lo + lane; e < hi; e += kWave) {
        const uint32_t k = keys[pin[e]];
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
    }
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    uint32_t prefix = mn;
    if (mn != mx) {
        const int hb = 31 - __clz(mn ^ mx);  // highest differing bit
        prefix = hb == 31 ? 0u : (mn & ~((2u << hb) - 1u));
        for (int top = hb + 1; top > 0; top -= 8) {  // digit = key bits [shift, top)
            const int shift = top > 8 ? top - 8 : 0;
            const uint32_t wmask = (1u << (top - shift)) - 1u;
            const uint64_t want = (uint64_t)prefix >> top;
            whist[4 * lane] = 0;
            whist[4 * lane + 1] = 0;
            whist[4 * lane + 2] = 0;
            whist[4 * lane + 3] = 0;
            wave_lds_sync();
            for (int e = lo + lane; e < hi; e += kWave) {
                const uint32_t k = keys[pin[e]];
                if (((uint64_t)k >> top) == want) atomicAdd(&whist[(k >> shift) & wmask], 1u);
            }
            wave_lds_sync();
            const uint32_t c0 = whist[4 * lane], c1 = whist[4 * lane + 1];
            const uint32_t c2 = whist[4 * lane + 2], c3 = whist[4 * lane + 3];
            const uint32_t sum = c0 + c1 + c2 + c3;
            const uint32_t incl = wave_incl_scan(sum);
            const uint32_t excl = incl - sum;
            const bool mine = excl <= r && r < incl;
            const uint64_t who = ballot(mine);
            const int owner = __ffsll((unsigned long long)who) - 1;
            uint32_t bin = 0, below = excl;
            if (mine) {
                if (r < below + c0) bin = 0;
                else if (r < below + c0 + c1) { bin = 1; below += c0; }
                else if (r < below + c0 + c1 + c2) { bin = 2; below += c0 + c1; }
                else { bin = 3; below += c0 + c1 + c2; }
            }
            bin = __shfl(bin + 4u * (uint32_t)lane, owner, kWave);
            below = __shfl(below, owner, kWave);
            wave_lds_sync();  // every lane has read the bins before the next clear
            prefix |= bin << shift;
            r -= below;
        }
    }
    const uint32_t v = prefix;
    const uint32_t teq = right_empty ? 0xffffffffu : r;
    uint32_t run_lt = 0, run_eq = 0;
    for (int e0 = lo; e0 < hi; e0 += kWave) {
        const int e = e0 + lane;
        const bool valid = e < hi;
        const uint16_t p = valid ? pin[e] : (uint16_t)0;
        const uint32_t k = valid ? keys[p] : 0u;
        const bool lt = valid && k < v;
        const bool eq = valid && k == v;
        const uint64_t mlt = ballot(lt), meq = ballot(eq);
        const uint32_t ltb = run_lt + lane_prefix(mlt);
        const uint32_t eqb = run_eq + lane_prefix(meq);
        if (valid) {
            const uint32_t el = eqb < teq ? eqb : teq;
            int dest;
            if (lt) dest = lo + (int)(ltb + el);
            else if (eq && eqb < teq) dest = lo + (int)(ltb + eqb);
            else dest = mid + (e - lo) - (int)(ltb + el);
            if (dest >= lo && dest < hi) pout[dest] = p;  // always true for a consistent split
        }
        run_lt += (uint32_t)__popcll(mlt);
        run_eq += (uint32_t)__popcll(meq);
    }
    return v;
}


// Workgroup-wide min and max of keys[lo, hi).  sh: >= kBuildNT/64 * 2 words.
__device__ inline void block_minmax(const uint32_t* __restrict__ keys, int64_t lo, int64_t hi,
                                    uint32_t* sh, uint32_t* mn_out, uint32_t* mx_out) {
    constexpr int NW = kBuildNT / kWave;
    uint32_t mn = 0xffffffffu, mx = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += kBuildNT) {
        const uint32_t k = keys[e];
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
    }
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        sh[w] = mn;
        sh[NW + w] = mx;
    }
    __syncthreads();
    uint32_t a = sh[0], b = sh[NW];
    for (int i = 1; i < NW; i++) {
        a = sh[i] < a ? sh[i] : a;
        b = sh[NW + i] > b ? sh[NW + i] : b;
    }
    __syncthreads();
    *mn_out = a;
    *mx_out = b;
}

// One workgroup splits node [lo, hi) (mid < hi) of a tree whose planes have
// stride n: 8-bit radix select of the rank (mid - lo) key along plane c over
// the low `sb` key bits (the higher bits equal prefix0 for every key of the
// node), then a stable partition of all planes and input rows into `out`.
// Writes the split coordinate to *split_out.  sh: >= 264 words of LDS.
__device__ inline void block_node_split(const uint32_t* __restrict__ in,
                                        const int32_t* __restrict__ in_idx,
                                        uint32_t* __restrict__ out, int32_t* __restrict__ out_idx,
                                        int d, int c, int64_t n, int64_t lo, int64_t hi,
                                        int64_t mid, uint32_t prefix0, int sb,
                                        uint32_t* __restrict__ split_out, bool fl, uint32_t* sh) {
    uint32_t* hist = sh;              // [256]
    uint32_t* lds = sh + 256;         // [NT/64 + 1]
    uint32_t* sel = sh + 256 + kBuildNT / kWave + 1;  // [2]
    uint32_t r = (uint32_t)(mid - lo);
    const uint32_t* keys = in + (int64_t)c * n;
    uint32_t prefix = prefix0;
    for (int hb = sb; hb > 0; hb -= 8) {
        const int shift = hb > 8 ? hb - 8 : 0;
        const uint32_t wmask = (1u << (hb - shift)) - 1u;
        hist[threadIdx.x] = 0;
        __syncthreads();
        const uint64_t pre = (uint64_t)prefix >> hb;
        constexpr int PER = 8;  // loads issued together
        for (int64_t b = lo + threadIdx.x; b < hi; b += PER * kBuildNT) {
            uint32_t k[PER];
#pragma unroll
            for (int i = 0; i < PER; i++) k[i] = b + i * kBuildNT < hi ? keys[b + i * kBuildNT] : 0u;
#pragma unroll
            for (int i = 0; i < PER; i++)
                if (b + i * kBuildNT < hi && ((uint64_t)k[i] >> hb) == pre)
                    atomicAdd(&hist[(k[i] >> shift) & wmask], 1u);
        }
        __syncthreads();
        const uint32_t cnt = hist[threadIdx.x];
        uint32_t tot;
        const uint32_t ex = block_excl_scan<kBuildNT>(cnt, lds, &tot);
        if (cnt > 0 && ex <= r && r < ex + cnt) {
            sel[0] = prefix | ((uint32_t)threadIdx.x << shift);
            sel[1] = r - ex;
        }
        __syncthreads();
        prefix = sel[0];
        r = sel[1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *split_out = key_to_coord(prefix, fl);
    block_partition_range(in, in_idx, out, out_idx, d, c, n, lo, hi, lo, mid, hi, prefix, r, 0u,
                          0u, lds);
}

// LDS bytes of block_subtree for subtrees of up to S points.
__host__ __device__ inline size_t subtree_lds_bytes(int d, int S) {
    return (size_t)d * S * 4 + (size_t)S * 4 + (size_t)S * 4 + (kBuildNT / kWave) * 256 * 4;
}

// One workgroup finishes the subtree rooted at node j0 of level ls (at most S
// points): loads it into LDS, and a wave per node selects (bitwise radix with
// ballots) and stable-partitions every node down to the leaves at level L.
// Writes the coordinates and input rows in leaf order (as planes and as packed
// records), the split values of the subtree's nodes and its leaves' bounding
// boxes.  `in` and `out_pts` may
// alias (the subtree is read completely before it is written).
__device__ inline void block_subtree(const uint32_t* in, const int32_t* in_idx, int64_t n, int d,
                                     int L, int ls, int64_t j0, int S, bool fl, uint32_t* out_pts,
                                     int32_t* out_idx, uint32_t* __restrict__ split,
                                     uint32_t* __restrict__ bbox, uint32_t* __restrict__ rec,
                                     uint32_t* sm) {
    uint32_t* skeys = sm;                                    // [d][S]
    int32_t* sidx = (int32_t*)(sm + (size_t)d * S);          // [S]
    uint16_t* pa = (uint16_t*)(sidx + S);                    // [S]
    uint16_t* pb = pa + S;                                   // [S]
    uint32_t* hists = (uint32_t*)(pb + S);                   // [waves][256]
    const int64_t base = node_start(n, ls, j0);
    const int s = (int)(node_start(n, ls, j0 + 1) - base);
    for (int e = threadIdx.x; e < s; e += kBuildNT) {
        for (int c = 0; c < d; c++) skeys[c * S + e] = in[(int64_t)c * n + base + e];
        sidx[e] = in_idx[base + e];
        pa[e] = (uint16_t)e;
    }
    __syncthreads();
    const int w = threadIdx.x / kWave;
    constexpr int NW = kBuildNT / kWave;
    uint16_t* pin = pa;
    uint16_t* pout = pb;
    for (int t = 0; t < L - ls; t++) {
        const int l = ls + t;
        const int c = l % d;
        const int nodes = 1 << t;
        for (int u = w; u < nodes; u += NW) {
            const int64_t jj = (j0 << t) + u;
            const int lo = (int)(node_start(n, l, jj) - base);
            const int hi = (int)(node_start(n, l, jj + 1) - base);
            const int mid = (int)(node_start(n, l + 1, 2 * jj + 1) - base);
            const uint32_t v = wave_select_partition(skeys + c * S, pin, pout, lo, hi, mid,
                                                     hists + 256 * w);
            if (lane_id() == 0) split[((int64_t)1 << l) + jj] = key_to_coord(v, fl);
        }
        __syncthreads();
        uint16_t* tmp = pin;
        pin = pout;
        pout = tmp;
    }
    const int rw = record_words(d);
    for (int e = threadIdx.x; e < s; e += kBuildNT) {
        const int p = pin[e];
        uint32_t* r = rec + (base + e) * rw;
        for (int c = 0; c < d; c++) {
            const uint32_t v = key_to_coord(skeys[c * S + p], fl);
            out_pts[(int64_t)c * n + base + e] = v;
            r[c] = v;
        }
        out_idx[base + e] = sidx[p];
        r[d] = (uint32_t)sidx[p];
        for (int c = d + 1; c < rw; c++) r[c] = 0;
    }
    const int nl = 1 << (L - ls);
    for (int q = threadIdx.x; q < nl * d; q += kBuildNT) {
        const int leafl = q / d, c = q % d;
        const int64_t jj = (j0 << (L - ls)) + leafl;
        const int llo = (int)(node_start(n, L, jj) - base);
        const int lhi = (int)(node_start(n, L, jj + 1) - base);
        uint32_t mn = 0xffffffffu, mx = 0;
        for (int e = llo; e < lhi; e++) {
            const uint32_t k = skeys[c * S + pin[e]];
            mn = k < mn ? k : mn;
            mx = k > mx ? k : mx;
        }
        if (llo == lhi) {  // empty leaf (leaf size 1 only)
            mn = empty_min_key(fl);
            mx = empty_max_key(fl);
        }
        bbox[jj * 2 * d + c] = key_to_coord(mn, fl);
        bbox[jj * 2 * d + d + c] = key_to_coord(mx, fl);
    }
    __syncthreads();
}

}  // namespace pg
