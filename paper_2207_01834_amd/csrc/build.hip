// Static kd-tree construction on the GPU (level-synchronous object-median
// splits).
//
// What is computed (Section 5 and Appendix C, "Parallel vEB Construction":
// one median partition per level, O(n) work per level): node j of level l
// owns leaf-order positions [floor(j n/2^l), floor((j+1) n/2^l)); its left
// child receives the r = floor((2j+1)n/2^(l+1)) - floor(j n/2^l) smallest
// points under (coordinate along dimension l mod d, input row), its right
// child the rest, and the split value is the coordinate of the rank-r point.
//
// How (MI355X): coordinates become order-preserving 32-bit keys stored as SoA
// planes.  Every partition is stable, so each node segment stays in input-row
// order and "ties by input row" becomes "ties by position in the segment".
//   * wide levels (< 1024 nodes of > 4096 points): radix select over 11-bit digits with
//     multi-workgroup LDS histograms merged by global atomics, then a stable
//     scatter whose per-workgroup offsets come from a per-node scan;
//   * middle levels (the other nodes of > S points): one workgroup per node
//     does an 8-bit radix select and the stable partition itself;
//   * bottom levels (node <= S = 1024 points): one workgroup per subtree loads
//     it into LDS, and each wave selects (8-bit digit histograms, or direct
//     ranks for nodes of at most 64 points) and partitions whole nodes until
//     the leaves, then writes the coordinates, the input rows, the split
//     values and the per-leaf bounding boxes.  A small S keeps several
//     subtrees per compute unit, which hides the latency of the top subtree
//     levels, where only one or two waves of a workgroup have a node.
#include <utility>

#include "build.hpp"
#include "build_dev.hpp"
#include "wave.hpp"

namespace pg {

namespace {

constexpr int kNT = kBuildNT;       // threads per workgroup
constexpr int kChunk = 8192;        // elements per histogram workgroup in the wide levels
constexpr int kScat = 1024;         // elements per count/scatter workgroup in the wide levels
constexpr int kWideDigit = 11;      // radix digit width in the wide levels
constexpr int kWideNodes = 1024;    // levels with fewer nodes use the wide path...
constexpr int64_t kWideMinPts = 4096;  // ...while their nodes hold more points than this
constexpr int kBoxLevels = 8;       // tree levels of internal boxes per launch

struct NodeSel {
    uint32_t prefix;  // selected key bits so far; the pivot key at the end
    uint32_t rank;    // target rank among keys matching prefix; at the end the
                      // number of pivot-equal keys that go left
};

__device__ inline int64_t split_rank_pos(int64_t n, int l, int64_t j, int64_t* lo,
                                         int64_t* hi, int64_t* mid) {
    *lo = node_start(n, l, j);
    *hi = node_start(n, l, j + 1);
    *mid = node_start(n, l + 1, 2 * j + 1);
    return (*mid < *hi ? *mid : *hi - 1) - *lo;
}

// ---------------------------------------------------------------------------
// Ingest: caller's [n][d] rows -> key planes + input-row plane; range check;
// -0.0 -> +0.0; per-dimension OR of (key ^ key of row 0).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT)
ingest_kernel(const uint32_t* __restrict__ in, int64_t n, int d, int fl,
              uint32_t* __restrict__ keys, int32_t* __restrict__ idx,
              uint32_t* __restrict__ vary, uint32_t* __restrict__ keybase,
              uint32_t* __restrict__ err) {
    __shared__ uint32_t s_vary[8];
    __shared__ uint32_t s_err;
    if (threadIdx.x < 8) s_vary[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    uint32_t k0[8], vl[8];
#pragma unroll
    for (int c = 0; c < 8; c++) {
        uint32_t b0 = c < d ? in[c] : 0u;
        if (fl && b0 == 0x80000000u) b0 = 0;
        k0[c] = coord_to_key(b0, fl);
        vl[c] = 0;
    }
    uint32_t bad = 0;
    // grid-stride: few workgroups, so the per-workgroup global atomics stay few
    const int64_t stride = (int64_t)gridDim.x * kNT;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int c = 0; c < 8; c++) {
            if (c < d) {
                uint32_t b = in[i * d + c];
                if (fl) {
                    if (b == 0x80000000u) b = 0;
                    if (!(fabsf(__uint_as_float(b)) <= 1e18f)) bad = 1;  // also NaN, inf
                } else {
                    const int32_t x = (int32_t)b;
                    if (x < -(1 << 29) || x >= (1 << 29)) bad = 1;
                }
                const uint32_t k = coord_to_key(b, fl);
                keys[(int64_t)c * n + i] = k;
                vl[c] |= k ^ k0[c];
            }
        }
        idx[i] = (int32_t)i;
    }
    if (blockIdx.x == 0 && threadIdx.x < d) {
        uint32_t kb = 0;
#pragma unroll
        for (int c = 0; c < 8; c++) kb = (int)threadIdx.x == c ? k0[c] : kb;
        keybase[threadIdx.x] = kb;
    }
#pragma unroll
    for (int c = 0; c < 8; c++) {
        if (c < d) {
            uint32_t v = vl[c];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) v |= __shfl_xor(v, off, kWave);
            if (lane_id() == 0 && v) atomicOr(&s_vary[c], v);
        }
    }
    if (__ballot(bad != 0) != 0 && lane_id() == 0) atomicOr(&s_err, 1u);
    __syncthreads();
    if (threadIdx.x < d && s_vary[threadIdx.x]) atomicOr(&vary[threadIdx.x], s_vary[threadIdx.x]);
    if (threadIdx.x == 0 && s_err) atomicOr(err, 1u);
}

// ---------------------------------------------------------------------------
// Wide levels.
// ---------------------------------------------------------------------------
__global__ void wide_init_kernel(NodeSel* ns, int64_t J, int64_t n, int l, uint32_t prefix0,
                                 int write_split, uint32_t* split_level, int fl) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    int64_t lo, hi, mid;
    int64_t r = split_rank_pos(n, l, j, &lo, &hi, &mid);
    ns[j].prefix = prefix0;
    ns[j].rank = (uint32_t)r;
    if (write_split) split_level[j] = key_to_coord(prefix0, fl);
}

// first: the level's first digit pass, where every node's selected prefix
// is still prefix0 (the selection state is not read).
__global__ void __launch_bounds__(kNT)
wide_hist_kernel(const uint32_t* __restrict__ keys, int64_t n, int l, int bpn,
                 const NodeSel* __restrict__ ns, int shift, int width, int first, uint32_t prefix0,
                 uint32_t* __restrict__ ghist) {
    extern __shared__ uint32_t lh[];
    const int64_t j = blockIdx.x / bpn;
    const int t = blockIdx.x % bpn;
    const int64_t lo = node_start(n, l, j), hi = node_start(n, l, j + 1);
    const int64_t e0 = lo + (int64_t)t * kChunk;
    const int64_t e1 = min(e0 + kChunk, hi);
    const int nb = 1 << width;
    for (int b = threadIdx.x; b < nb; b += kNT) lh[b] = 0;
    __syncthreads();
    const int hs = shift + width;
    const uint64_t pre = (uint64_t)(first ? prefix0 : ns[j].prefix) >> hs;
    constexpr int PER = 8;  // loads issued together
    for (int64_t b = e0 + threadIdx.x; b < e1; b += PER * kNT) {
        uint32_t k[PER];
#pragma unroll
        for (int i = 0; i < PER; i++) k[i] = b + i * kNT < e1 ? keys[b + i * kNT] : 0u;
#pragma unroll
        for (int i = 0; i < PER; i++)
            if (b + i * kNT < e1 && ((uint64_t)k[i] >> hs) == pre)
                atomicAdd(&lh[(k[i] >> shift) & (nb - 1)], 1u);
    }
    __syncthreads();
    uint32_t* gh = ghist + j * nb;
    for (int b = threadIdx.x; b < nb; b += kNT) {
        uint32_t c = lh[b];
        if (c) atomicAdd(&gh[b], c);
    }
}

// first: the selection starts from (prefix0, the node's split rank), as
// wide_init_kernel would have set it.
__global__ void __launch_bounds__(kNT)
wide_select_kernel(uint32_t* __restrict__ ghist, NodeSel* __restrict__ ns, int shift, int width,
                   int last, int first, uint32_t prefix0, int64_t n, int l,
                   uint32_t* __restrict__ split_level, int fl) {
    __shared__ uint32_t lds[kNT / kWave + 1];
    const int64_t j = blockIdx.x;
    const int nb = 1 << width;
    const int per = (nb + kNT - 1) / kNT;  // <= 8
    uint32_t* gh = ghist + j * nb;
    uint32_t loc[8];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        int b = threadIdx.x * per + i;
        loc[i] = (i < per && b < nb) ? gh[b] : 0u;
        sum += loc[i];
    }
    uint32_t prefix, r;
    if (first) {
        int64_t lo, hi, mid;
        prefix = prefix0;
        r = (uint32_t)split_rank_pos(n, l, j, &lo, &hi, &mid);
    } else {
        prefix = ns[j].prefix;
        r = ns[j].rank;
    }
    uint32_t tot;
    uint32_t excl = block_excl_scan<kNT>(sum, lds, &tot);
    if (sum > 0 && excl <= r && r < excl + sum) {
        uint32_t cum = excl;
        for (int i = 0; i < per; i++) {
            if (r < cum + loc[i]) {
                uint32_t bin = threadIdx.x * per + i;
                uint32_t np = prefix | (bin << shift);
                ns[j].prefix = np;
                ns[j].rank = r - cum;
                if (last) split_level[j] = key_to_coord(np, fl);
                break;
            }
            cum += loc[i];
        }
    }
    for (int i = 0; i < per; i++) {
        int b = threadIdx.x * per + i;
        if (b < nb) gh[b] = 0;
    }
}

// Per scatter workgroup: the counts (lt | eq << 32) of its keys against the
// pivot, per wave over the part block_partition_range gives that wave
// (wcnt: waves x blocks), and per workgroup (bcnt, which the scan turns into
// offsets): the scatter then skips its own counting pass.
__global__ void __launch_bounds__(kNT)
wide_count_kernel(const uint32_t* __restrict__ keys, int64_t n, int l, int bpn,
                  const NodeSel* __restrict__ ns, uint64_t* __restrict__ bcnt,
                  uint64_t* __restrict__ wcnt) {
    constexpr int NW = kNT / kWave;
    __shared__ uint64_t red[NW];
    const int64_t j = blockIdx.x / bpn;
    const int t = blockIdx.x % bpn;
    const int64_t lo = node_start(n, l, j), hi = node_start(n, l, j + 1);
    const int64_t e0 = lo + (int64_t)t * kScat;
    const int64_t e1 = min(e0 + kScat, hi);
    const uint32_t v = ns[j].prefix;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t part = (e1 - e0 + NW - 1) / NW;
    const int64_t s0 = e0 + w * part < e1 ? e0 + w * part : e1;
    const int64_t s1 = s0 + part < e1 ? s0 + part : e1;
    uint32_t nlt = 0, neq = 0;
    constexpr int PER = 4;  // 64-element groups per step: their loads are issued together
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
            nlt += (uint32_t)__popcll(__ballot(valid && k[i] < v));
            neq += (uint32_t)__popcll(__ballot(valid && k[i] == v));
        }
    }
    const uint64_t acc = (uint64_t)nlt | ((uint64_t)neq << 32);
    if (lane == 0) {
        red[w] = acc;
        wcnt[(int64_t)blockIdx.x * NW + w] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < NW; i++) s += red[i];
        bcnt[blockIdx.x] = s;
    }
}

// Per node: exclusive scan of the per-workgroup (lt, eq) counts.
__global__ void __launch_bounds__(kNT)
wide_scan_kernel(uint64_t* __restrict__ bcnt, int bpn) {
    __shared__ uint64_t lds[kNT / kWave + 1];
    uint64_t* b = bcnt + (int64_t)blockIdx.x * bpn;
    constexpr int PER = 8;  // consecutive counts per thread
    uint64_t run = 0;
    for (int t0 = 0; t0 < bpn; t0 += PER * kNT) {
        const int t = t0 + PER * threadIdx.x;
        uint64_t v[PER];
        uint64_t sum = 0;
#pragma unroll
        for (int i = 0; i < PER; i++) {
            v[i] = t + i < bpn ? b[t + i] : 0ull;
            sum += v[i];
        }
        uint64_t tot;
        uint64_t ex = run + block_excl_scan<kNT>(sum, lds, &tot);
#pragma unroll
        for (int i = 0; i < PER; i++) {
            if (t + i < bpn) b[t + i] = ex;
            ex += v[i];
        }
        run += tot;
    }
}

__global__ void __launch_bounds__(kNT)
wide_scatter_kernel(const uint32_t* __restrict__ in, const int32_t* __restrict__ in_idx,
                    uint32_t* __restrict__ out, int32_t* __restrict__ out_idx, int d, int c,
                    int64_t n, int l, int bpn, const NodeSel* __restrict__ ns,
                    const uint64_t* __restrict__ boff, const uint64_t* __restrict__ wcnt) {
    __shared__ uint32_t lds[2 * (kNT / kWave)];
    const int64_t j = blockIdx.x / bpn;
    const int t = blockIdx.x % bpn;
    int64_t lo, hi, mid;
    split_rank_pos(n, l, j, &lo, &hi, &mid);
    const int64_t e0 = lo + (int64_t)t * kScat;
    const int64_t e1 = min(e0 + kScat, hi);
    const uint32_t v = ns[j].prefix, teq = ns[j].rank;
    block_partition_range(in, in_idx, out, out_idx, d, c, n, e0, e1, lo, mid, hi, v, teq,
                          (uint32_t)(boff[blockIdx.x] & 0xffffffffull),
                          (uint32_t)(boff[blockIdx.x] >> 32), lds,
                          wcnt + (int64_t)blockIdx.x * (kNT / kWave));
}

// ---------------------------------------------------------------------------
// Middle levels: one workgroup per node selects (8-bit digits) and partitions.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT)
node_kernel(const uint32_t* __restrict__ in, const int32_t* __restrict__ in_idx,
            uint32_t* __restrict__ out, int32_t* __restrict__ out_idx, int d, int c, int64_t n,
            int l, uint32_t prefix0, int sb, uint32_t* __restrict__ split_level, int fl) {
    __shared__ uint32_t sh[272];
    const int64_t j = blockIdx.x;
    int64_t lo, hi, mid;
    split_rank_pos(n, l, j, &lo, &hi, &mid);
    block_node_split(in, in_idx, out, out_idx, d, c, n, lo, hi, mid, prefix0, sb,
                     &split_level[j], fl != 0, sh);
}

// ---------------------------------------------------------------------------
// Bottom levels: one workgroup per subtree, in LDS.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kNT)
subtree_kernel(const uint32_t* __restrict__ in, const int32_t* __restrict__ in_idx, int64_t n,
               int d, int L, int ls, int S, int fl, uint32_t* __restrict__ out_pts,
               int32_t* __restrict__ out_idx, uint32_t* __restrict__ split,
               uint32_t* __restrict__ bbox, uint32_t* __restrict__ rec) {
    extern __shared__ uint32_t sm[];
    block_subtree(in, in_idx, n, d, L, ls, blockIdx.x, S, fl != 0, out_pts, out_idx, split, bbox,
                  rec, sm);
}

// ---------------------------------------------------------------------------
// Internal bounding boxes (the subtree boxes the search of Appendix C prunes
// by): box(h) = union of box(2h) and box(2h+1), heap-indexed, min[d] then
// max[d].  A workgroup reads the 2^b boxes of level lt below one node of
// level lt-b and writes the b levels above them, ping-ponging two LDS tiles
// of order-preserving keys.  An empty leaf (leaf size 1 only) carries the box
// of the point 0, which only widens its ancestors' boxes.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kNT)
node_box_kernel(uint32_t* __restrict__ box, int d, int lt, int b, int fl) {
    extern __shared__ uint32_t sm[];
    const int w = 2 * d;
    const int G = 1 << b;
    uint32_t* cur = sm;
    uint32_t* nxt = sm + G * w;
    const int64_t base = (((int64_t)1 << lt) + (int64_t)blockIdx.x * G) * w;
    for (int e = threadIdx.x; e < G * w; e += kNT) cur[e] = coord_to_key(box[base + e], fl != 0);
    __syncthreads();
    for (int r = 1; r <= b; r++) {
        const int cnt = G >> r;
        const int64_t out = (((int64_t)1 << (lt - r)) + (int64_t)blockIdx.x * cnt) * w;
        for (int e = threadIdx.x; e < cnt * w; e += kNT) {
            const int u = e / w, c = e - u * w;
            const uint32_t a = cur[2 * u * w + c], o = cur[(2 * u + 1) * w + c];
            const uint32_t v = c < d ? (a < o ? a : o) : (a > o ? a : o);
            nxt[e] = v;
            box[out + e] = key_to_coord(v, fl != 0);
        }
        __syncthreads();
        uint32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
}

}  // namespace

int subtree_capacity(int) { return 1024; }

pg_status ingest_points(const void* points, int64_t n, int d, bool fl, uint32_t* keys,
                        int32_t* idx, uint32_t* vary_host, uint32_t* keybase_host,
                        hipStream_t s) {
    DevBuf aux(s);
    PG_TRY(aux.alloc(sizeof(uint32_t) * 17));
    uint32_t* vary = aux.as<uint32_t>();
    uint32_t* keybase = vary + 8;
    uint32_t* err = vary + 16;
    PG_HIP(hipMemsetAsync(vary, 0, sizeof(uint32_t) * 17, s));
    if (n > 0) {
        const unsigned grid = cdiv(n, kNT) < 2048u ? cdiv(n, kNT) : 2048u;
        hipLaunchKernelGGL(ingest_kernel, dim3(grid), dim3(kNT), 0, s,
                           (const uint32_t*)points, n, d, fl ? 1 : 0, keys, idx, vary, keybase,
                           err);
        PG_LAUNCH_CHECK();
    }
    uint32_t host[17];
    PG_HIP(hipMemcpyAsync(host, vary, sizeof(host), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (host[16]) return fail(PG_ERR_RANGE, "coordinate out of range (int32: [-2^29, 2^29); float32: finite, |x| <= 1e18)");
    for (int c = 0; c < d; c++) {
        vary_host[c] = host[c];
        keybase_host[c] = host[8 + c];
    }
    return PG_OK;
}

pg_status build_from_keys(uint32_t* kA, int32_t* iA, uint32_t* kB, int32_t* iB, int64_t n,
                          int d, int leaf, bool fl, const uint32_t* vary,
                          const uint32_t* keybase, hipStream_t s, pg_tree* T) {
    const int L = T->L;
    const int S = subtree_capacity(d);
    int ls = 0;
    while (((n + ((int64_t)1 << ls) - 1) >> ls) > S) ls++;
    const int ifl = fl ? 1 : 0;

    uint32_t* cur_k = kA;
    int32_t* cur_i = iA;
    uint32_t* oth_k = kB;
    int32_t* oth_i = iB;

    DevBuf nsel(s), ghist(s), bcnt(s);
    int wide_levels = 0;
    // a wide level costs seven launches, a node level one: smaller builds
    // (launch-bound) move to node levels once nodes hold few points
    while (wide_levels < ls && ((int64_t)1 << wide_levels) < kWideNodes &&
           (n >> wide_levels) > kWideMinPts)
        wide_levels++;
    int64_t blocks_max = 1;  // scatter workgroups of the widest level
    if (wide_levels > 0) {
        const int64_t Jmax = (int64_t)1 << (wide_levels - 1);
        for (int l = 0; l < wide_levels; l++) {
            const int64_t J = (int64_t)1 << l;
            const int64_t b = J * (int64_t)cdiv((n + J - 1) / J, kScat);
            blocks_max = b > blocks_max ? b : blocks_max;
        }
        PG_TRY(nsel.alloc(sizeof(NodeSel) * Jmax));
        PG_TRY(ghist.alloc(sizeof(uint32_t) * Jmax * (1 << kWideDigit)));
        PG_TRY(bcnt.alloc(sizeof(uint64_t) * blocks_max * (1 + kNT / kWave)));
        PG_HIP(hipMemsetAsync(ghist.p, 0, sizeof(uint32_t) * Jmax * (1 << kWideDigit), s));
    }

    for (int l = 0; l < ls; l++) {
        const int64_t J = (int64_t)1 << l;
        const int c = l % d;
        const int sb = vary[c] ? 32 - __builtin_clz(vary[c]) : 0;
        const uint32_t lowmask = sb >= 32 ? 0xffffffffu : ((1u << sb) - 1u);
        const uint32_t prefix0 = keybase[c] & ~lowmask;
        uint32_t* split_level = T->split + J;
        if (l < wide_levels) {
            const int64_t smax = (n + J - 1) / J;
            const int bpn = (int)cdiv(smax, kChunk);
            const unsigned nblk = (unsigned)(J * bpn);
            const int spn = (int)cdiv(smax, kScat);
            const unsigned nsblk = (unsigned)(J * spn);
            NodeSel* ns = nsel.as<NodeSel>();
            if (sb == 0) {
                // every key of the dimension is equal: no digit pass
                hipLaunchKernelGGL(wide_init_kernel, dim3(cdiv(J, kNT)), dim3(kNT), 0, s, ns, J, n, l,
                                   prefix0, 1, split_level, ifl);
                PG_LAUNCH_CHECK();
            }
            for (int hb = sb; hb > 0; hb -= kWideDigit) {
                const int shift = hb > kWideDigit ? hb - kWideDigit : 0;
                const int width = hb - shift;
                const int first = hb == sb ? 1 : 0;
                const uint32_t* keys = cur_k + (int64_t)c * n;
                hipLaunchKernelGGL(wide_hist_kernel, dim3(nblk), dim3(kNT),
                                   sizeof(uint32_t) << width, s, keys, n, l, bpn, ns, shift,
                                   width, first, prefix0, ghist.as<uint32_t>());
                PG_LAUNCH_CHECK();
                hipLaunchKernelGGL(wide_select_kernel, dim3((unsigned)J), dim3(kNT), 0, s,
                                   ghist.as<uint32_t>(), ns, shift, width, shift == 0 ? 1 : 0, first,
                                   prefix0, n, l, split_level, ifl);
                PG_LAUNCH_CHECK();
            }
            uint64_t* wcnt = bcnt.as<uint64_t>() + blocks_max;
            hipLaunchKernelGGL(wide_count_kernel, dim3(nsblk), dim3(kNT), 0, s,
                               cur_k + (int64_t)c * n, n, l, spn, ns, bcnt.as<uint64_t>(), wcnt);
            PG_LAUNCH_CHECK();
            hipLaunchKernelGGL(wide_scan_kernel, dim3((unsigned)J), dim3(kNT), 0, s,
                               bcnt.as<uint64_t>(), spn);
            PG_LAUNCH_CHECK();
            hipLaunchKernelGGL(wide_scatter_kernel, dim3(nsblk), dim3(kNT), 0, s, cur_k, cur_i,
                               oth_k, oth_i, d, c, n, l, spn, ns, bcnt.as<uint64_t>(), wcnt);
            PG_LAUNCH_CHECK();
        } else {
            hipLaunchKernelGGL(node_kernel, dim3((unsigned)J), dim3(kNT), 0, s, cur_k, cur_i,
                               oth_k, oth_i, d, c, n, l, prefix0, sb, split_level, ifl);
            PG_LAUNCH_CHECK();
        }
        std::swap(cur_k, oth_k);
        std::swap(cur_i, oth_i);
    }

    // LDS for the largest subtree present (ceil(n / 2^ls) <= S points), so
    // that more workgroups fit on a compute unit
    const int64_t smax = (n + ((int64_t)1 << ls) - 1) >> ls;
    const int Se = smax < 1 ? 1 : (int)smax;
    const size_t lds = subtree_lds_bytes(d, Se);
    hipLaunchKernelGGL(subtree_kernel, dim3((unsigned)((int64_t)1 << ls)), dim3(kNT), lds, s,
                       cur_k, cur_i, n, d, L, ls, Se, ifl, T->pts, T->pidx, T->split, T->bbox,
                       T->rec);
    PG_LAUNCH_CHECK();
    return internal_boxes(T, s);
}

namespace {
// Leaf boxes of a tree with explicit leaf offsets, from its points, as
// order-preserving keys first (starting from the empty box, which an empty
// leaf keeps), then converted to coordinates.
__global__ void box_keys_init_kernel(uint32_t* __restrict__ box, int64_t leaves, int d, int fl) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e < leaves * 2 * d) box[e] = (e % (2 * d)) < d ? empty_min_key(fl != 0) : empty_max_key(fl != 0);
}

// One lane per leaf-order position.  Positions of a wave are consecutive,
// so lanes of one leaf are contiguous: a segmented min/max toward the first
// lane of each leaf, then one atomic per (leaf, dimension) and wave.
__global__ void __launch_bounds__(kNT)
offset_leaf_box_kernel(TreeView tv, int fl, uint32_t* __restrict__ box) {
    const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const bool valid = p < tv.n;
    if (__ballot(valid) == 0) return;
    uint32_t j = 0xffffffffu;
    if (valid) {
        uint32_t lo = 0, hi = 1u << tv.L;  // loff[lo] <= p < loff[hi]
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
            atomicMin(&box[(int64_t)j * 2 * d + c], mn);
            atomicMax(&box[(int64_t)j * 2 * d + d + c], mx);
        }
    }
}

__global__ void box_keys_to_coords_kernel(uint32_t* __restrict__ box, int64_t count, int fl) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e < count) box[e] = key_to_coord(box[e], fl != 0);
}
}  // namespace

pg_status offset_boxes(pg_tree* T, hipStream_t s) {
    const int64_t leaves = (int64_t)1 << T->L;
    const int64_t count = leaves * 2 * T->d;
    const int fl = T->dtype == PG_FLOAT32 ? 1 : 0;
    hipLaunchKernelGGL(box_keys_init_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s, T->bbox,
                       leaves, T->d, fl);
    PG_LAUNCH_CHECK();
    if (T->n > 0) {
        hipLaunchKernelGGL(offset_leaf_box_kernel, dim3(cdiv(T->n, kNT)), dim3(kNT), 0, s,
                           T->view(), fl, T->bbox);
        PG_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(box_keys_to_coords_kernel, dim3(cdiv(count, kNT)), dim3(kNT), 0, s, T->bbox,
                       count, fl);
    PG_LAUNCH_CHECK();
    return internal_boxes(T, s);
}

pg_status internal_boxes(pg_tree* T, hipStream_t s) {
    // bottom-up, kBoxLevels levels per launch
    const int d = T->d;
    const int ifl = T->dtype == PG_FLOAT32 ? 1 : 0;
    for (int lt = T->L; lt > 0;) {
        const int b = lt < kBoxLevels ? lt : kBoxLevels;
        hipLaunchKernelGGL(node_box_kernel, dim3((unsigned)((int64_t)1 << (lt - b))), dim3(kNT),
                           sizeof(uint32_t) * 2 * (2 * d) << b, s, T->nbox, d, lt, b, ifl);
        PG_LAUNCH_CHECK();
        lt -= b;
    }
    return PG_OK;
}

pg_status build_tree(const void* points, int64_t n, int d, int leaf, int dtype, hipStream_t s,
                     pg_tree* T) {
    const bool fl = dtype == PG_FLOAT32;
    T->n = n;
    T->d = d;
    T->leaf = leaf;
    T->dtype = dtype;
    T->stream = s;
    T->L = tree_levels(n, leaf);
    const int64_t nleaves = (int64_t)1 << T->L;
    const int64_t nn = n > 0 ? n : 1;
    PG_TRY(dalloc(&T->pts, (size_t)d * nn, s));
    PG_TRY(dalloc(&T->pidx, (size_t)nn + kTreePad, s));
    PG_TRY(dalloc(&T->split, (size_t)nleaves, s));
    PG_TRY(dalloc(&T->nbox, (size_t)nleaves * 2 * 2 * d, s));
    T->bbox = T->nbox + (size_t)nleaves * 2 * d;
    PG_TRY(dalloc(&T->rec, ((size_t)nn + kTreePad) * record_words(d), s));
    if (n == 0) return PG_OK;
    DevBuf tmpk(s), tmpi(s);
    PG_TRY(tmpk.alloc(sizeof(uint32_t) * (size_t)d * n));
    PG_TRY(tmpi.alloc(sizeof(int32_t) * (size_t)n));
    uint32_t vary[8] = {0}, keybase[8] = {0};
    // Keys go into the tree's own arrays first; the bottom-level pass reads
    // each subtree into LDS before writing coordinates back in place.
    PG_TRY(ingest_points(points, n, d, fl, T->pts, T->pidx, vary, keybase, s));
    return build_from_keys(T->pts, T->pidx, tmpk.as<uint32_t>(), tmpi.as<int32_t>(), n, d, leaf,
                           fl, vary, keybase, s, T);
}

}  // namespace pg
