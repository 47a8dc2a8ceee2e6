// Internal helpers shared by the kernels and the host runtime of
// libpargeo_hip.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "pargeo_hip.h"

namespace pg {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Errors: thread-local last-error text plus status propagation.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
pg_status fail(pg_status st, const std::string& msg);

#define PG_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return ::pg::fail(e_ == hipErrorOutOfMemory ? PG_ERR_NOMEM : PG_ERR_DEVICE, \
                              std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define PG_LAUNCH_CHECK()                                                         \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess)                                                     \
            return ::pg::fail(PG_ERR_DEVICE, std::string("kernel launch: ") +     \
                                                 hipGetErrorString(e_));         \
    } while (0)

#define PG_TRY(expr)                                                              \
    do {                                                                          \
        pg_status s_ = (expr);                                                    \
        if (s_ != PG_OK) return s_;                                               \
    } while (0)

// Stream-ordered device memory (pool-backed).
pg_status dmalloc(void** p, size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);

template <typename T>
pg_status dalloc(T** p, size_t count, hipStream_t s) {
    return dmalloc(reinterpret_cast<void**>(p), count * sizeof(T), s);
}

// RAII holder for temporaries released in stream order.
struct DevBuf {
    void* p = nullptr;
    hipStream_t s = nullptr;
    DevBuf() = default;
    explicit DevBuf(hipStream_t st) : s(st) {}
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { if (p) dfree(p, s); }
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
    pg_status alloc(size_t bytes) {
        if (p) { dfree(p, s); p = nullptr; }
        return dmalloc(&p, bytes ? bytes : 4, s);
    }
};

// ---------------------------------------------------------------------------
// Order-preserving 32-bit keys of the stored coordinates.
//   int32 : offset binary (x + 2^31)
//   float : sign-magnitude flip (negative: all bits inverted; else sign set)
// Keys compare as unsigned integers exactly as the coordinates compare.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t coord_to_key(uint32_t bits, bool fl) {
    if (!fl) return bits ^ 0x80000000u;
    return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
}
__host__ __device__ inline uint32_t key_to_coord(uint32_t key, bool fl) {
    if (!fl) return key ^ 0x80000000u;
    return (key & 0x80000000u) ? (key & 0x7fffffffu) : ~key;
}

// Keys of an empty box's min and max: at or above / at or below every valid
// coordinate (int32: [-2^29, 2^29); float32: |x| <= 1e18), so min / max
// unions ignore the box, and its coordinates (int32 2^29 - 1 and -2^29,
// float32 +-FLT_MAX) keep the box-distance arithmetic in range.
__host__ __device__ inline uint32_t empty_min_key(bool fl) { return fl ? 0xff7fffffu : 0x9fffffffu; }
__host__ __device__ inline uint32_t empty_max_key(bool fl) { return fl ? 0x00800000u : 0x60000000u; }

// Leaf-order position where node j of level l starts: floor(j n / 2^l).
// Exact in 64 bits: n < 2^31 and j <= 2^32 (levels <= 31).
__host__ __device__ inline int64_t node_start(int64_t n, int l, int64_t j) {
    return (int64_t)(((uint64_t)j * (uint64_t)n) >> l);
}

__host__ inline int tree_levels(int64_t n, int leaf) {
    int L = 0;
    while (((n + ((int64_t)1 << L) - 1) >> L) > leaf) L++;
    return L;
}

// Words of one packed leaf record: d coordinates, the input row, zero
// padding to 4, 8 or 16 words (16, 32 or 64 bytes: whole 16-byte loads).
__host__ __device__ inline int record_words(int d) { return d <= 3 ? 4 : (d <= 7 ? 8 : 16); }

// Static trees allocate this many spare entries after the last leaf-order
// record and row, so a loop that reads them in groups may overrun the last
// group without leaving the allocation (the spare entries hold no data).
constexpr int kTreePad = 4;

// Device view of a static kd-tree (what the search kernels read).
struct TreeView {
    int64_t n;
    int d, L, rw;
    const uint32_t* pts;    // [d][n] coordinates in leaf order (SoA planes)
    const int32_t* pidx;    // [n] input row of each leaf-order point
    const uint32_t* split;  // [2^L] split coordinate of heap node h (h >= 1)
    const uint32_t* bbox;   // [2^L][2d] per leaf: min[d], max[d] coordinates
    const uint32_t* rec;    // [n][rw] leaf-order records: coordinates, row, 0...
    const uint32_t* nbox;   // [2^(L+1)][2d] box of heap node h at h*2d (leaves: = bbox);
                            // null when only the leaf boxes exist
    const int64_t* loff;    // [2^L + 1] leaf j holds positions [loff[j], loff[j+1]);
                            // null: the closed form floor(j n / 2^L) (trees grown
                            // in place keep their splits but not that form)
    const uint8_t* sdim;    // [2^L] split dimension of internal node h; null: level mod d
    // Explicit-node trees (xn != null: spatial-median splits down to at most
    // `leaf` points per node, any depth): nodes numbered breadth-first, root 0,
    // the two children of a node consecutive.  split, bbox and sdim are then
    // unused, nbox is [N][2d] by node, loff is [nleaves + 1] in leaf order.
    const uint4* xn;        // [N] internal {split, first child, parent, meta};
                            //     leaf {leaf index j, 0, parent, meta}
    const uint2* xspan;     // [N] leaf-index span [jlo, jhi) of the node's subtree
    const uint32_t* lnode;  // [nleaves] node of leaf j
    int64_t nleaves;        // leaves (2^L for heap trees)
};

// Meta word of an explicit node: split dimension in bits 0..3, and flags.
constexpr uint32_t kXLeaf = 1u << 8;      // the node is a leaf
constexpr uint32_t kXEmpty = 1u << 9;     // a leaf without points
constexpr uint32_t kXChildLeaf = 1u << 10;   // child s is a leaf: bit 10 + s
constexpr uint32_t kXChildEmpty = 1u << 12;  // child s is an empty leaf: bit 12 + s
constexpr uint32_t kXNone = 0xffffffffu;     // no node (the root's parent)

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace pg

// Handle layout (host side).
struct pg_tree {
    int64_t n = 0;
    int d = 0, leaf = 0, L = 0, dtype = 0;
    hipStream_t stream = nullptr;
    uint32_t* pts = nullptr;
    int32_t* pidx = nullptr;
    uint32_t* split = nullptr;
    uint32_t* nbox = nullptr;  // allocation of every node's box; bbox points into it
    uint32_t* bbox = nullptr;
    uint32_t* rec = nullptr;
    int64_t* loff = nullptr;   // explicit leaf offsets [2^L + 1]; null: closed form
    uint8_t* sdim = nullptr;   // split dimension per internal node; null: level mod d
    // explicit-node trees (see TreeView): L is the number of levels
    uint4* xn = nullptr;
    uint2* xspan = nullptr;
    uint32_t* lnode = nullptr;
    int64_t nnodes = 0, nleaves = 0;
    std::vector<int64_t> lvl;  // host: level l holds nodes [lvl[l], lvl[l+1])
    int rule = 0;              // spatial rule bits the tree was built with
    pg::TreeView view() const {
        return pg::TreeView{n, d, L, pg::record_words(d), pts, pidx, split, bbox, rec, nbox, loff, sdim,
                            xn, xspan, lnode, xn ? nleaves : ((int64_t)1 << L)};
    }
};
