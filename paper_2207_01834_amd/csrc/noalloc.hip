// pg_knn_noalloc: the k-NN of pg_knn for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).  Its temporaries -- the range-check flag, the query
// permutation, the bucket keys and counts of the query ordering, the
// partial sums of their scan, and the redo list of int32 trees -- are carved
// from one file-scope device array instead of the library's allocator.
//
// Each GPU holds its own copy of the array from the library's load on that
// device until the process ends.  Its address is taken once per device, with
// that device current, by hipGetSymbolAddress; host code uses only that
// address.  Every call on a GPU shares the array: calls that overlap on one
// GPU (concurrent streams or threads) race, and must be serialised by the
// caller.  Nothing in it needs to survive a call; the flag and the counters
// are cleared by a fill kernel at the start of each call.
#include <mutex>

#include "knn.hpp"
#include "scan.hpp"

namespace pg {

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
// Largest query count of one call: order, keys and redo list take 4 bytes per
// query each, bucket counts at most 1, plus the flags and partial sums.
constexpr int64_t kNoAllocMaxQueries = (int64_t)1 << 22;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The address of this device's copy of `scratch`.
pg_status scratch_base(uint8_t** out) {
    int dev = 0;
    PG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PG_ERR_UNSUPPORTED, "pg_knn_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PG_ERR_DEVICE, std::string("pg_knn_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<uint8_t*>(g_scratch_ptr[dev]);
    return PG_OK;
}

inline size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

}  // namespace pg

using namespace pg;

extern "C" {

pg_status pg_knn_noalloc(const pg_tree* t, const void* queries, int64_t m, int32_t k, int32_t* out_idx,
                         void* out_dist, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_knn_noalloc: tree is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_knn_noalloc: k must be in [1, 64]");
    if (m < 0 || m > kNoAllocMaxQueries)
        return fail(PG_ERR_INVALID, "pg_knn_noalloc: m must be in [0, 2^22] (the scratch array's limit)");
    if (m > 0 && (!queries || !out_idx || !out_dist)) return fail(PG_ERR_INVALID, "pg_knn_noalloc: NULL pointer");
    if (m == 0) return PG_OK;
    hipStream_t s = (hipStream_t)stream;
    uint8_t* base = nullptr;
    PG_TRY(scratch_base(&base));
    // layout: flag, redo count | order [m] | keys + counts [m + nb] | sums | redo [m]
    const int64_t nb = t->n > 0 ? order_buckets(t->view(), m) : 1;
    size_t off = 256;
    KnnWs ws;
    ws.nredo = reinterpret_cast<uint32_t*>(base + 4);
    ws.order = reinterpret_cast<int32_t*>(base + off);
    off += up256(sizeof(int32_t) * (size_t)m);
    ws.work = reinterpret_cast<uint32_t*>(base + off);
    off += up256(sizeof(uint32_t) * (size_t)(m + nb));
    ws.sums = reinterpret_cast<uint32_t*>(base + off);
    off += up256(sizeof(uint32_t) * (size_t)scan_partials(nb));
    ws.redo = reinterpret_cast<int32_t*>(base + off);
    off += up256(sizeof(int32_t) * (size_t)m);
    if (off > kScratchBytes) return fail(PG_ERR_INVALID, "pg_knn_noalloc: workspace exceeds the scratch array");
    PG_TRY(check_queries_ws(queries, m, t->d, t->dtype == PG_FLOAT32, reinterpret_cast<uint32_t*>(base), s));
    return knn_static(t, queries, m, k, false, out_idx, out_dist, s, false, &ws);
}

}  // extern "C"
