// C ABI of libpargeo_hip.so: argument validation, handles, memory, errors.
#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "build.hpp"
#include "knn.hpp"
#include "range.hpp"

namespace pg {

namespace {
thread_local std::string g_last_error = "no error";
std::once_flag g_pool_once;

void configure_pool() {
    // Keep freed blocks in the stream-ordered pool instead of returning them
    // at every synchronisation: repeated builds reuse the same memory.
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

pg_status fail(pg_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

namespace {
// The caller's allocator (pg_set_allocator), and the number of device
// blocks not yet released (either allocator's): the allocator may only be
// replaced while none are held, so every block goes back to its maker.
pg_allocator g_alloc = {nullptr, nullptr, nullptr};
std::atomic<int64_t> g_outstanding{0};
}  // namespace

namespace {
// Blocks of at least kCacheMin bytes that the library frees are kept, per
// stream and size class, for the next allocation of that class on that
// stream: stream order makes such a reuse safe without an event, and
// hipMallocAsync / hipFreeAsync of large blocks were measured holding the
// host for 0.05-3 ms each (a B1 rebuild makes a dozen of each).  Classes
// round a size up to a quarter of its power of two (at most 25% slack).
// Cached bytes above the limit (PG_CACHE_LIMIT_MIB, default 8 GiB), or all
// of them on an allocation failure, pg_release_cached or a change of
// allocator, go back to the device after a device synchronisation.
constexpr size_t kCacheMin = (size_t)1 << 20;
std::mutex g_cache_mu;
std::unordered_map<void*, size_t> g_block_class;  // every large block of the default path
std::map<std::pair<hipStream_t, size_t>, std::vector<void*>> g_cache;
size_t g_cached_bytes = 0;

size_t cache_limit() {
    static const size_t lim = [] {
        const char* e = std::getenv("PG_CACHE_LIMIT_MIB");
        return e ? (size_t)std::strtoull(e, nullptr, 10) << 20 : (size_t)8 << 30;
    }();
    return lim;
}

size_t size_class(size_t b) {
    if (b < kCacheMin) return b;
    const int e = 63 - __builtin_clzll((unsigned long long)b);
    const size_t step = (size_t)1 << (e - 2);
    return (b + step - 1) / step * step;
}

// Returns cached blocks to the device until at most `keep` bytes stay
// cached.  Caller holds g_cache_mu.
void trim_locked(size_t keep) {
    if (g_cached_bytes <= keep) return;
    (void)hipDeviceSynchronize();  // the blocks' last uses, on any stream, are done
    for (auto it = g_cache.begin(); it != g_cache.end() && g_cached_bytes > keep;) {
        auto& v = it->second;
        while (!v.empty() && g_cached_bytes > keep) {
            void* q = v.back();
            v.pop_back();
            g_cached_bytes -= it->first.second;
            g_block_class.erase(q);
            (void)hipFreeAsync(q, nullptr);
        }
        it = v.empty() ? g_cache.erase(it) : std::next(it);
    }
}
}  // namespace

pg_status dmalloc(void** p, size_t bytes, hipStream_t s) {
    if (g_alloc.alloc) {
        *p = g_alloc.alloc(bytes ? bytes : 4, (void*)s, g_alloc.ctx);
        if (!*p)
            return fail(PG_ERR_NOMEM, std::string("allocator returned NULL for ") +
                                          std::to_string(bytes) + " bytes");
        g_outstanding++;
        return PG_OK;
    }
    std::call_once(g_pool_once, configure_pool);
    const size_t want = size_class(bytes ? bytes : 4);
    if (want >= kCacheMin) {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        auto it = g_cache.find({s, want});
        if (it != g_cache.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            g_cached_bytes -= want;
            g_outstanding++;
            return PG_OK;
        }
    }
    hipError_t e = hipMallocAsync(p, want, s);
    if (e == hipErrorOutOfMemory && want >= kCacheMin) {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        trim_locked(0);
        (void)hipGetLastError();
        e = hipMallocAsync(p, want, s);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? PG_ERR_NOMEM : PG_ERR_DEVICE,
                    std::string("hipMallocAsync(") + std::to_string(bytes) + "): " +
                        hipGetErrorString(e));
    }
    if (want >= kCacheMin) {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        g_block_class[*p] = want;
    }
    g_outstanding++;
    return PG_OK;
}

void dfree(void* p, hipStream_t s) {
    if (!p) return;
    g_outstanding--;
    if (g_alloc.release) {
        g_alloc.release(p, (void*)s, g_alloc.ctx);
        return;
    }
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        auto it = g_block_class.find(p);
        if (it != g_block_class.end()) {
            g_cache[{s, it->second}].push_back(p);
            g_cached_bytes += it->second;
            if (g_cached_bytes > cache_limit()) trim_locked(cache_limit() / 2);
            return;
        }
    }
    (void)hipFreeAsync(p, s);
}

void release_cached() {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    trim_locked(0);
}

static void tree_release(pg_tree* t) {
    if (!t) return;
    dfree(t->pts, t->stream);
    dfree(t->pidx, t->stream);
    dfree(t->split, t->stream);
    dfree(t->nbox, t->stream);
    dfree(t->rec, t->stream);
    if (t->loff) dfree(t->loff, t->stream);
    if (t->sdim) dfree(t->sdim, t->stream);
    if (t->xn) dfree(t->xn, t->stream);
    if (t->xspan) dfree(t->xspan, t->stream);
    if (t->lnode) dfree(t->lnode, t->stream);
    delete t;
}

}  // namespace pg

using namespace pg;

extern "C" {

const char* pg_last_error(void) { return g_last_error.c_str(); }

const char* pg_version(void) { return "pargeo_hip 0.1 (gfx950)"; }

pg_status pg_set_allocator(const pg_allocator* a) {
    if (a && (!a->alloc || !a->release))
        return fail(PG_ERR_INVALID, "pg_set_allocator: alloc and release must both be set");
    if (g_outstanding.load() != 0)
        return fail(PG_ERR_INVALID, "pg_set_allocator: " + std::to_string(g_outstanding.load()) +
                                        " device blocks are still held (free every handle first)");
    release_cached();
    g_alloc = a ? *a : pg_allocator{nullptr, nullptr, nullptr};
    return PG_OK;
}

pg_status pg_release_cached(void) {
    release_cached();
    return PG_OK;
}

pg_status pg_kdtree_build(const void* points, int64_t n, int32_t d, int32_t leaf, int32_t dtype,
                          void* stream, pg_tree** out) {
    if (!out) return fail(PG_ERR_INVALID, "pg_kdtree_build: out is NULL");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_kdtree_build: d must be in [1, 8]");
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_kdtree_build: leaf must be in [1, 64]");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_kdtree_build: n must be in [0, 2^31)");
    if (dtype != PG_INT32 && dtype != PG_FLOAT32) return fail(PG_ERR_INVALID, "pg_kdtree_build: bad dtype");
    if (n > 0 && !points) return fail(PG_ERR_INVALID, "pg_kdtree_build: points is NULL");
    pg_tree* t = new (std::nothrow) pg_tree();
    if (!t) return fail(PG_ERR_NOMEM, "pg_kdtree_build: host allocation failed");
    pg_status st = build_tree(points, n, d, leaf, dtype, (hipStream_t)stream, t);
    if (st != PG_OK) {
        tree_release(t);
        return st;
    }
    *out = t;
    return PG_OK;
}

pg_status pg_kdtree_build_spatial(const void* points, int64_t n, int32_t d, int32_t leaf,
                                  int32_t dtype, int32_t dim_rule, void* stream, pg_tree** out) {
    if (!out) return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: out is NULL");
    if (d < 1 || d > 8) return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: d must be in [1, 8]");
    if (leaf < 1 || leaf > 64) return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: leaf must be in [1, 64]");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: n must be in [0, 2^31)");
    if (dtype != PG_INT32 && dtype != PG_FLOAT32) return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: bad dtype");
    if (n > 0 && !points) return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: points is NULL");
    if (dim_rule < 0 || dim_rule > 3)
        return fail(PG_ERR_INVALID, "pg_kdtree_build_spatial: dim_rule must be in [0, 3]");
    pg_tree* t = new (std::nothrow) pg_tree();
    if (!t) return fail(PG_ERR_NOMEM, "pg_kdtree_build_spatial: host allocation failed");
    pg_status st = build_tree_spatial(points, n, d, leaf, dtype, dim_rule, (hipStream_t)stream, t);
    if (st != PG_OK) {
        tree_release(t);
        return st;
    }
    *out = t;
    return PG_OK;
}

pg_status pg_tree_offsets(const pg_tree* t, int64_t* loff_host, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_tree_offsets: tree is NULL");
    if (!loff_host) return fail(PG_ERR_INVALID, "pg_tree_offsets: loff_host is NULL");
    const int64_t leaves = t->xn ? t->nleaves : (int64_t)1 << t->L;
    if (t->loff) {
        hipStream_t s = (hipStream_t)stream;
        PG_HIP(hipMemcpyAsync(loff_host, t->loff, sizeof(int64_t) * (leaves + 1),
                              hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    } else {
        for (int64_t j = 0; j <= leaves; j++) loff_host[j] = node_start(t->n, t->L, j);
    }
    return PG_OK;
}

pg_status pg_tree_split_dims(const pg_tree* t, uint8_t* dims_host, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_tree_split_dims: tree is NULL");
    if (!dims_host) return fail(PG_ERR_INVALID, "pg_tree_split_dims: dims_host is NULL");
    if (t->xn) return fail(PG_ERR_UNSUPPORTED, "pg_tree_split_dims: explicit-node tree (use pg_tree_export_nodes)");
    const int64_t nodes = (int64_t)1 << t->L;
    if (t->sdim) {
        hipStream_t s = (hipStream_t)stream;
        PG_HIP(hipMemcpyAsync(dims_host, t->sdim, nodes, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    } else {
        dims_host[0] = 0;
        for (int64_t h = 1; h < nodes; h++) {
            int l = 63 - __builtin_clzll((unsigned long long)h);
            dims_host[h] = (uint8_t)(l % t->d);
        }
    }
    return PG_OK;
}

pg_status pg_knn(const pg_tree* t, const void* queries, int64_t m, int32_t k, int32_t* out_idx,
                 void* out_dist, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_knn: tree is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_knn: k must be in [1, 64]");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_knn: m must be in [0, 2^31)");
    if (m > 0 && (!queries || !out_idx || !out_dist)) return fail(PG_ERR_INVALID, "pg_knn: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    PG_TRY(check_queries(queries, m, t->d, t->dtype == PG_FLOAT32, s));
    return knn_static(t, queries, m, k, false, out_idx, out_dist, s);
}

pg_status pg_knn_all(const pg_tree* t, int32_t k, int32_t* out_idx, void* out_dist, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_knn_all: tree is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_knn_all: k must be in [1, 64]");
    if (t->n > 0 && (!out_idx || !out_dist)) return fail(PG_ERR_INVALID, "pg_knn_all: NULL pointer");
    return knn_static(t, nullptr, t->n, k, true, out_idx, out_dist, (hipStream_t)stream);
}

pg_status pg_range_count(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                         int64_t* offsets, int64_t* total_host, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_range_count: tree is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_range_count: m must be in [0, 2^31)");
    if (m > 0 && (!boxes || !counts)) return fail(PG_ERR_INVALID, "pg_range_count: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    PG_TRY(check_queries(boxes, 2 * m, t->d, t->dtype == PG_FLOAT32, s));
    return range_count(t, boxes, m, counts, offsets, total_host, s);
}

pg_status pg_range_report(const pg_tree* t, const void* boxes, int64_t m, const int64_t* offsets,
                          int32_t* out_idx, int64_t capacity, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_range_report: tree is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_range_report: m must be in [0, 2^31)");
    if (capacity < 0) return fail(PG_ERR_INVALID, "pg_range_report: capacity < 0");
    if (m > 0 && (!boxes || !offsets || (capacity > 0 && !out_idx)))
        return fail(PG_ERR_INVALID, "pg_range_report: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    PG_TRY(check_queries(boxes, 2 * m, t->d, t->dtype == PG_FLOAT32, s));
    return range_report(t, boxes, m, offsets, out_idx, capacity, s);
}

pg_status pg_range_search(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                          int64_t* offsets, int32_t* out_idx, int64_t capacity, int64_t* total_host,
                          void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_range_search: tree is NULL");
    if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PG_ERR_INVALID, "pg_range_search: m must be in [0, 2^31)");
    if (capacity < 0) return fail(PG_ERR_INVALID, "pg_range_search: capacity < 0");
    if (!offsets || (m > 0 && !boxes) || (capacity > 0 && !out_idx))
        return fail(PG_ERR_INVALID, "pg_range_search: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    PG_TRY(check_queries(boxes, 2 * m, t->d, t->dtype == PG_FLOAT32, s));
    return range_search(t, boxes, m, counts, offsets, out_idx, capacity, total_host, s);
}

pg_status pg_knn_graph(const pg_tree* t, int32_t k, int32_t* out_idx, void* out_dist, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_knn_graph: tree is NULL");
    if (k < 1 || k > 64) return fail(PG_ERR_INVALID, "pg_knn_graph: k must be in [1, 64]");
    if (t->n > 0 && (!out_idx || !out_dist)) return fail(PG_ERR_INVALID, "pg_knn_graph: NULL pointer");
    return knn_static(t, nullptr, t->n, k, true, out_idx, out_dist, (hipStream_t)stream, true);
}

pg_status pg_tree_info(const pg_tree* t, int64_t* n, int32_t* d, int32_t* leaf, int32_t* levels,
                       int32_t* dtype) {
    if (!t) return fail(PG_ERR_INVALID, "pg_tree_info: tree is NULL");
    if (n) *n = t->n;
    if (d) *d = t->d;
    if (leaf) *leaf = t->leaf;
    if (levels) *levels = t->L;
    if (dtype) *dtype = t->dtype;
    return PG_OK;
}

pg_status pg_tree_export(const pg_tree* t, void* splits_host, int32_t* perm_host, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_tree_export: tree is NULL");
    if (t->xn) return fail(PG_ERR_UNSUPPORTED, "pg_tree_export: explicit-node tree (use pg_tree_export_nodes)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t ni = ((int64_t)1 << t->L) - 1;
    if (splits_host && ni > 0)
        PG_HIP(hipMemcpyAsync(splits_host, t->split + 1, sizeof(uint32_t) * ni,
                              hipMemcpyDeviceToHost, s));
    if (perm_host && t->n > 0)
        PG_HIP(hipMemcpyAsync(perm_host, t->pidx, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    return PG_OK;
}

pg_status pg_tree_nodes(const pg_tree* t, int64_t* nodes, int64_t* leaves) {
    if (!t) return fail(PG_ERR_INVALID, "pg_tree_nodes: tree is NULL");
    const int64_t heap_leaves = (int64_t)1 << t->L;
    if (nodes) *nodes = t->xn ? t->nnodes : 2 * heap_leaves - 1;
    if (leaves) *leaves = t->xn ? t->nleaves : heap_leaves;
    return PG_OK;
}

pg_status pg_tree_export_nodes(const pg_tree* t, void* split_host, int32_t* dim_host,
                               int64_t* child_host, int64_t* lo_host, int64_t* hi_host,
                               int32_t* level_host, int32_t* perm_host, void* stream) {
    if (!t) return fail(PG_ERR_INVALID, "pg_tree_export_nodes: tree is NULL");
    if (!t->xn) return fail(PG_ERR_UNSUPPORTED, "pg_tree_export_nodes: not an explicit-node tree (use pg_tree_export)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = t->nnodes, NL = t->nleaves;
    std::vector<uint4> xn((size_t)N);
    std::vector<uint2> sp((size_t)N);
    std::vector<int64_t> loff((size_t)NL + 1);
    PG_HIP(hipMemcpyAsync(xn.data(), t->xn, sizeof(uint4) * N, hipMemcpyDeviceToHost, s));
    PG_HIP(hipMemcpyAsync(sp.data(), t->xspan, sizeof(uint2) * N, hipMemcpyDeviceToHost, s));
    PG_HIP(hipMemcpyAsync(loff.data(), t->loff, sizeof(int64_t) * (NL + 1), hipMemcpyDeviceToHost, s));
    if (perm_host && t->n > 0)
        PG_HIP(hipMemcpyAsync(perm_host, t->pidx, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    for (int64_t u = 0; u < N; u++) {
        const bool leaf = (xn[u].w & kXLeaf) != 0;
        if (split_host) ((uint32_t*)split_host)[u] = leaf ? 0u : xn[u].x;
        if (dim_host) dim_host[u] = leaf ? -1 : (int32_t)(xn[u].w & 15u);
        if (child_host) child_host[u] = leaf ? -1 : (int64_t)xn[u].y;
        if (lo_host) lo_host[u] = loff[sp[u].x];
        if (hi_host) hi_host[u] = loff[sp[u].y];
    }
    if (level_host)
        for (size_t l = 0; l + 1 < t->lvl.size(); l++)
            for (int64_t u = t->lvl[l]; u < t->lvl[l + 1]; u++) level_host[u] = (int32_t)l;
    return PG_OK;
}

void pg_tree_free(pg_tree* t) { tree_release(t); }

}  // extern "C"
