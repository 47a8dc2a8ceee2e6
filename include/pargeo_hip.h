/*
 * pargeo_hip.h -- C ABI of libpargeo_hip.so, a GPU (AMD Instinct MI355X,
 * gfx950) implementation of the kd-tree hot path of ParGeo (Wang et al.,
 * "ParGeo: A Library for Parallel Computational Geometry", ESA 2022):
 * kd-tree construction and batched k-nearest-neighbour search, static and in
 * the batch-dynamic BDL-tree form.
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers unless marked (host).  Point and query
 *     arrays are row-major [count][d], 32-bit coordinates of the given dtype.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it; calls that must report a data-dependent error or count (marked
 *     "synchronises") wait for the stream before returning.
 *   - Argument errors (bad sizes, null pointers) are returned before anything
 *     is enqueued and leave every output untouched.  pg_last_error() then
 *     gives a message (thread-local).
 *   - Coordinates: int32 values must lie in [-2^29, 2^29) (so squared
 *     distances are exact in int64 for d <= 8); float32 values must be finite
 *     with |x| <= 1e18.  -0.0 is stored as +0.0.
 *   - k-NN results: for each query the k points with the smallest
 *     (squared Euclidean distance, id) keys in ascending order (ties in
 *     distance go to the smaller id).  Squared distances are exact int64 for
 *     int32 input, float32 for float32 input.  When fewer than k points
 *     exist the remaining slots hold id -1 and distance INT64_MAX / +inf.
 *   - Handles are owned by the library until the matching *_free call; the
 *     caller's input arrays are copied and may be reused once the stream has
 *     passed the call.  Device memory is stream-ordered (hipMallocAsync).
 */
#ifndef PARGEO_HIP_H
#define PARGEO_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PG_OK = 0,
    PG_ERR_INVALID = 1,     /* bad argument (size, pointer, handle)          */
    PG_ERR_RANGE = 2,       /* coordinate out of range / non-finite          */
    PG_ERR_NOMEM = 3,       /* device allocation failed                      */
    PG_ERR_DEVICE = 4,      /* a HIP call or kernel launch failed            */
    PG_ERR_UNSUPPORTED = 5  /* valid request the library does not serve     */
} pg_status;

typedef enum { PG_INT32 = 0, PG_FLOAT32 = 1 } pg_dtype;

typedef struct pg_tree pg_tree;
typedef struct pg_bdl pg_bdl;

/* Device memory.  By default the library allocates stream-ordered from the
 * device's pool (hipMallocAsync / hipFreeAsync) and keeps the blocks of
 * 1 MiB or more that it frees, per stream and size class (sizes rounded up
 * by at most a quarter), for its next allocation of that class on that
 * stream; up to PG_CACHE_LIMIT_MIB (environment, default 8192) MiB stay
 * cached.  pg_release_cached returns them to the device (after a device
 * synchronisation), as an allocation failure does first; call it before
 * destroying a stream the library has run on, so that no block stays
 * filed under a stream handle the runtime may hand out again, and before
 * making another device current (the release synchronises and frees on the
 * current device).
 * pg_set_allocator installs the caller's allocator instead (a framework's
 * caching allocator, say):
 * alloc(bytes, stream, ctx) returns device memory usable in stream order on
 * `stream` (NULL on failure: the call returns PG_ERR_NOMEM), release(p,
 * stream, ctx) takes back a block after the work queued on `stream` so far.
 * NULL restores the default.  Returns PG_ERR_INVALID while the library
 * holds any device block (free every handle first, so each block goes back
 * to the allocator that made it) or when only one of the two functions is
 * given.  Not thread-safe against concurrent library calls. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* ctx);
    void (*release)(void* p, void* stream, void* ctx);
    void* ctx;
} pg_allocator;
pg_status pg_set_allocator(const pg_allocator* a);
/* Returns the default path's cached blocks to the device (synchronises the
 * device).  Not thread-safe against concurrent library calls. */
pg_status pg_release_cached(void);

/* Text of the last non-OK status on this thread (never NULL). */
const char* pg_last_error(void);
/* Library version string (host). */
const char* pg_version(void);

/* ---------------------------------------------------------------------- */
/* Static kd-tree                                                          */
/* ---------------------------------------------------------------------- */

/* Builds a kd-tree over n points (Section 5; Appendix C, "Parallel vEB
 * Construction" / Algorithm 1: object-median splits, one median partition
 * per level).  Readings: the split dimension of level l is l mod d; node j of
 * level l holds leaf-order positions [floor(j n/2^l), floor((j+1) n/2^l)) and
 * its left child takes the floor((2j+1)n/2^(l+1)) - floor(j n/2^l) smallest
 * points under (coordinate, input row); every leaf sits at depth
 * L = min{L : ceil(n/2^L) <= leaf}, so a leaf holds at most `leaf` points.
 * The split value of a node is the coordinate of its right child's smallest
 * point (the largest left point when the right child is empty).
 *   points : [n][d] int32 or float32 (dtype), device
 *   n      : 0 <= n < 2^31        d : 1..8        leaf : 1..64
 *   out    : (host) receives the handle
 * Synchronises (one 8-byte read of the range check).  PG_ERR_RANGE if a
 * coordinate is out of range. */
pg_status pg_kdtree_build(const void* points, int64_t n, int32_t d, int32_t leaf,
                          int32_t dtype, void* stream, pg_tree** out);

/* Builds a kd-tree by spatial-median splits (the alternative split rule
 * Section 6.3 measures: a node's space is cut in half along a dimension),
 * split, as Section 5 defines a kd-tree, until a node holds a small constant
 * number of points.  Readings: a node holding at most `leaf` points, or only
 * identical points, is a leaf; the root's space is the bounding box of the
 * points; a node cuts its cell (dim_rule bit 1 clear) or the bounding box of
 * its own points (bit 1 set) along dimension depth mod d (bit 0 clear) or
 * along the space's widest side, the lowest dimension on ties (bit 0 set);
 * the cut s of space [lo, hi] (lo < hi) is floor((lo + hi + 1) / 2) for
 * int32 and the float nearest (lo + hi) / 2 for float32 (the next float above
 * lo when that is lo itself), s = lo when lo == hi; points with coordinate
 * < s go to the first child (cell [lo, s-], s- the value just below s), the
 * others to the second (cell [s, hi]), each side keeping the parent's order.
 * The result is an explicit-node tree of any depth: nodes numbered
 * breadth-first (root 0, the two children of a node consecutive), leaves
 * holding at most `leaf` points apart from identical points, empty leaves
 * where a cut leaves one side empty.  pg_tree_nodes and
 * pg_tree_export_nodes describe it; pg_tree_offsets gives the leaf ranges in
 * leaf order; every query call accepts it (pg_knn, pg_knn_all,
 * pg_knn_graph, pg_range_*).  Arguments and errors as pg_kdtree_build;
 * dim_rule in [0, 3]. */
pg_status pg_kdtree_build_spatial(const void* points, int64_t n, int32_t d, int32_t leaf,
                                  int32_t dtype, int32_t dim_rule, void* stream, pg_tree** out);

/* Split dimension of every internal heap node (host, [2^L] bytes, index 0
 * unused): l mod d.  PG_ERR_UNSUPPORTED for explicit-node trees
 * (pg_kdtree_build_spatial), which pg_tree_export_nodes describes. */
pg_status pg_tree_split_dims(const pg_tree* t, uint8_t* dims_host, void* stream);

/* Number of nodes and of leaves (host outputs; either may be NULL): 2^(L+1)
 * - 1 and 2^L for trees from pg_kdtree_build, the node and leaf counts of
 * explicit-node trees. */
pg_status pg_tree_nodes(const pg_tree* t, int64_t* nodes, int64_t* leaves);

/* Copies an explicit-node tree out, in its breadth-first numbering (host
 * arrays of pg_tree_nodes' node count N; any may be NULL; synchronises):
 *   split_host : [N] 32-bit cut values (int32 or float32 per dtype; 0 for leaves)
 *   dim_host   : [N] cut dimension, -1 for leaves
 *   child_host : [N] first child (the second is child + 1), -1 for leaves
 *   lo_host, hi_host : [N] the node's leaf-order positions [lo, hi)
 *   level_host : [N] depth (root 0)
 *   perm_host  : [n] input rows in leaf order
 * PG_ERR_UNSUPPORTED for trees from pg_kdtree_build (pg_tree_export). */
pg_status pg_tree_export_nodes(const pg_tree* t, void* split_host, int32_t* dim_host,
                               int64_t* child_host, int64_t* lo_host, int64_t* hi_host,
                               int32_t* level_host, int32_t* perm_host, void* stream);

/* Leaf offsets (host, [leaves + 1], leaves from pg_tree_nodes): leaf j holds
 * leaf-order positions [loff[j], loff[j+1]) (the closed form
 * floor(j n / 2^L) for trees from pg_kdtree_build).  Synchronises for
 * spatial-median trees. */
pg_status pg_tree_offsets(const pg_tree* t, int64_t* loff_host, void* stream);

/* k-NN of m query points over the tree (Appendix C, "Data-Parallel k-NN":
 * queries in parallel, each search serial).
 *   queries  : [m][d], same dtype as the tree, device
 *   k        : 1..64
 *   out_idx  : [m][k] int32, input row of each neighbour (-1 = none)
 *   out_dist : [m][k] int64 (int32 trees) or float32 (float32 trees)
 * Synchronises (query range check). */
pg_status pg_knn(const pg_tree* t, const void* queries, int64_t m, int32_t k,
                 int32_t* out_idx, void* out_dist, void* stream);

/* pg_knn for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, results and range check (it synchronises), with every temporary
 * taken from a 64 MiB device array the library holds on each GPU it runs on
 * until the process ends, instead of from the allocator.
 *   m : 0 <= m <= 2^22 (4,194,304); larger m is PG_ERR_INVALID, nothing runs
 * Calls share that array on a GPU: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller. */
pg_status pg_knn_noalloc(const pg_tree* t, const void* queries, int64_t m, int32_t k,
                         int32_t* out_idx, void* out_dist, void* stream);

/* All-points k-NN: the queries are the tree's own n points (each point is
 * its own first neighbour unless an identical point has a smaller row).
 * Output row i belongs to input row i.  Does not synchronise. */
pg_status pg_knn_all(const pg_tree* t, int32_t k, int32_t* out_idx, void* out_dist,
                     void* stream);

/* k-NN graph (the graph generator of Section 2's third module, built on the
 * tree's k-NN search): row i holds the k points nearest to input row i
 * other than row i itself, in the pg_knn_all layout and order (an
 * identical point is a neighbour at distance 0).  When fewer than k other
 * points exist the remaining slots are padded.  Rows are directed edges
 * i -> out_idx[i][r].  Does not synchronise. */
pg_status pg_knn_graph(const pg_tree* t, int32_t k, int32_t* out_idx, void* out_dist,
                       void* stream);

/* Tree facts (host outputs; any may be NULL); levels: L for trees from
 * pg_kdtree_build, the number of depths (deepest node's depth + 1) for
 * explicit-node trees. */
pg_status pg_tree_info(const pg_tree* t, int64_t* n, int32_t* d, int32_t* leaf,
                       int32_t* levels, int32_t* dtype);

/* Copies a tree from pg_kdtree_build out for inspection (synchronises;
 * PG_ERR_UNSUPPORTED for explicit-node trees, see pg_tree_export_nodes):
 *   splits_host : (host) [2^L - 1] 32-bit split values of heap nodes 1..2^L-1
 *                 (node h has children 2h, 2h+1; node 2^l + j is node j of
 *                 level l), int32 or float32 per dtype
 *   perm_host   : (host) [n] int32 input rows in leaf order; leaf j holds
 *                 positions [floor(j n/2^L), floor((j+1) n/2^L)) */
pg_status pg_tree_export(const pg_tree* t, void* splits_host, int32_t* perm_host,
                         void* stream);

/* Well-separated pair decomposition of the tree's points (Section 2's
 * second module generates it from the kd-tree; the recursive pairing of
 * Callahan and Kosaraju).  Readings: a node's ball is centred at its
 * bounding box's centre with the half diagonal as radius; nodes a, b are
 * well separated for s when |c_a - c_b|^2 >= (s + 2)^2 r^2, r the larger
 * radius (in double: half side (hi - lo) * 0.5, centre (lo + hi) * 0.5,
 * sums over dimensions in order, no fused multiply-adds); every internal
 * node starts with the pair of its children; an unseparated pair splits the
 * node of larger radius (the first on ties, never a leaf); pairs with an
 * empty node are dropped.  With leaf size 1 every pair of distinct points
 * lies in exactly one pair.
 *   t          : a tree from pg_kdtree_build with leaf 1 (PG_ERR_UNSUPPORTED
 *                otherwise)
 *   s          : separation, positive and finite
 *   out_pairs  : [capacity][2] uint32, device, 8-byte aligned: heap node
 *                indices (a, b), a on the first child's side of the node
 *                that started the pairing; node 2^l + j holds leaf-order
 *                positions [floor(j n/2^l), floor((j+1) n/2^l)) (rows via
 *                pg_tree_export's perm); pairs come round by round of the
 *                refinement, in a fixed order
 *   count_host : (host) receives the number of pairs
 * When there are more than `capacity` pairs the first `capacity` are
 * written, *count_host is set and PG_ERR_INVALID returned (capacity 0 only
 * counts).  Synchronises once per refinement round. */
pg_status pg_wspd(const pg_tree* t, double s, uint32_t* out_pairs, int64_t capacity,
                  int64_t* count_host, void* stream);

/* Releases the tree (stream-ordered on the stream it was built on). */
void pg_tree_free(pg_tree* t);

/* Orthogonal range search over the tree (the kd-tree range query of the
 * paper's first module, Section 2, timed in Table 1; queries in parallel as
 * in Appendix C).  Reading, where the paper does not define the query: a
 * query is a closed axis-aligned box, and its result is every point p with
 * lo_c <= p_c <= hi_c for all c (empty when lo_c > hi_c for some c);
 * coordinates compare as values (-0.0 == +0.0).
 *   boxes : [m][2][d] device, the tree's dtype: lo[d] then hi[d] per box;
 *           coordinates obey the build's range rules
 *   0 <= m < 2^31
 *
 * Counting pass.
 *   counts     : [m] int32, number of points in each box
 *   offsets    : [m+1] int64 or NULL; receives the exclusive prefix sum of
 *                counts (offsets[m] = total), the layout pg_range_report
 *                writes
 *   total_host : (host, may be NULL) receives the total; then synchronises
 * Synchronises (box range check). */
pg_status pg_range_count(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                         int64_t* offsets, int64_t* total_host, void* stream);

/* Reporting pass: the input rows of box i's points go to
 * out_idx[offsets[i] ...], in the tree's leaf order (deterministic for a
 * given tree; sort a box's slice for row order).
 *   offsets  : [m] int64 device, normally from pg_range_count
 *   out_idx  : [capacity] int32 device
 * A slot at or beyond `capacity` is never written; if one was needed the
 * call returns PG_ERR_INVALID after the launch (the other slots are
 * written).  Synchronises (box range check, overflow flag). */
pg_status pg_range_report(const pg_tree* t, const void* boxes, int64_t m, const int64_t* offsets,
                          int32_t* out_idx, int64_t capacity, void* stream);

/* Both passes in one call (the boxes are checked and put in walking order
 * once): counts, offsets and, when the total fits, the rows.
 *   counts     : [m] int32 device, or NULL (a temporary is used)
 *   offsets    : [m+1] int64 device (required): exclusive prefix sum of the
 *                counts, offsets[m] = total
 *   out_idx    : [capacity] int32 device; box i's rows at offsets[i] ...,
 *                leaf order as in pg_range_report
 *   total_host : (host, may be NULL) receives the total
 * When the total exceeds `capacity`, returns PG_ERR_INVALID with counts,
 * offsets and *total_host written and out_idx untouched; a caller can then
 * size out_idx and call pg_range_report with these offsets.  Synchronises. */
pg_status pg_range_search(const pg_tree* t, const void* boxes, int64_t m, int32_t* counts,
                          int64_t* offsets, int32_t* out_idx, int64_t capacity,
                          int64_t* total_host, void* stream);

/* ---------------------------------------------------------------------- */
/* BDL-tree (batch-dynamic kd-tree, Section 5; Appendix C)                 */
/* ---------------------------------------------------------------------- */
/* A buffer tree of fewer than X points plus static kd-trees i = 0, 1, ...
 * of capacity X * 2^i (the logarithmic method).  Every point carries an
 * int64 id: the value of a global insertion counter (0, 1, 2, ... in batch
 * order).  Readings where the paper is silent: bit i of F is set iff static
 * tree i is non-empty; F_new = F + floor(|P|/X); a destroyed tree moves whole
 * into the smallest new tree above it; tree-bound points fill new trees in
 * ascending order; a tree is rebuilt when fewer than X 2^i / 2 of its points
 * are live (the buffer is exempt).
 *
 * A handle (BDL, B1 and B2 alike) keeps device scratch for its erase and
 * k-NN calls from one call to the next, grown as needed and released with
 * the handle: calls on one handle, k-NN included, must not overlap.
 *
 * Creates an empty BDL-tree (host only; no device work).
 *   d : 1..8   dtype : PG_INT32 / PG_FLOAT32   leaf : 1..64
 *   buffer_X : X in [1, 2^31) */
pg_status pg_bdl_create(int32_t d, int32_t dtype, int32_t leaf, int64_t buffer_X, pg_bdl** out);
/* As pg_bdl_create, but every static tree and the buffer tree is built with
 * spatial-median splits (Section 6.3 runs each tree both ways; cells halved
 * as in pg_kdtree_build_spatial with dim_rule 0: split dimension depth mod
 * d, down to at most `leaf` points per leaf).  Results are the same (same
 * definition on the same live set); only the cost differs. */
pg_status pg_bdl_create_spatial(int32_t d, int32_t dtype, int32_t leaf, int64_t buffer_X,
                                pg_bdl** out);

/* Batch insertion (Section 5 "Parallel Batch Insertion"; Algorithm 3).
 *   points   : [m][d] device, the tree's dtype; copied
 *   first_id : (host, may be NULL) id of points[0]; points[r] gets first_id+r
 * Synchronises (range check, tree builds).  PG_ERR_RANGE leaves the tree
 * unchanged; PG_ERR_UNSUPPORTED when a tree would exceed 2^31 points. */
pg_status pg_bdl_insert(pg_bdl* b, const void* points, int64_t m, void* stream,
                        int64_t* first_id);

/* Batch deletion (Algorithms 2 and 4): every live point whose coordinates
 * equal one of the m given points is removed (absent points are no-ops);
 * static trees left below half capacity are gathered and reinserted.
 *   n_erased : (host, may be NULL) number of points removed
 * Synchronises. */
pg_status pg_bdl_erase(pg_bdl* b, const void* points, int64_t m, void* stream,
                       int64_t* n_erased);

/* Data-parallel k-NN over the live points of all trees (Section 5
 * "Data-Parallel k-NN": one k-NN buffer per query carried across the
 * trees, largest tree first).  While every id is below 2^31 the buffer
 * holds packed (distance, id) keys; int32 queries whose k-th key reaches
 * the packed range's limit are searched again with exact pairs.
 *   out_id   : [m][k] int64 ids (-1 = none)
 *   out_dist : [m][k] int64 / float32 squared distances
 * Synchronises (query range check). */
pg_status pg_bdl_knn(const pg_bdl* b, const void* queries, int64_t m, int32_t k,
                     int64_t* out_id, void* out_dist, void* stream);

/* Number of live points (host; -1 for a NULL handle). */
int64_t pg_bdl_size(const pg_bdl* b);

/* Host-side state: F (bit i = static tree i non-empty), live buffer points,
 * live points of static trees 0..max_trees-1 (any output may be NULL). */
pg_status pg_bdl_stats(const pg_bdl* b, int64_t* tree_mask, int64_t* buffer_count,
                       int64_t* live_counts, int32_t max_trees);

/* Releases every tree and the handle's scratch (stream-ordered on the
 * streams they were made on). */
void pg_bdl_free(pg_bdl* b);

/* ---------------------------------------------------------------------- */
/* B1: the first baseline of Section 6.3 (rebuild on every batch)          */
/* ---------------------------------------------------------------------- */
/* One static kd-tree over all live points, rebuilt from scratch after every
 * insert batch and after every erase batch that removes a point.  Ids and
 * results as in the BDL-tree (same definition on the same live set). */
typedef struct pg_b1 pg_b1;

/* Creates an empty B1 tree (host only).  d 1..8, leaf 1..64. */
pg_status pg_b1_create(int32_t d, int32_t dtype, int32_t leaf, pg_b1** out);
/* As pg_b1_create, rebuilding with spatial-median splits
 * (pg_kdtree_build_spatial, dim_rule 0). */
pg_status pg_b1_create_spatial(int32_t d, int32_t dtype, int32_t leaf, pg_b1** out);
/* Inserts m device points and rebuilds.  first_id as in pg_bdl_insert.
 * Synchronises.  PG_ERR_UNSUPPORTED beyond 2^31 - 1 points. */
pg_status pg_b1_insert(pg_b1* b, const void* points, int64_t m, void* stream, int64_t* first_id);
/* Removes every live point equal to one of the m given points, then
 * rebuilds over the rest.  n_erased as in pg_bdl_erase.  Synchronises. */
pg_status pg_b1_erase(pg_b1* b, const void* points, int64_t m, void* stream, int64_t* n_erased);
/* k-NN over the live points; layout and order as pg_bdl_knn.
 * Synchronises (query range check). */
pg_status pg_b1_knn(const pg_b1* b, const void* queries, int64_t m, int32_t k, int64_t* out_id,
                    void* out_dist, void* stream);
/* Live points (host; -1 for a NULL handle). */
int64_t pg_b1_size(const pg_b1* b);
/* Releases the tree and the handle's scratch. */
void pg_b1_free(pg_b1* b);

/* ---------------------------------------------------------------------- */
/* B2: the second baseline of Section 6.3 (batch updates without           */
/* rebalancing)                                                            */
/* ---------------------------------------------------------------------- */
/* One static kd-tree built over the initial points whose splits never
 * change: an inserted point joins the leaf its descent reaches (right at or
 * above a split), so leaves grow without bound; an erased point becomes a
 * tombstone.  Ids as in the BDL-tree: the initial points get 0..n-1, then
 * an insertion counter continues.  k-NN and erase results are those of the
 * BDL-tree on the same live set (same definition); only the cost differs. */
typedef struct pg_b2 pg_b2;

/* Builds the tree over points [n][d] (device, copied); leaf and ranges as
 * pg_kdtree_build.  Synchronises.  PG_ERR_RANGE on an out-of-range point. */
pg_status pg_b2_create(const void* points, int64_t n, int32_t d, int32_t leaf, int32_t dtype,
                       void* stream, pg_b2** out);
/* As pg_b2_create, with the fixed splits those of the spatial-median tree
 * of the initial points (pg_kdtree_build_spatial, dim_rule 0); an inserted
 * point descends by the same rule (coordinate < cut: first child), and may
 * join an empty leaf. */
pg_status pg_b2_create_spatial(const void* points, int64_t n, int32_t d, int32_t leaf,
                               int32_t dtype, void* stream, pg_b2** out);
/* Inserts m device points in place (new arrays of the grown size; leaf and
 * internal boxes recomputed).  first_id as in pg_bdl_insert.  Synchronises
 * (range check).  PG_ERR_UNSUPPORTED beyond 2^31 - 1 stored points. */
pg_status pg_b2_insert(pg_b2* b, const void* points, int64_t m, void* stream, int64_t* first_id);
/* Tombstones every live point equal to one of the m given points (no
 * rebalancing, no rebuild).  n_erased as in pg_bdl_erase.  Synchronises. */
pg_status pg_b2_erase(pg_b2* b, const void* points, int64_t m, void* stream, int64_t* n_erased);
/* k-NN over the live points; layout and order as pg_bdl_knn.
 * Synchronises (query range check). */
pg_status pg_b2_knn(const pg_b2* b, const void* queries, int64_t m, int32_t k, int64_t* out_id,
                    void* out_dist, void* stream);
/* Live points (host; -1 for a NULL handle). */
int64_t pg_b2_size(const pg_b2* b);
/* Stored points including tombstones, and the tree's depth (host outputs,
 * either may be NULL). */
pg_status pg_b2_stats(const pg_b2* b, int64_t* stored, int32_t* levels);
/* Releases the tree and the handle's scratch. */
void pg_b2_free(pg_b2* b);

/* ---------------------------------------------------------------------- */
/* Batched uneven clouds (float32) and the differentiable k-NN backward    */
/* ---------------------------------------------------------------------- */
/* Where the per-query k-list of the batched launch lives. */
typedef enum { PG_KLIST_DEFAULT = 0, PG_KLIST_VGPR = 1, PG_KLIST_LDS = 2 } pg_klist;

/* Tuning of the batched launch; 0 = default.  Every setting gives identical
 * results. */
typedef struct {
    int32_t leaf;           /* leaf size of every cloud's tree (default 16)  */
    int32_t blocks_per_cu;  /* persistent workgroups per compute unit (4)    */
    int32_t lane_queries;   /* queries each lane searches per work item,
                               1..8 (1): a wave takes 64 x lane_queries     */
    int32_t klist;          /* pg_klist: registers (default) or LDS          */
} pg_tune;

typedef struct pg_batch pg_batch;

/* Workspace bytes needed by pg_batch_create for these clouds.
 *   offsets_host : (host) [n_clouds+1], offsets[0] = 0, non-decreasing; cloud c
 *                  is rows [offsets[c], offsets[c+1]) of the point array;
 *                  total rows < 2^31
 *   d : 1..8 */
pg_status pg_batch_workspace(const int64_t* offsets_host, int32_t n_clouds, int32_t d,
                             const pg_tune* tune, size_t* bytes);

/* Plans a batch of clouds: uploads the per-cloud layout (largest cloud
 * first) into `workspace` (device, >= pg_batch_workspace bytes; NULL = the
 * library allocates and owns it).  Synchronises once.  The handle keeps a
 * reference to the workspace, which must outlive it. */
pg_status pg_batch_create(const int64_t* offsets_host, int32_t n_clouds, int32_t d,
                          const pg_tune* tune, void* workspace, size_t workspace_bytes,
                          void* stream, pg_batch** out);

/* Per-cloud all-points k-NN of every cloud (the static search of Appendix C
 * within each cloud), built and queried in one persistent launch with an
 * atomic work queue (preceded by one small reset launch).  Allocates nothing,
 * does not synchronise: may be captured in a HIP graph.  Calls sharing one
 * workspace must not overlap.
 *   points  : [N][d] float32, device (finite, |x| <= 1e18: see pg_batch_check)
 *   out_idx : [N][k] int32 global rows of the neighbours (-1 = none)
 *   out_d2  : [N][k] float32 squared distances */
pg_status pg_batch_knn_self(pg_batch* b, const float* points, int32_t k, int32_t* out_idx,
                            float* out_d2, void* stream);

/* k-NN of a separate query set per cloud (the static search of Appendix C
 * within each cloud, from the root), in the same persistent launch:
 * every cloud's tree is built from `points` as in pg_batch_knn_self and
 * cloud c's queries search it.  A cloud may have points and no queries,
 * queries and no points (their rows are padding), or neither.
 *   points         : [N][d] float32, device (the clouds of pg_batch_create)
 *   queries        : [M][d] float32, device (finite, |x| <= 1e18)
 *   q_offsets_host : (host) [n_clouds+1], q_offsets[0] = 0, non-decreasing;
 *                    cloud c's queries are rows [q_offsets[c], q_offsets[c+1]);
 *                    M = q_offsets[n_clouds] < 2^31
 *   out_idx        : [M][k] int32 global rows of the neighbours (-1 = none)
 *   out_d2         : [M][k] float32 squared distances
 * The handle keeps the last query layout: a call with the same q_offsets
 * uploads nothing, allocates nothing and does not synchronise (it may be
 * captured in a HIP graph); a call with new q_offsets uploads them and
 * synchronises once.  Calls sharing one workspace must not overlap. */
pg_status pg_batch_knn(pg_batch* b, const float* points, const float* queries,
                       const int64_t* q_offsets_host, int32_t k, int32_t* out_idx, float* out_d2,
                       void* stream);

/* Range check of float32 points (synchronises); PG_ERR_RANGE if any is
 * non-finite or |x| > 1e18. */
pg_status pg_batch_check(const float* points, int64_t n, int32_t d, void* stream);

/* Reads the workspace's flag word (synchronises): bit 0, a wait of the last
 * launch timed out; bit 1, a pg_batch_backward since then met a cloud whose
 * largest term bound (2 max|g| sqrt(max D)) is not a finite float. */
pg_status pg_batch_status(const pg_batch* b, void* stream, int32_t* flags);

/* Times every tuning candidate (leaf 8/16/32 x 2/4 workgroups per CU x 1/4
 * queries per lane x k-list in registers/LDS: 24 launches) on these points
 * and returns the fastest.  Results are cached per (device, cloud-count
 * bucket, point-count bucket, d, k) -- buckets are powers of two -- for the
 * life of the process, and, when the environment variable PG_TUNE_CACHE
 * names a file, across processes: a key found there is returned without
 * timing, a new choice is appended (one text line per key; unreadable lines
 * are ignored).  Synchronises when it times. */
pg_status pg_batch_autotune(const float* points, const int64_t* offsets_host, int32_t n_clouds,
                            int32_t d, int32_t k, void* stream, pg_tune* best);

/* Releases the handle (and the workspace if the library allocated it). */
void pg_batch_free(pg_batch* b);

/* Backward of L = sum_{i,r} g[i,r] * D[i,r] for the handle's last
 * pg_batch_knn_self (same points, same k; the clouds' trees are still in the
 * workspace), with the neighbour sets held fixed.  Every point is a query and
 * a neighbour, so one gradient receives both roles:
 *   grad_points[j] = sum_r 2 g[j,r] (x_j - x_{idx[j,r]})
 *                  - sum_{(i,r): idx[i,r] = j} 2 g[i,r] (x_i - x_j)
 * Queries are taken in each cloud's leaf order, so most neighbour terms are
 * summed in LDS; all sums are int64 fixed point scaled from the cloud's
 * largest term (about 38 bits per term), hence independent of the order of
 * the adds: deterministic.  Not in the paper (the gradient of its k-NN
 * distances).
 *   idx, d2  : [N][k] device, the forward's outputs (global rows, float32 D)
 *   grad_d2  : [N][k] device float32; a cloud whose term bound is not a
 *              finite float (NaN or infinite entries, or terms beyond 3e38)
 *              receives NaN gradients and sets bit 1 of pg_batch_status
 *   grad_points : [N][d] device float32, written (not accumulated)
 * Allocates scratch (stream-ordered pool); does not synchronise. */
pg_status pg_batch_backward(pg_batch* b, const float* points, int32_t k, const int32_t* idx,
                            const float* d2, const float* grad_d2, float* grad_points,
                            void* stream);

/* Backward of L = sum_{i,r} g[i,r] * D(q_i, x_{idx[i,r]}) with the neighbour
 * sets held fixed (the forward's idx):
 *   grad_q[i] = sum_r 2 g[i,r] (q_i - x_j)
 *   grad_p[j] = - sum_{(i,r): idx[i,r] = j} 2 g[i,r] (q_i - x_j)
 * Deterministic: each point's contributions are added in ascending (i, r)
 * order.  idx entries < 0 (padding) are skipped.
 *   queries [m][d], points [n][d], idx [m][k] int32 rows of points,
 *   grad_d2 [m][k] float32; grad_q [m][d] and grad_p [n][d] are overwritten;
 *   grad_q == grad_p is allowed when queries == points (m == n): the array
 *   then receives the sum of both roles. */
pg_status pg_knn_backward(const float* queries, const float* points, int64_t m, int64_t n,
                          int32_t d, int32_t k, const int32_t* idx, const float* grad_d2,
                          float* grad_q, float* grad_p, void* stream);

/* The same gradients with float atomics for grad_p (each pair subtracts its
 * term in whatever order the hardware takes them: not bit-reproducible, the
 * sums differ by rounding only).  Arguments, aliasing and errors as
 * pg_knn_backward; grad_q is the same deterministic per-query sum.  On the
 * 4,096-cloud workload it is slower than both deterministic kernels (random
 * float atomics bound it); it is kept as the plain reference form. */
pg_status pg_knn_backward_atomic(const float* queries, const float* points, int64_t m, int64_t n,
                               int32_t d, int32_t k, const int32_t* idx, const float* grad_d2,
                               float* grad_q, float* grad_p, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PARGEO_HIP_H */
