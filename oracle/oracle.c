/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, serial (the brute-force search may split its queries over
 * threads, which changes no result), obviously-correct implementation of what
 * the GPU path computes.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or table with the
 * GPU library.
 *
 * Coordinates come in one of two types:
 *   dt = 0 : int32 coordinates; squared distances are exact in int64;
 *   dt = 1 : float32 coordinates; squared distances in FP64, summed over
 *            dimensions 0..d-1 in order.
 *
 * Definition of the k-NN result used throughout (the paper leaves the order of
 * equal distances open; the reading adopted is the lexicographic order on
 * (squared distance, id), smaller id first): for a query q over the point set
 * {(p_j, id_j)}, the result is the k smallest keys (D(q,p_j), id_j) in
 * ascending order; when fewer than k points exist, the remaining slots hold
 * id -1 and distance INT64_MAX (int) or +inf (float).
 *
 * Parts:
 *   or_knn_brute   -- the definition written out (all pairs).
 *   or_kd_build    -- static kd-tree by object-median splits (Section 5;
 *                     Appendix C "Parallel vEB Construction", Algorithm 1 and
 *                     the proof of its work bound), with the readings: split
 *                     dimension = level mod d, split rank floor((2j+1)n/2^(l+1))
 *                     under the key (coordinate, index), all leaves at depth
 *                     L = min{L : ceil(n/2^L) <= leaf}.
 *   or_kd_knn      -- the single-query search of Appendix C "Data-Parallel
 *                     k-NN" (descend to the leaf, fill from siblings while
 *                     fewer than k candidates, then contained / disjoint /
 *                     intersecting subtree boxes), run for every query, with
 *                     the 2k candidate buffer the same passage describes.
 *                     Counts visited internal nodes, leaves and points.
 *   or_range_brute -- the orthogonal range query (Section 2, first module;
 *                     Table 1) written out: every point inside a closed box.
 *   or_kd_range    -- the same query on the tree (whole subtrees inside the
 *                     box are reported, subtrees outside it skipped).
 *   or_sp_build    -- the tree by spatial-median splits (cell halving, or
 *                     halving of each node's point box), split until a node
 *                     holds at most `leaf` points, with the readings stated
 *                     at its definition.
 *   or_wspd        -- the well-separated pair decomposition generated from the
 *                     kd-tree (Section 2, second module), by the recursive
 *                     pairing of Callahan and Kosaraju, with the readings
 *                     stated at its definition.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

#define OR_DT_INT 0
#define OR_DT_F32 1

/* ------------------------------------------------------------------------ */
/* Keys: (squared distance, id), compared lexicographically.                 */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t di; double df; int64_t id; } or_key;

static int key_less(const or_key* a, const or_key* b, int dt) {
    if (dt == OR_DT_INT) {
        if (a->di != b->di) return a->di < b->di;
    } else {
        if (a->df != b->df) return a->df < b->df;
    }
    return a->id < b->id;
}

static int key_cmp_int(const void* x, const void* y) {
    const or_key* a = (const or_key*)x; const or_key* b = (const or_key*)y;
    if (a->di != b->di) return a->di < b->di ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}
static int key_cmp_f(const void* x, const void* y) {
    const or_key* a = (const or_key*)x; const or_key* b = (const or_key*)y;
    if (a->df != b->df) return a->df < b->df ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Squared Euclidean distance between query row q and point row p. */
static or_key dist_key(const void* pts, int64_t j, const void* qs, int64_t i,
                       int d, int dt, int64_t id) {
    or_key k; k.di = 0; k.df = 0.0; k.id = id;
    if (dt == OR_DT_INT) {
        const int32_t* P = (const int32_t*)pts; const int32_t* Q = (const int32_t*)qs;
        for (int c = 0; c < d; c++) {
            int64_t diff = (int64_t)Q[i * d + c] - (int64_t)P[j * d + c];
            k.di += diff * diff;
        }
    } else {
        const float* P = (const float*)pts; const float* Q = (const float*)qs;
        for (int c = 0; c < d; c++) {
            double diff = (double)Q[i * d + c] - (double)P[j * d + c];
            k.df += diff * diff;
        }
    }
    return k;
}

static void write_result(const or_key* best, int cnt, int k, int dt,
                         int64_t* out_id, void* out_dist, int64_t row) {
    for (int r = 0; r < k; r++) {
        if (r < cnt) {
            out_id[row * k + r] = best[r].id;
            if (dt == OR_DT_INT) ((int64_t*)out_dist)[row * k + r] = best[r].di;
            else ((double*)out_dist)[row * k + r] = best[r].df;
        } else {
            out_id[row * k + r] = -1;
            if (dt == OR_DT_INT) ((int64_t*)out_dist)[row * k + r] = INT64_MAX;
            else ((double*)out_dist)[row * k + r] = INFINITY;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* O1: brute force -- the definition.  For each query every point's key is  */
/* offered to a sorted list of the k smallest keys seen so far.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    const void* pts; const int64_t* ids; const uint8_t* alive; int64_t n; int d, dt;
    const void* qs; int64_t q0, q1; int k; int64_t* out_id; void* out_dist;
} brute_job;

static void* brute_worker(void* arg) {
    brute_job* J = (brute_job*)arg;
    or_key* best = (or_key*)malloc(sizeof(or_key) * (size_t)(J->k > 0 ? J->k : 1));
    for (int64_t i = J->q0; i < J->q1; i++) {
        int cnt = 0;
        for (int64_t j = 0; j < J->n; j++) {
            if (J->alive && !J->alive[j]) continue;
            or_key key = dist_key(J->pts, j, J->qs, i, J->d, J->dt, J->ids ? J->ids[j] : j);
            if (cnt == J->k && !key_less(&key, &best[J->k - 1], J->dt)) continue;
            int pos = cnt < J->k ? cnt++ : J->k - 1;
            while (pos > 0 && key_less(&key, &best[pos - 1], J->dt)) { best[pos] = best[pos - 1]; pos--; }
            best[pos] = key;
        }
        write_result(best, cnt, J->k, J->dt, J->out_id, J->out_dist, i);
    }
    free(best);
    return NULL;
}

/* pts [n][d], ids [n] (NULL: id = row index), alive [n] (NULL: all alive),
 * qs [m][d]; out_id [m][k]; out_dist [m][k] int64 (dt 0) or double (dt 1). */
int or_knn_brute(const void* pts, const int64_t* ids, const uint8_t* alive, int64_t n,
                 int d, int dt, const void* qs, int64_t m, int k,
                 int64_t* out_id, void* out_dist, int nthreads) {
    if (d < 1 || k < 1 || n < 0 || m < 0) return 1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (m < nthreads) nthreads = m > 0 ? (int)m : 1;
    brute_job jobs[256]; pthread_t th[256];
    for (int t = 0; t < nthreads; t++) {
        brute_job J = {pts, ids, alive, n, d, dt, qs, m * t / nthreads, m * (t + 1) / nthreads, k, out_id, out_dist};
        jobs[t] = J;
    }
    if (nthreads == 1) { brute_worker(&jobs[0]); return 0; }
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, brute_worker, &jobs[t]);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2: static kd-tree, object-median splits.                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n; int d, dt, L;
    const void* pts;          /* caller's [n][d] array, kept by reference     */
    int64_t* perm;            /* [n] point rows in leaf order                 */
    double* split;            /* [2^L] heap 1-based, split value of node h    */
    double* bmin; double* bmax; /* [2^(L+1)][d] tight box of node h's points  */
} or_tree;

static double coord(const or_tree* T, int64_t row, int c) {
    if (T->dt == OR_DT_INT) return (double)((const int32_t*)T->pts)[row * T->d + c];
    return (double)((const float*)T->pts)[row * T->d + c];
}

/* Node (level l, j) covers positions [floor(j n / 2^l), floor((j+1) n / 2^l)). */
static int64_t node_lo(int64_t n, int l, int64_t j) { return (int64_t)(((__int128)j * n) >> l); }

/* Key of a point for the split along dimension c: (coordinate, row index). */
static int cut_less(const or_tree* T, int64_t a, int64_t b, int c) {
    double x = coord(T, a, c), y = coord(T, b, c);
    if (x != y) return x < y;
    return a < b;
}

/* Quickselect: rearrange perm[lo,hi) so that position r holds the element of
 * rank r - lo under cut_less, with smaller keys before and larger after.
 * Keys are distinct (the row index breaks ties), so the split set is unique. */
static void select_rank(const or_tree* T, int64_t* perm, int64_t lo, int64_t hi, int64_t r,
                        int c, uint64_t* seed) {
    while (hi - lo > 1) {
        *seed = *seed * 6364136223846793005ULL + 1442695040888963407ULL;
        int64_t piv = perm[lo + (int64_t)((*seed >> 33) % (uint64_t)(hi - lo))];
        /* three-way partition around piv: [lo,a) less, [a,b) == piv, [b,hi) greater */
        int64_t a = lo, b = lo, e = hi;
        while (b < e) {
            int64_t x = perm[b];
            if (x == piv) { b++; }
            else if (cut_less(T, x, piv, c)) { int64_t t = perm[a]; perm[a] = x; perm[b] = t; a++; b++; }
            else { e--; int64_t t = perm[e]; perm[e] = x; perm[b] = t; }
        }
        if (r < a) hi = a;
        else if (r >= b) lo = b;
        else return;
    }
}

static void build_rec(or_tree* T, int l, int64_t j, uint64_t* seed) {
    if (l == T->L) return;
    int64_t lo = node_lo(T->n, l, j), hi = node_lo(T->n, l, j + 1);
    int64_t mid = node_lo(T->n, l + 1, 2 * j + 1);
    int c = l % T->d;
    /* The split value is the key of the first right element; when the right
     * child is empty (only possible for leaf size 1) it is the largest left
     * key.  Internal nodes are never empty. */
    int64_t at = mid < hi ? mid : hi - 1;
    select_rank(T, T->perm, lo, hi, at, c, seed);
    int64_t h = ((int64_t)1 << l) + j;
    T->split[h] = coord(T, T->perm[at], c);
    build_rec(T, l + 1, 2 * j, seed);
    build_rec(T, l + 1, 2 * j + 1, seed);
}

static int tree_depth(int64_t n, int leaf) {
    int L = 0;
    while (((n + ((int64_t)1 << L) - 1) >> L) > leaf) L++;
    return L;
}

void or_kd_free(or_tree* T) {
    if (!T) return;
    free(T->perm); free(T->split); free(T->bmin); free(T->bmax); free(T);
}

or_tree* or_kd_build(const void* pts, int64_t n, int d, int dt, int leaf) {
    if (d < 1 || leaf < 1 || n < 0) return NULL;
    or_tree* T = (or_tree*)calloc(1, sizeof(or_tree));
    T->n = n; T->d = d; T->dt = dt; T->pts = pts;
    T->L = tree_depth(n, leaf);
    int64_t nn = (int64_t)1 << (T->L + 1);
    T->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    T->split = (double*)calloc((size_t)(nn / 2 + 1), sizeof(double));
    T->bmin = (double*)malloc(sizeof(double) * (size_t)(nn * d));
    T->bmax = (double*)malloc(sizeof(double) * (size_t)(nn * d));
    for (int64_t i = 0; i < n; i++) T->perm[i] = i;
    uint64_t seed = 0x9E3779B97F4A7C15ULL;
    build_rec(T, 0, 0, &seed);
    /* Tight boxes: leaves from their points, internal nodes from children. */
    int64_t first_leaf = (int64_t)1 << T->L;
    for (int64_t h = first_leaf; h < nn; h++) {
        int64_t j = h - first_leaf;
        int64_t lo = node_lo(n, T->L, j), hi = node_lo(n, T->L, j + 1);
        for (int c = 0; c < d; c++) { T->bmin[h * d + c] = INFINITY; T->bmax[h * d + c] = -INFINITY; }
        for (int64_t i = lo; i < hi; i++)
            for (int c = 0; c < d; c++) {
                double v = coord(T, T->perm[i], c);
                if (v < T->bmin[h * d + c]) T->bmin[h * d + c] = v;
                if (v > T->bmax[h * d + c]) T->bmax[h * d + c] = v;
            }
    }
    for (int64_t h = first_leaf - 1; h >= 1; h--)
        for (int c = 0; c < d; c++) {
            double a = T->bmin[2 * h * d + c], b = T->bmin[(2 * h + 1) * d + c];
            T->bmin[h * d + c] = a < b ? a : b;
            a = T->bmax[2 * h * d + c]; b = T->bmax[(2 * h + 1) * d + c];
            T->bmax[h * d + c] = a > b ? a : b;
        }
    return T;
}

int or_kd_levels(const or_tree* T) { return T->L; }

/* Copies the split values (heap index 1..2^L-1, as double) and the leaf-order
 * point rows out of the tree. */
void or_kd_export(const or_tree* T, double* split_out, int64_t* perm_out) {
    int64_t ni = ((int64_t)1 << T->L);
    for (int64_t h = 1; h < ni; h++) split_out[h - 1] = T->split[h];
    for (int64_t i = 0; i < T->n; i++) perm_out[i] = T->perm[i];
}

/* ------------------------------------------------------------------------ */
/* O3: kd-tree k-NN (Appendix C, "Data-Parallel k-NN").                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    or_key* buf; int cnt, k;  /* 2k candidate buffer */
    int dt;
} knn_buffer;

static int cmp_dt_int(const void* a, const void* b) { return key_cmp_int(a, b); }
static int cmp_dt_f(const void* a, const void* b) { return key_cmp_f(a, b); }

/* Keep the k smallest candidates (selection by sorting the buffer). */
static void buffer_trim(knn_buffer* B) {
    qsort(B->buf, (size_t)B->cnt, sizeof(or_key), B->dt == OR_DT_INT ? cmp_dt_int : cmp_dt_f);
    if (B->cnt > B->k) B->cnt = B->k;
}

static void buffer_add(knn_buffer* B, or_key key) {
    B->buf[B->cnt++] = key;
    if (B->cnt == 2 * B->k) buffer_trim(B);
}

/* The current k-th smallest key (only meaningful when cnt >= k). */
static or_key buffer_kth(knn_buffer* B) {
    buffer_trim(B);
    return B->buf[B->k - 1];
}

typedef struct {
    const or_tree* T; const void* qs; int64_t qi; const int64_t* ids; const uint8_t* alive;
    knn_buffer* B;
    int64_t n_internal, n_leaves, n_points;
} knn_ctx;

static double qcoord(const knn_ctx* C, int c) {
    if (C->T->dt == OR_DT_INT) return (double)((const int32_t*)C->qs)[C->qi * C->T->d + c];
    return (double)((const float*)C->qs)[C->qi * C->T->d + c];
}

static void add_point(knn_ctx* C, int64_t row) {
    if (C->alive && !C->alive[row]) return;
    C->n_points++;
    buffer_add(C->B, dist_key(C->T->pts, row, C->qs, C->qi, C->T->d, C->T->dt,
                              C->ids ? C->ids[row] : row));
}

static void add_subtree(knn_ctx* C, int l, int64_t j) {
    /* every leaf under (l, j) */
    int L = C->T->L;
    int64_t j0 = j << (L - l), j1 = (j + 1) << (L - l);
    int64_t lo = node_lo(C->T->n, L, j0), hi = node_lo(C->T->n, L, j1);
    C->n_leaves += j1 - j0;
    for (int64_t i = lo; i < hi; i++) add_point(C, C->T->perm[i]);
}

/* Smallest and largest squared distance from the query to the box of node h.
 * Integer coordinates: exact in int64.  Float coordinates: the same FP64
 * operations, in the same order, as dist_key, so that (rounding being
 * monotone) lo <= D(q,p) <= hi holds for the computed distance of every
 * point p in the box. */
static void box_bounds(const knn_ctx* C, int64_t h, or_key* lo_key, or_key* hi_key) {
    const or_tree* T = C->T; int d = T->d;
    int64_t loi = 0, hii = 0; double lof = 0.0, hif = 0.0;
    if (T->bmin[h * d] > T->bmax[h * d]) {
        /* a node without points (its box is [+inf, -inf]): beyond every
         * distance, so it is never entered or added */
        lo_key->di = INT64_MAX; lo_key->df = INFINITY; lo_key->id = INT64_MAX;
        hi_key->di = INT64_MAX; hi_key->df = INFINITY; hi_key->id = INT64_MAX;
        return;
    }
    for (int c = 0; c < d; c++) {
        double q = qcoord(C, c), a = T->bmin[h * d + c], b = T->bmax[h * d + c];
        if (T->dt == OR_DT_INT) {
            int64_t qi = (int64_t)q, ai = (int64_t)a, bi = (int64_t)b;
            int64_t gap = qi < ai ? ai - qi : (qi > bi ? qi - bi : 0);
            int64_t far = (qi - ai > bi - qi) ? qi - ai : bi - qi;
            loi += gap * gap; hii += far * far;
        } else {
            double gap = q < a ? a - q : (q > b ? q - b : 0.0);
            double fa = fabs(q - a), fb = fabs(q - b);
            double far = fa > fb ? fa : fb;
            lof += gap * gap; hif += far * far;
        }
    }
    lo_key->di = loi; lo_key->df = lof; lo_key->id = INT64_MIN;
    hi_key->di = hii; hi_key->df = hif; hi_key->id = INT64_MAX;
}

static void knn_rec(knn_ctx* C, int l, int64_t j) {
    const or_tree* T = C->T;
    if (l == T->L) { /* leaf: add all of its points */
        C->n_leaves++;
        int64_t lo = node_lo(T->n, l, j), hi = node_lo(T->n, l, j + 1);
        for (int64_t i = lo; i < hi; i++) add_point(C, T->perm[i]);
        return;
    }
    C->n_internal++;
    int64_t h = ((int64_t)1 << l) + j;
    int c = l % T->d;
    int64_t near_j = qcoord(C, c) < T->split[h] ? 2 * j : 2 * j + 1;
    int64_t far_j = near_j ^ 1;
    knn_rec(C, l + 1, near_j);
    /* unwinding: the sibling subtree (l+1, far_j) */
    if (C->B->cnt < C->B->k) { add_subtree(C, l + 1, far_j); return; }
    or_key kth = buffer_kth(C->B), lo, hi;
    int64_t hf = ((int64_t)1 << (l + 1)) + far_j;
    box_bounds(C, hf, &lo, &hi);
    int contained = T->dt == OR_DT_INT ? hi.di <= kth.di : hi.df <= kth.df;
    int disjoint = T->dt == OR_DT_INT ? lo.di > kth.di : lo.df > kth.df;
    if (contained) add_subtree(C, l + 1, far_j);
    else if (!disjoint) knn_rec(C, l + 1, far_j);
}

/* k-NN of every query row over the tree.  ids/alive as in or_knn_brute.
 * counters (may be NULL): [0] internal nodes, [1] leaves, [2] points, summed. */
int or_kd_knn(const or_tree* T, const int64_t* ids, const uint8_t* alive,
              const void* qs, int64_t m, int k,
              int64_t* out_id, void* out_dist, int64_t* counters) {
    if (!T || k < 1 || m < 0) return 1;
    knn_buffer B; B.k = k; B.dt = T->dt; B.buf = (or_key*)malloc(sizeof(or_key) * (size_t)(2 * k));
    int64_t ci = 0, cl = 0, cp = 0;
    for (int64_t i = 0; i < m; i++) {
        B.cnt = 0;
        knn_ctx C = {T, qs, i, ids, alive, &B, 0, 0, 0};
        if (T->n > 0) knn_rec(&C, 0, 0);
        buffer_trim(&B);
        write_result(B.buf, B.cnt, k, T->dt, out_id, out_dist, i);
        ci += C.n_internal; cl += C.n_leaves; cp += C.n_points;
    }
    free(B.buf);
    if (counters) { counters[0] = ci; counters[1] = cl; counters[2] = cp; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O7: orthogonal range search (the kd-tree range query of Section 2's      */
/* first module and of Table 1).  The paper does not spell the query out;   */
/* the reading used: a query is a closed axis-aligned box [lo, hi], and its */
/* result is every (live) point p with lo_c <= p_c <= hi_c for all c.  A box */
/* with lo_c > hi_c in some dimension is empty.  Coordinates are compared as */
/* values (float32 widened to double, so -0.0 equals +0.0).                 */
/* ------------------------------------------------------------------------ */
static int in_box(const void* pts, int64_t j, const void* boxes, int64_t i, int d, int dt) {
    for (int c = 0; c < d; c++) {
        double p, lo, hi;
        if (dt == OR_DT_INT) {
            const int32_t* P = (const int32_t*)pts; const int32_t* B = (const int32_t*)boxes;
            p = P[j * d + c]; lo = B[i * 2 * d + c]; hi = B[i * 2 * d + d + c];
        } else {
            const float* P = (const float*)pts; const float* B = (const float*)boxes;
            p = P[j * d + c]; lo = B[i * 2 * d + c]; hi = B[i * 2 * d + d + c];
        }
        if (!(lo <= p && p <= hi)) return 0;
    }
    return 1;
}

/* The definition written out.  boxes [m][2][d] (lo[d] then hi[d]).
 * counts [m] receives each box's number of live points.  When offsets is not
 * NULL (offsets[i] = first output slot of box i), out_id also receives the
 * ids of those points in row order (ids NULL: id = row). */
int or_range_brute(const void* pts, const int64_t* ids, const uint8_t* alive, int64_t n,
                   int d, int dt, const void* boxes, int64_t m,
                   int64_t* counts, const int64_t* offsets, int64_t* out_id) {
    if (d < 1 || n < 0 || m < 0 || !counts) return 1;
    for (int64_t i = 0; i < m; i++) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++) {
            if (alive && !alive[j]) continue;
            if (!in_box(pts, j, boxes, i, d, dt)) continue;
            if (offsets) out_id[offsets[i] + c] = ids ? ids[j] : j;
            c++;
        }
        counts[i] = c;
    }
    return 0;
}

/* Range search on the oracle's kd-tree: a node whose box lies inside the
 * query reports all its points, a node whose box misses the query is
 * skipped, otherwise its children are searched (leaves test every point).
 * Counts the nodes whose box was tested and the points tested one by one. */
typedef struct {
    const or_tree* T; const void* boxes; int64_t i; const int64_t* ids; const uint8_t* alive;
    int64_t c; const int64_t* offsets; int64_t* out_id; int64_t n_nodes, n_points;
} range_ctx;

static void range_emit(range_ctx* C, int64_t row) {
    if (C->alive && !C->alive[row]) return;
    if (C->offsets) C->out_id[C->offsets[C->i] + C->c] = C->ids ? C->ids[row] : row;
    C->c++;
}

static void range_rec(range_ctx* C, int l, int64_t j) {
    const or_tree* T = C->T;
    const int d = T->d;
    const int64_t h = ((int64_t)1 << l) + j;
    const int64_t lo = node_lo(T->n, l, j), hi = node_lo(T->n, l, j + 1);
    if (lo == hi) return;
    C->n_nodes++;
    int inside = 1, miss = 0;
    for (int c = 0; c < d; c++) {
        double qlo, qhi;
        if (T->dt == OR_DT_INT) {
            const int32_t* B = (const int32_t*)C->boxes;
            qlo = B[C->i * 2 * d + c]; qhi = B[C->i * 2 * d + d + c];
        } else {
            const float* B = (const float*)C->boxes;
            qlo = B[C->i * 2 * d + c]; qhi = B[C->i * 2 * d + d + c];
        }
        const double bl = T->bmin[h * d + c], bh = T->bmax[h * d + c];
        if (bh < qlo || bl > qhi) miss = 1;
        if (bl < qlo || bh > qhi) inside = 0;
    }
    if (miss) return;
    if (inside || l == T->L) {
        for (int64_t p = lo; p < hi; p++) {
            if (!inside) {
                C->n_points++;
                if (!in_box(T->pts, T->perm[p], C->boxes, C->i, d, T->dt)) continue;
            }
            range_emit(C, T->perm[p]);
        }
        return;
    }
    range_rec(C, l + 1, 2 * j);
    range_rec(C, l + 1, 2 * j + 1);
}

/* Arguments as or_range_brute (ids of a box come in leaf order here).
 * counters (may be NULL): [0] node boxes tested, [1] points tested. */
int or_kd_range(const or_tree* T, const int64_t* ids, const uint8_t* alive,
                const void* boxes, int64_t m, int64_t* counts, const int64_t* offsets,
                int64_t* out_id, int64_t* counters) {
    if (!T || m < 0 || !counts) return 1;
    int64_t cn = 0, cp = 0;
    for (int64_t i = 0; i < m; i++) {
        range_ctx C = {T, boxes, i, ids, alive, 0, offsets, out_id, 0, 0};
        if (T->n > 0) range_rec(&C, 0, 0);
        counts[i] = C.c;
        cn += C.n_nodes; cp += C.n_points;
    }
    if (counters) { counters[0] = cn; counters[1] = cp; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O8: kd-tree by spatial-median splits (Section 6.3 compares them with the */
/* object-median splits: a node's space is cut in half along a dimension;   */
/* Section 5 defines the kd-tree as splitting until a node holds a small    */
/* constant number of points).  Readings:                                   */
/*  - a node is a leaf when it holds at most `leaf` points, or when all of   */
/*    its points are identical (no cut can separate them);                  */
/*  - the space of the root is the bounding box of the points; a node cuts  */
/*    its cell (rule bit 1 clear) or the bounding box of its own points     */
/*    (rule bit 1 set);                                                     */
/*  - the cut dimension is depth mod d (rule bit 0 clear) or the space's    */
/*    widest side hi - lo, the lowest dimension on ties (bit 0 set);        */
/*  - spaces are closed intervals [lo, hi] of representable coordinates,    */
/*    and the cut s of [lo, hi] with lo < hi lies in (lo, hi]: int32        */
/*    floor((lo + hi + 1) / 2); float32 the float nearest (lo + hi) / 2     */
/*    (sum and halving in double), or the next float above lo when that     */
/*    nearest float is lo itself.  When lo == hi, s = lo;                   */
/*  - points with coordinate < s go left (to the cell [lo, s'] with s' the  */
/*    value just below s), the others right (cell [s, hi]), each side in    */
/*    the parent's order (a stable partition).                              */
/* Both children of a cut always shrink the cut side, so every path ends.   */
/* Nodes are numbered breadth-first: the root is 0, a level's nodes come in */
/* leaf order, and an internal node's children are consecutive.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n; int d, dt, leaf, rule, depth;
    const void* pts;
    int64_t count, cap;  /* nodes */
    double* split; int32_t* dim; int64_t* child; int64_t* lo; int64_t* hi; int32_t* level;
    double* clo; double* chi;  /* cell of each node, [cap][d] */
    int64_t* perm;             /* rows in leaf order */
} or_sp_tree;

static double sp_coord(const or_sp_tree* T, int64_t row, int c) {
    return T->dt == OR_DT_INT ? (double)((const int32_t*)T->pts)[row * T->d + c]
                              : (double)((const float*)T->pts)[row * T->d + c];
}

/* The cut of [lo, hi] (see the readings above). */
static double sp_cut(double lo, double hi, int dt) {
    if (!(lo < hi)) return lo;
    if (dt == OR_DT_INT) {
        int64_t t = (int64_t)lo + (int64_t)hi + 1;
        return (double)(t >= 0 ? t / 2 : -((-t + 1) / 2));
    }
    float s = (float)(0.5 * (lo + hi));
    if ((double)s <= lo) s = nextafterf((float)lo, INFINITY);
    return (double)s;
}

/* The largest coordinate below s. */
static double sp_below(double s, int dt) {
    return dt == OR_DT_INT ? s - 1.0 : (double)nextafterf((float)s, -INFINITY);
}

static int sp_grow(or_sp_tree* T, int64_t need) {
    if (need <= T->cap) return 0;
    int64_t cap = T->cap ? T->cap : 64;
    while (cap < need) cap *= 2;
    T->split = (double*)realloc(T->split, sizeof(double) * (size_t)cap);
    T->dim = (int32_t*)realloc(T->dim, sizeof(int32_t) * (size_t)cap);
    T->child = (int64_t*)realloc(T->child, sizeof(int64_t) * (size_t)cap);
    T->lo = (int64_t*)realloc(T->lo, sizeof(int64_t) * (size_t)cap);
    T->hi = (int64_t*)realloc(T->hi, sizeof(int64_t) * (size_t)cap);
    T->level = (int32_t*)realloc(T->level, sizeof(int32_t) * (size_t)cap);
    T->clo = (double*)realloc(T->clo, sizeof(double) * (size_t)(cap * T->d));
    T->chi = (double*)realloc(T->chi, sizeof(double) * (size_t)(cap * T->d));
    if (!T->split || !T->dim || !T->child || !T->lo || !T->hi || !T->level || !T->clo || !T->chi)
        return 1;
    T->cap = cap;
    return 0;
}

void or_sp_free(or_sp_tree* T) {
    if (!T) return;
    free(T->split); free(T->dim); free(T->child); free(T->lo); free(T->hi); free(T->level);
    free(T->clo); free(T->chi); free(T->perm); free(T);
}

or_sp_tree* or_sp_build(const void* pts, int64_t n, int d, int dt, int leaf, int rule) {
    if (d < 1 || d > 8 || leaf < 1 || n < 0 || rule < 0 || rule > 3) return NULL;
    or_sp_tree* T = (or_sp_tree*)calloc(1, sizeof(or_sp_tree));
    T->n = n; T->d = d; T->dt = dt; T->leaf = leaf; T->rule = rule; T->pts = pts;
    T->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!T->perm || !tmp || sp_grow(T, 1)) { free(tmp); or_sp_free(T); return NULL; }
    for (int64_t i = 0; i < n; i++) T->perm[i] = i;
    /* the root: every point, the points' bounding box as its cell */
    T->count = 1;
    T->lo[0] = 0; T->hi[0] = n; T->level[0] = 0;
    for (int c = 0; c < d; c++) { T->clo[c] = INFINITY; T->chi[c] = -INFINITY; }
    for (int64_t i = 0; i < n; i++)
        for (int c = 0; c < d; c++) {
            double x = sp_coord(T, i, c);
            if (x < T->clo[c]) T->clo[c] = x;
            if (x > T->chi[c]) T->chi[c] = x;
        }
    /* breadth-first: node u's children are appended when u is cut */
    for (int64_t u = 0; u < T->count; u++) {
        const int64_t lo = T->lo[u], hi = T->hi[u];
        T->split[u] = 0.0; T->dim[u] = -1; T->child[u] = -1;
        if (T->level[u] + 1 > T->depth) T->depth = T->level[u] + 1;
        if (hi - lo <= leaf) continue;
        double blo[8], bhi[8];
        for (int c = 0; c < d; c++) { blo[c] = INFINITY; bhi[c] = -INFINITY; }
        for (int64_t p = lo; p < hi; p++)
            for (int c = 0; c < d; c++) {
                double x = sp_coord(T, T->perm[p], c);
                if (x < blo[c]) blo[c] = x;
                if (x > bhi[c]) bhi[c] = x;
            }
        int same = 1;
        for (int c = 0; c < d; c++) if (blo[c] != bhi[c]) same = 0;
        if (same) continue;  /* identical points: a leaf */
        const double* slo = (rule & 2) ? blo : T->clo + u * d;
        const double* shi = (rule & 2) ? bhi : T->chi + u * d;
        int c = T->level[u] % d;
        if (rule & 1) {
            c = 0;
            for (int e = 1; e < d; e++)
                if (shi[e] - slo[e] > shi[c] - slo[c]) c = e;
        }
        const double s = sp_cut(slo[c], shi[c], dt);
        /* stable partition of perm[lo, hi) by coordinate < s */
        int64_t w = lo, nr = 0;
        for (int64_t p = lo; p < hi; p++) {
            int64_t row = T->perm[p];
            if (sp_coord(T, row, c) < s) T->perm[w++] = row;
            else tmp[nr++] = row;
        }
        for (int64_t t = 0; t < nr; t++) T->perm[w + t] = tmp[t];
        if (sp_grow(T, T->count + 2)) { free(tmp); or_sp_free(T); return NULL; }
        const int64_t a = T->count, b = a + 1;
        T->count += 2;
        T->split[u] = s; T->dim[u] = c; T->child[u] = a;
        T->lo[a] = lo; T->hi[a] = w; T->lo[b] = w; T->hi[b] = hi;
        T->level[a] = T->level[b] = T->level[u] + 1;
        for (int e = 0; e < d; e++) {
            T->clo[a * d + e] = T->clo[b * d + e] = T->clo[u * d + e];
            T->chi[a * d + e] = T->chi[b * d + e] = T->chi[u * d + e];
        }
        /* the children's cells: the cut side of the node's cell (in the
         * point-box form the cells are carried along but unused) */
        T->chi[a * d + c] = sp_below(s, dt);
        T->clo[b * d + c] = s;
    }
    free(tmp);
    return T;
}

int64_t or_sp_nodes(const or_sp_tree* T) { return T->count; }
int or_sp_depth(const or_sp_tree* T) { return T->depth; }

/* Copies the tree out: per node (count entries) split value (0 for
 * leaves), split dimension (-1 for leaves), first child (-1 for leaves; the
 * second child follows it), leaf-order range [lo, hi), depth; rows in leaf
 * order (n entries).  Any output may be NULL. */
void or_sp_export(const or_sp_tree* T, double* split, int32_t* dim, int64_t* child, int64_t* lo,
                  int64_t* hi, int32_t* level, int64_t* perm) {
    size_t c = (size_t)T->count;
    if (split) memcpy(split, T->split, sizeof(double) * c);
    if (dim) memcpy(dim, T->dim, sizeof(int32_t) * c);
    if (child) memcpy(child, T->child, sizeof(int64_t) * c);
    if (lo) memcpy(lo, T->lo, sizeof(int64_t) * c);
    if (hi) memcpy(hi, T->hi, sizeof(int64_t) * c);
    if (level) memcpy(level, T->level, sizeof(int32_t) * c);
    if (perm && T->n > 0) memcpy(perm, T->perm, sizeof(int64_t) * (size_t)T->n);
}

/* ------------------------------------------------------------------------ */
/* O9: well-separated pair decomposition (WSPD) from the kd-tree (Section 2, */
/* second module, after Callahan and Kosaraju).  Readings:                  */
/*  - the tree is the object-median tree with leaf size 1, so every leaf     */
/*    holds at most one point and the pairs cover every pair of distinct   */
/*    points exactly once;                                                  */
/*  - a node's ball is centred at the centre of its bounding box, with the  */
/*    half diagonal as radius; nodes a and b are well separated for s when  */
/*    the distance of the centres is at least (s + 2) r, r the larger of    */
/*    the two radii (balls of radius r around each set, at least s r        */
/*    apart), tested on squares: |c_a - c_b|^2 >= (s + 2)^2 r^2, every      */
/*    quantity in double: half side (hi - lo) * 0.5, centre (lo + hi) * 0.5,*/
/*    sums over dimensions 0..d-1 in order;                                 */
/*  - a pair that is not separated is refined by splitting the node with    */
/*    the larger radius (the first on ties; never a leaf), and pairs with  */
/*    an empty node are dropped;                                            */
/*  - every internal node pairs its two children, then both children are  */
/*    processed the same way.                                               */
/* Output: pairs (a, b) of heap node indices, a from the first child's side.*/
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_tree* T; double s2; int64_t cnt, cap; int64_t* out;
} wspd_ctx;

static int64_t node_points(const or_tree* T, int64_t h) {
    int l = 63 - __builtin_clzll((unsigned long long)h);
    int64_t j = h - ((int64_t)1 << l);
    return node_lo(T->n, l, j + 1) - node_lo(T->n, l, j);
}

static double half_diag2(const or_tree* T, int64_t h) {
    double r2 = 0.0;
    for (int c = 0; c < T->d; c++) {
        double t = (T->bmax[h * T->d + c] - T->bmin[h * T->d + c]) * 0.5;
        r2 += t * t;
    }
    return r2;
}

static double centre_gap2(const or_tree* T, int64_t a, int64_t b) {
    double g2 = 0.0;
    for (int c = 0; c < T->d; c++) {
        double ca = (T->bmin[a * T->d + c] + T->bmax[a * T->d + c]) * 0.5;
        double cb = (T->bmin[b * T->d + c] + T->bmax[b * T->d + c]) * 0.5;
        double t = ca - cb;
        g2 += t * t;
    }
    return g2;
}

static void wspd_pair(wspd_ctx* C, int64_t a, int64_t b) {
    const or_tree* T = C->T;
    if (node_points(T, a) == 0 || node_points(T, b) == 0) return;
    double ra = half_diag2(T, a), rb = half_diag2(T, b);
    double r2 = ra > rb ? ra : rb;
    if (centre_gap2(T, a, b) >= C->s2 * r2) {
        if (C->out && C->cnt < C->cap) {
            C->out[2 * C->cnt] = a;
            C->out[2 * C->cnt + 1] = b;
        }
        C->cnt++;
        return;
    }
    int64_t first_leaf = (int64_t)1 << T->L;
    int split_a = (ra >= rb && a < first_leaf) || b >= first_leaf;
    if (split_a) {
        wspd_pair(C, 2 * a, b);
        wspd_pair(C, 2 * a + 1, b);
    } else {
        wspd_pair(C, a, 2 * b);
        wspd_pair(C, a, 2 * b + 1);
    }
}

static void wspd_node(wspd_ctx* C, int64_t h) {
    if (h >= ((int64_t)1 << C->T->L)) return;
    wspd_pair(C, 2 * h, 2 * h + 1);
    wspd_node(C, 2 * h);
    wspd_node(C, 2 * h + 1);
}

/* Returns the number of pairs (writing at most cap of them to out[cap][2]);
 * -1 for bad arguments (s not positive and finite, or leaf size above 1). */
int64_t or_wspd(const or_tree* T, double s, int64_t* out, int64_t cap) {
    if (!(s > 0.0) || !(s < INFINITY)) return -1;
    if ((T->n + ((int64_t)1 << T->L) - 1) >> T->L > 1) return -1;
    wspd_ctx C = {T, (s + 2.0) * (s + 2.0), 0, cap, out};
    if (T->L > 0) wspd_node(&C, 1);
    return C.cnt;
}
