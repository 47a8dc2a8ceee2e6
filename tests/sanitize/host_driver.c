/* Exercises the host side of libpargeo_hip (built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on its host code only, by
 * tests/test_sanitizers.py) on a machine without a GPU: argument
 * validation and error reporting of every entry point family, handle
 * lifetimes that need no device work, and the batched launch's workspace
 * planning.  Exits non-zero when a call returns the wrong status; the
 * sanitizers abort on a memory error, undefined behaviour or a leak. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pargeo_hip.h"

static int fails = 0;
#define EXPECT(call, want)                                                           \
    do {                                                                             \
        pg_status got_ = (call);                                                     \
        if (got_ != (want)) {                                                        \
            fprintf(stderr, "%s: status %d, expected %d (%s)\n", #call, (int)got_, \
                    (int)(want), pg_last_error());                                   \
            fails++;                                                                 \
        }                                                                            \
    } while (0)

int main(void) {
    if (!pg_version() || !pg_last_error()) return 2;
    int32_t idx[4];
    int64_t d64[4], n = 0, cnt = 0;
    int32_t d = 0, leaf = 0, lv = 0, dt = 0;
    float q[6] = {0};
    pg_tree* t = NULL;

    /* static tree entry points */
    EXPECT(pg_kdtree_build(NULL, 10, 3, 16, PG_INT32, NULL, &t), PG_ERR_INVALID);
    EXPECT(pg_kdtree_build(q, 2, 0, 16, PG_INT32, NULL, &t), PG_ERR_INVALID);
    EXPECT(pg_kdtree_build(q, 2, 3, 0, PG_INT32, NULL, &t), PG_ERR_INVALID);
    EXPECT(pg_kdtree_build(q, 2, 3, 16, 7, NULL, &t), PG_ERR_INVALID);
    EXPECT(pg_kdtree_build(q, 2, 3, 16, PG_INT32, NULL, NULL), PG_ERR_INVALID);
    EXPECT(pg_kdtree_build_spatial(NULL, 10, 3, 16, PG_INT32, 0, NULL, &t), PG_ERR_INVALID);
    EXPECT(pg_knn(NULL, q, 2, 3, idx, d64, NULL), PG_ERR_INVALID);
    EXPECT(pg_knn_noalloc(NULL, q, 2, 3, idx, d64, NULL), PG_ERR_INVALID);
    EXPECT(pg_knn_all(NULL, 3, idx, d64, NULL), PG_ERR_INVALID);
    EXPECT(pg_knn_graph(NULL, 3, idx, d64, NULL), PG_ERR_INVALID);
    EXPECT(pg_tree_info(NULL, &n, &d, &leaf, &lv, &dt), PG_ERR_INVALID);
    EXPECT(pg_tree_nodes(NULL, &n, &cnt), PG_ERR_INVALID);
    EXPECT(pg_wspd(NULL, 2.0, NULL, 0, &cnt, NULL), PG_ERR_INVALID);
    EXPECT(pg_range_count(NULL, q, 1, idx, NULL, NULL, NULL), PG_ERR_INVALID);
    pg_tree_free(NULL);

    /* BDL-tree and B1: creation and release need no device work */
    pg_bdl* b = NULL;
    EXPECT(pg_bdl_create(0, PG_INT32, 16, 1024, &b), PG_ERR_INVALID);
    EXPECT(pg_bdl_create(3, PG_INT32, 0, 1024, &b), PG_ERR_INVALID);
    EXPECT(pg_bdl_create(3, PG_INT32, 16, 0, &b), PG_ERR_INVALID);
    EXPECT(pg_bdl_create(3, PG_FLOAT32, 16, 1024, &b), PG_OK);
    if (b) {
        if (pg_bdl_size(b) != 0) fails++;
        int64_t mask = -1, buf = -1, live[8];
        EXPECT(pg_bdl_stats(b, &mask, &buf, live, 8), PG_OK);
        if (mask != 0 || buf != 0) fails++;
        EXPECT(pg_bdl_insert(b, NULL, 0, NULL, &cnt), PG_OK);
        EXPECT(pg_bdl_erase(b, NULL, 0, NULL, &cnt), PG_OK);
        EXPECT(pg_bdl_knn(b, q, 1, 0, d64, d64, NULL), PG_ERR_INVALID);
        EXPECT(pg_bdl_knn(b, NULL, 0, 3, NULL, NULL, NULL), PG_OK);
        pg_bdl_free(b);
    }
    EXPECT(pg_bdl_create_spatial(2, PG_INT32, 8, 16, &b), PG_OK);
    pg_bdl_free(b);
    if (pg_bdl_size(NULL) != -1) fails++;
    pg_b1* b1 = NULL;
    EXPECT(pg_b1_create(9, PG_INT32, 16, &b1), PG_ERR_INVALID);
    EXPECT(pg_b1_create(3, PG_INT32, 16, &b1), PG_OK);
    if (b1) {
        EXPECT(pg_b1_insert(b1, NULL, 0, NULL, &cnt), PG_OK);
        EXPECT(pg_b1_knn(b1, NULL, 0, 5, NULL, NULL, NULL), PG_OK);
        if (pg_b1_size(b1) != 0) fails++;
        pg_b1_free(b1);
    }
    pg_b2* b2 = NULL;
    EXPECT(pg_b2_create(NULL, 10, 3, 16, PG_INT32, NULL, &b2), PG_ERR_INVALID);
    pg_b2_free(NULL);

    /* batched clouds: workspace planning is host work */
    int64_t offs[6] = {0, 0, 1, 300, 4000, 70000};
    size_t bytes = 0, prev = 0;
    EXPECT(pg_batch_workspace(offs, 5, 3, NULL, &bytes), PG_OK);
    if (bytes == 0) fails++;
    for (int l = 1; l <= 64; l *= 2) {
        pg_tune tn = {l, 2, 4, PG_KLIST_LDS};
        EXPECT(pg_batch_workspace(offs, 5, 8, &tn, &bytes), PG_OK);
        if (bytes == 0) fails++;
        prev = bytes;
    }
    (void)prev;
    EXPECT(pg_batch_workspace(offs, 0, 3, NULL, &bytes), PG_ERR_INVALID);
    EXPECT(pg_batch_workspace(offs, 5, 9, NULL, &bytes), PG_ERR_INVALID);
    int64_t bad[3] = {0, 5, 2};
    EXPECT(pg_batch_workspace(bad, 2, 3, NULL, &bytes), PG_ERR_INVALID);
    EXPECT(pg_batch_check(NULL, 5, 3, NULL), PG_ERR_INVALID);
    pg_tune best;
    EXPECT(pg_batch_autotune(NULL, NULL, 1, 3, 5, NULL, &best), PG_ERR_INVALID);
    EXPECT(pg_knn_backward(NULL, NULL, 1, 1, 3, 5, NULL, NULL, NULL, NULL, NULL), PG_ERR_INVALID);
    pg_batch_free(NULL);

    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("host sanitizer driver: ok\n");
    return 0;
}
