/* Exercises the CPU oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built and run by tests/test_sanitizers.py): random and
 * duplicate-heavy sets, int32 and float32, every search against the brute
 * definition, spatial trees of every rule, WSPD.  Exits non-zero on a
 * mismatch; the sanitizers abort on a memory or UB error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* the oracle's entry points (oracle/oracle.c); trees are opaque here */
int or_knn_brute(const void* pts, const int64_t* ids, const uint8_t* alive, int64_t n, int d, int dt,
                 const void* qs, int64_t m, int k, int64_t* out_id, void* out_dist, int nthreads);
void* or_kd_build(const void* pts, int64_t n, int d, int dt, int leaf);
void or_kd_free(void* T);
int or_kd_levels(const void* T);
void or_kd_export(const void* T, double* split_out, int64_t* perm_out);
int or_kd_knn(const void* T, const int64_t* ids, const uint8_t* alive, const void* qs, int64_t m, int k,
              int64_t* out_id, void* out_dist, int64_t* counters);
int or_range_brute(const void* pts, const int64_t* ids, const uint8_t* alive, int64_t n, int d, int dt,
                   const void* boxes, int64_t m, int64_t* counts, const int64_t* offsets, int64_t* out_id);
int or_kd_range(const void* T, const int64_t* ids, const uint8_t* alive, const void* boxes, int64_t m,
                int64_t* counts, const int64_t* offsets, int64_t* out_id, int64_t* counters);
void* or_sp_build(const void* pts, int64_t n, int d, int dt, int leaf, int rule);
void or_sp_free(void* T);
int64_t or_sp_nodes(const void* T);
int or_sp_depth(const void* T);
void or_sp_export(const void* T, double* split, int32_t* dim, int64_t* child, int64_t* lo, int64_t* hi,
                  int32_t* level, int64_t* perm);
int64_t or_wspd(const void* T, double s, int64_t* out, int64_t cap);

static uint64_t rng = 88172645463325252ull;
static uint64_t next(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

static int fails = 0;
#define CHECK(c, ...)                 \
    do {                              \
        if (!(c)) {                   \
            fprintf(stderr, __VA_ARGS__); \
            fprintf(stderr, "\n");    \
            fails++;                  \
        }                             \
    } while (0)

static void make_points(void* p, int64_t n, int d, int dt, int span) {
    for (int64_t i = 0; i < n * d; i++) {
        if (dt == 0) ((int32_t*)p)[i] = (int32_t)(next() % (uint64_t)span) - span / 2;
        else ((float*)p)[i] = (float)((double)(next() % (uint64_t)span) / 7.0 - span / 14.0);
    }
}

static void knn_case(int64_t n, int d, int dt, int leaf, int k, int span) {
    const size_t w = 4;
    void* pts = malloc(w * (size_t)(n > 0 ? n : 1) * d);
    int64_t m = 37;
    void* qs = malloc(w * (size_t)m * d);
    make_points(pts, n, d, dt, span);
    make_points(qs, m, d, dt, span);
    uint8_t* alive = malloc((size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) alive[i] = (uint8_t)(next() % 5 != 0);
    int64_t *bi = malloc(sizeof(int64_t) * m * k), *ki = malloc(sizeof(int64_t) * m * k);
    double *bd = malloc(sizeof(double) * m * k), *kd = malloc(sizeof(double) * m * k);
    for (int live = 0; live < 2; live++) {
        const uint8_t* a = live ? alive : NULL;
        CHECK(or_knn_brute(pts, NULL, a, n, d, dt, qs, m, k, bi, bd, 3) == 0, "brute failed");
        void* T = or_kd_build(pts, n, d, dt, leaf);
        CHECK(T != NULL, "build failed");
        int64_t cnt[3] = {0, 0, 0};
        CHECK(or_kd_knn(T, NULL, a, qs, m, k, ki, kd, cnt) == 0, "kd knn failed");
        CHECK(memcmp(bi, ki, sizeof(int64_t) * m * k) == 0, "ids differ n=%lld d=%d dt=%d", (long long)n, d, dt);
        CHECK(memcmp(bd, kd, sizeof(double) * m * k) == 0, "distances differ n=%lld d=%d dt=%d", (long long)n, d, dt);
        int L = or_kd_levels(T);
        double* split = malloc(sizeof(double) * ((size_t)1 << L));
        int64_t* perm = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        or_kd_export(T, split, perm);
        /* range: boxes around query points */
        double* boxes = malloc(sizeof(double) * m * 2 * d);
        void* bx = malloc(w * (size_t)m * 2 * d);
        for (int64_t i = 0; i < m; i++)
            for (int c = 0; c < d; c++) {
                const int r = (int)(next() % (uint64_t)(span / 4 + 1));
                if (dt == 0) {
                    ((int32_t*)bx)[i * 2 * d + c] = ((int32_t*)qs)[i * d + c] - r;
                    ((int32_t*)bx)[i * 2 * d + d + c] = ((int32_t*)qs)[i * d + c] + r;
                } else {
                    ((float*)bx)[i * 2 * d + c] = ((float*)qs)[i * d + c] - (float)r / 7.0f;
                    ((float*)bx)[i * 2 * d + d + c] = ((float*)qs)[i * d + c] + (float)r / 7.0f;
                }
            }
        int64_t *c1 = malloc(sizeof(int64_t) * m), *c2 = malloc(sizeof(int64_t) * m);
        CHECK(or_range_brute(pts, NULL, a, n, d, dt, bx, m, c1, NULL, NULL) == 0, "range brute failed");
        int64_t rc[2];
        CHECK(or_kd_range(T, NULL, a, bx, m, c2, NULL, NULL, rc) == 0, "kd range failed");
        CHECK(memcmp(c1, c2, sizeof(int64_t) * m) == 0, "range counts differ");
        int64_t* off = malloc(sizeof(int64_t) * (m + 1));
        off[0] = 0;
        for (int64_t i = 0; i < m; i++) off[i + 1] = off[i] + c1[i];
        int64_t* rows = malloc(sizeof(int64_t) * (size_t)(off[m] > 0 ? off[m] : 1));
        CHECK(or_kd_range(T, NULL, a, bx, m, c2, off, rows, NULL) == 0, "kd range rows failed");
        free(rows); free(off); free(c1); free(c2); free(bx); free(boxes); free(split); free(perm);
        or_kd_free(T);
    }
    for (int rule = 0; rule < 4; rule++) {
        void* S = or_sp_build(pts, n, d, dt, leaf, rule);
        CHECK(S != NULL, "spatial build failed");
        const int64_t N = or_sp_nodes(S);
        double* sp = malloc(sizeof(double) * N);
        int32_t* dim = malloc(sizeof(int32_t) * N);
        int64_t *ch = malloc(sizeof(int64_t) * N), *lo = malloc(sizeof(int64_t) * N), *hi = malloc(sizeof(int64_t) * N);
        int32_t* lv = malloc(sizeof(int32_t) * N);
        int64_t* perm = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        or_sp_export(S, sp, dim, ch, lo, hi, lv, perm);
        CHECK(N == 0 || (lo[0] == 0 && hi[0] == n), "spatial root range");
        (void)or_sp_depth(S);
        free(sp); free(dim); free(ch); free(lo); free(hi); free(lv); free(perm);
        or_sp_free(S);
    }
    free(bi); free(ki); free(bd); free(kd); free(alive); free(pts); free(qs);
}

static void wspd_case(int64_t n, int dt) {
    void* pts = malloc(4 * (size_t)(n > 0 ? n : 1) * 2);
    make_points(pts, n, 2, dt, 1000);
    void* T = or_kd_build(pts, n, 2, dt, 1);
    const int64_t total = or_wspd(T, 2.0, NULL, 0);
    CHECK(total >= 0, "wspd failed");
    int64_t* out = malloc(sizeof(int64_t) * 2 * (size_t)(total > 0 ? total : 1));
    CHECK(or_wspd(T, 2.0, out, total) == total, "wspd count changed");
    CHECK(or_wspd(T, -1.0, NULL, 0) == -1, "bad s accepted");
    free(out);
    or_kd_free(T);
    free(pts);
}

int main(void) {
    const int64_t ns[] = {0, 1, 2, 17, 300, 2100, 20000};
    for (int t = 0; t < 7; t++)
        for (int dt = 0; dt < 2; dt++) {
            knn_case(ns[t], 1 + (int)(next() % 8), dt, 1 + (int)(next() % 16), 1 + (int)(next() % 12), 1000);
            knn_case(ns[t], 3, dt, 4, 7, 6);  /* duplicate-heavy */
        }
    wspd_case(0, 0);
    wspd_case(1, 1);
    wspd_case(400, 0);
    wspd_case(300, 1);
    wspd_case(3000, 0);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
