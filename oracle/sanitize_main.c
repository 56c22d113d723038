/*
 * Test driver of the oracle under the compilers' sanitizers (test
 * infrastructure only).  Builds a small seeded graph -- a grid with chords
 * -- and exercises every entry point of the oracle, the threaded runner
 * included, so that an AddressSanitizer / UndefinedBehaviorSanitizer build
 * and a ThreadSanitizer build can check them.  Exit status 0 on success.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* side x side grid plus side chords between seeded vertex pairs */
static orc_graph make_graph(int32_t side, int64_t **rp_out, int32_t **ci_out)
{
    const int32_t n = side * side;
    int64_t m = 0, cap = 8 * (int64_t)n + 8;
    int32_t *u = malloc(sizeof(int32_t) * cap), *v = malloc(sizeof(int32_t) * cap);
    for (int32_t r = 0; r < side; ++r)
        for (int32_t c = 0; c < side; ++c) {
            const int32_t x = r * side + c;
            if (c + 1 < side) { u[m] = x; v[m++] = x + 1; }
            if (r + 1 < side) { u[m] = x; v[m++] = x + side; }
        }
    for (int32_t k = 0; k < side; ++k) {
        const int32_t a = (int32_t)(orc_draw(9, 3, (uint64_t)k, 0) % (uint64_t)n);
        const int32_t b = (int32_t)(orc_draw(9, 3, (uint64_t)k, 1) % (uint64_t)n);
        if (a != b) { u[m] = a; v[m++] = b; }
    }
    int64_t *rp = calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) { rp[u[e] + 1]++; rp[v[e] + 1]++; }
    for (int32_t x = 0; x < n; ++x) rp[x + 1] += rp[x];
    int32_t *ci = malloc(sizeof(int32_t) * (size_t)(2 * m));
    int64_t *at = malloc(sizeof(int64_t) * (size_t)n);
    for (int32_t x = 0; x < n; ++x) at[x] = rp[x];
    for (int64_t e = 0; e < m; ++e) { ci[at[u[e]]++] = v[e]; ci[at[v[e]]++] = u[e]; }
    /* sort rows and drop duplicates */
    int64_t w = 0;
    int64_t *rp2 = calloc((size_t)n + 1, sizeof(int64_t));
    for (int32_t x = 0; x < n; ++x) {
        qsort(ci + rp[x], (size_t)(rp[x + 1] - rp[x]), sizeof(int32_t), cmp_i32);
        for (int64_t e = rp[x]; e < rp[x + 1]; ++e)
            if (e == rp[x] || ci[e] != ci[e - 1]) ci[w++] = ci[e];
        rp2[x + 1] = w;
    }
    free(u); free(v); free(at); free(rp);
    *rp_out = rp2;
    *ci_out = ci;
    orc_graph g = {n, rp2, ci};
    return g;
}

#define CHECK(cond)                                                 \
    do {                                                            \
        if (!(cond)) {                                              \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main(void)
{
    int64_t *rp;
    int32_t *ci;
    orc_graph g = make_graph(24, &rp, &ci);
    const int32_t n = g.n;
    orc_ws *w = orc_ws_create(n);
    int32_t *path = malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (int mode = 0; mode < 2; ++mode)
        for (uint64_t i = 0; i < 300; ++i) {
            orc_sample_info info;
            CHECK(orc_sample_path(&g, w, 5, 0, i, mode, path, &info) == ORC_OK);
            CHECK(info.d >= 1 && path[0] == info.s && path[info.d] == info.t);
        }
    orc_ws_free(w);
    int64_t lo, hi;
    orc_vd_bracket(&g, &lo, &hi);
    const int64_t vd = orc_exact_vd(&g);
    CHECK(lo <= vd && vd <= hi);
    CHECK(orc_eccentricity(&g, 0) <= vd - 1);
    const double omega = orc_omega_bracket(lo, hi, 0.05, 0.1);
    double *LL = malloc(sizeof(double) * n), *LU = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
    for (int32_t v = 0; v < n; ++v) d[v] = 0.999 * 0.1 / (4.0 * n);
    orc_neglog(n, d, LL);
    memcpy(LU, LL, sizeof(double) * n);
    uint32_t *c1 = calloc(n, sizeof(uint32_t)), *c2 = calloc(n, sizeof(uint32_t));
    orc_run_opts o = {1, 0, 0.05, omega, 200, 0, 0, 0};
    orc_run_result r1, r2;
    orc_check_info per[256];
    CHECK(orc_run(&g, &o, LL, LU, c1, &r1, per, 256) == ORC_OK);
    CHECK(orc_run_mt(&g, &o, LL, LU, c2, &r2, per, 256, 3) == ORC_OK);
    CHECK(r1.tau == r2.tau && r1.epochs == r2.epochs && memcmp(c1, c2, sizeof(uint32_t) * n) == 0);
    memset(c1, 0, sizeof(uint32_t) * n);
    memset(c2, 0, sizeof(uint32_t) * n);
    CHECK(orc_count(&g, 2, 1, 0, 500, 0, c1, NULL) == ORC_OK);
    CHECK(orc_count_mt(&g, 2, 1, 0, 500, 0, c2, NULL, 4) == ORC_OK);
    CHECK(memcmp(c1, c2, sizeof(uint32_t) * n) == 0);
    double C;
    CHECK(orc_calibrate_mt(&g, 1, omega, 0.1, 0, c1, &C, LL, LU, 2) == ORC_OK);
    double *bc = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * 3 * n), *y = malloc(sizeof(double) * n);
    orc_brandes(&g, bc);
    orc_features(&g, x);
    for (int32_t v = 0; v < n; ++v) y[v] = bc[v];
    double p[ORC_MLP_PARAMS], gr[ORC_MLP_PARAMS], losses[2];
    orc_mlp_init(3, p);
    const double loss = orc_mlp_loss_grad(p, x, y, n, gr);
    CHECK(loss == loss);
    orc_mlp_train(x, y, n, 2, 64, 1e-3, 1, 3, p, losses);
    double pr[4], yy[4] = {-3.0, 0.0, 2.0, -20.0};
    orc_prior_from_output(4, yy, omega, pr);
    free(LL); free(LU); free(d); free(c1); free(c2); free(bc); free(x); free(y); free(path);
    free(rp); free(ci);
    printf("oracle sanitizer driver: ok (n=%d, VD=%lld, tau=%llu)\n", n, (long long)vd, (unsigned long long)r1.tau);
    return 0;
}
