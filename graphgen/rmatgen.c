/* Multi-threaded builder for large R-MAT inputs.
 *
 * Produces exactly the graph that graphgen.rmat builds with numpy (same
 * Philox4x64-10 draw stream, same quadrant rule, same seeded relabelling,
 * same largest-component extraction and CSR layout), but in native code so
 * that graphs with 2^26 vertices and 2^30 edge draws build in about a
 * minute.  Input generation only: nothing here belongs to the sampling
 * method.
 *
 * Steps
 *  1. edge draw i of 2^scale * edge_factor: numpy's rng.random() stream
 *     consumed in chunks of 2^24 edges, one level of the recursion per pass
 *     over a chunk (draw index = chunk_base + level * chunk_len + j); the
 *     double is (raw >> 11) * 2^-53, as numpy's next_double;
 *  2. both directions of every non-loop edge, with the permuted ids, as
 *     keys src << scale | dst; parallel LSD radix sort; duplicates dropped;
 *  3. CSR over all 2^scale ids, components by BFS, the largest one kept
 *     (ties: the component of the smallest id), ids renumbered in ascending
 *     order of the permuted id.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- Philox4x64-10 (Salmon et al., SC'11), numpy's counter convention:
 * the stream's raw word k is word k mod 4 of the block at counter
 * k / 4 + 1 (numpy advances the counter before producing a block). */
/* four consecutive blocks at once (independent chains for the multipliers) */
static void philox_block4(uint64_t k0, uint64_t k1, uint64_t c_lo, uint64_t out[16])
{
    uint64_t c0[4], c1[4] = {0, 0, 0, 0}, c2[4] = {0, 0, 0, 0}, c3[4] = {0, 0, 0, 0};
    for (int q = 0; q < 4; ++q) c0[q] = c_lo + (uint64_t)q;
    for (int r = 0; r < 10; ++r) {
        for (int q = 0; q < 4; ++q) {
            const u128 p0 = (u128)0xD2E7470EE14C6C93ull * c0[q];
            const u128 p1 = (u128)0xCA5A826395121157ull * c2[q];
            const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
            const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
            const uint64_t n0 = hi1 ^ c1[q] ^ k0, n2 = hi0 ^ c3[q] ^ k1;
            c0[q] = n0;
            c1[q] = lo1;
            c2[q] = n2;
            c3[q] = lo0;
        }
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    for (int q = 0; q < 4; ++q) {
        out[4 * q + 0] = c0[q];
        out[4 * q + 1] = c1[q];
        out[4 * q + 2] = c2[q];
        out[4 * q + 3] = c3[q];
    }
}

typedef struct {
    int scale, ef;
    uint64_t key0, key1;
    double a, ab, abc;
    const int64_t *perm;
    uint64_t *keys;          /* 2 per draw, UINT64_MAX for loops */
    int64_t e0, e1;          /* this thread's draws */
} draw_job;

static void *draw_worker(void *p)
{
    draw_job *J = (draw_job *)p;
    const int64_t chunk = (int64_t)1 << 24;
    const int64_t total = ((int64_t)1 << J->scale) * J->ef;
    int64_t i = J->e0;
    while (i < J->e1) {
        const int64_t c = i / chunk;
        const int64_t cbeg = c * chunk;
        const int64_t clen = (total - cbeg) < chunk ? (total - cbeg) : chunk;
        const int64_t cend = cbeg + clen < J->e1 ? cbeg + clen : J->e1;
        const uint64_t base = (uint64_t)cbeg * (uint64_t)J->scale;
        /* tiles of edges so that the per-edge bit accumulators stay in cache
         * while every level of the recursion is drawn */
        enum { TILE = 2048 };
        uint32_t u[TILE], v[TILE];
        for (int64_t t0 = i; t0 < cend; t0 += TILE) {
            const int64_t cnt = (cend - t0) < TILE ? (cend - t0) : TILE;
            memset(u, 0, sizeof(u));
            memset(v, 0, sizeof(v));
            for (int l = 0; l < J->scale; ++l) {
                const uint64_t k0 = base + (uint64_t)l * (uint64_t)clen + (uint64_t)(t0 - cbeg);
                const uint64_t k1 = k0 + (uint64_t)cnt;          /* draws [k0, k1) */
                uint64_t words[16];
                for (uint64_t b = k0 >> 2; 4 * b < k1; b += 4) {
                    philox_block4(J->key0, J->key1, b + 1, words);
                    const uint64_t lo = 4 * b > k0 ? 4 * b : k0;
                    const uint64_t hi = 4 * b + 16 < k1 ? 4 * b + 16 : k1;
                    for (uint64_t k = lo; k < hi; ++k) {
                        const int64_t j = (int64_t)(k - k0);
                        const double r = (double)(words[k - 4 * b] >> 11) * (1.0 / 9007199254740992.0);
                        const uint32_t ub = r >= J->ab;
                        const uint32_t vb = ((r >= J->a) && (r < J->ab)) || (r >= J->abc);
                        u[j] = (u[j] << 1) | ub;
                        v[j] = (v[j] << 1) | vb;
                    }
                }
            }
            for (int64_t j = 0; j < cnt; ++j) {
                const uint64_t pu = (uint64_t)J->perm[u[j]], pv = (uint64_t)J->perm[v[j]];
                const int64_t at = 2 * (t0 + j);
                if (pu == pv) {
                    J->keys[at] = UINT64_MAX;
                    J->keys[at + 1] = UINT64_MAX;
                } else {
                    J->keys[at] = (pu << J->scale) | pv;
                    J->keys[at + 1] = (pv << J->scale) | pu;
                }
            }
        }
        i = cend;
    }
    return NULL;
}

/* ---- parallel LSD radix sort of uint64 keys on the low `bits` bits */
#define RB 11
#define RN (1 << RB)

typedef struct {
    const uint64_t *src;
    uint64_t *dst;
    int64_t b0, b1;
    int shift;
    int64_t *hist;           /* RN per thread */
    int phase;
} radix_job;

static void *radix_worker(void *p)
{
    radix_job *J = (radix_job *)p;
    if (J->phase == 0) {
        memset(J->hist, 0, sizeof(int64_t) * RN);
        for (int64_t i = J->b0; i < J->b1; ++i) J->hist[(J->src[i] >> J->shift) & (RN - 1)]++;
    } else {
        for (int64_t i = J->b0; i < J->b1; ++i) {
            const uint64_t k = J->src[i];
            J->dst[J->hist[(k >> J->shift) & (RN - 1)]++] = k;
        }
    }
    return NULL;
}

static int run_threads(int T, void *(*fn)(void *), void *jobs, size_t stride)
{
    pthread_t th[64];
    for (int t = 0; t < T; ++t)
        if (pthread_create(&th[t], NULL, fn, (char *)jobs + stride * t) != 0) return -1;
    for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* sorts keys[0..n) in place (tmp is scratch of the same size); returns the
 * buffer that holds the result */
static uint64_t *radix_sort(uint64_t *keys, uint64_t *tmp, int64_t n, int bits, int T)
{
    radix_job jobs[64];
    int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * RN * T);
    uint64_t *a = keys, *b = tmp;
    for (int shift = 0; shift < bits; shift += RB) {
        for (int t = 0; t < T; ++t) {
            jobs[t].src = a;
            jobs[t].dst = b;
            jobs[t].b0 = n * t / T;
            jobs[t].b1 = n * (t + 1) / T;
            jobs[t].shift = shift;
            jobs[t].hist = hist + (int64_t)RN * t;
            jobs[t].phase = 0;
        }
        run_threads(T, radix_worker, jobs, sizeof(radix_job));
        int64_t run = 0;
        for (int d = 0; d < RN; ++d)
            for (int t = 0; t < T; ++t) {
                const int64_t c = hist[(int64_t)RN * t + d];
                hist[(int64_t)RN * t + d] = run;
                run += c;
            }
        for (int t = 0; t < T; ++t) jobs[t].phase = 1;
        run_threads(T, radix_worker, jobs, sizeof(radix_job));
        uint64_t *x = a;
        a = b;
        b = x;
    }
    free(hist);
    return a;
}

typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t *row_ptr;
    int32_t *col_idx;
} kg_graph;

void kg_free(kg_graph *g)
{
    if (!g) return;
    free(g->row_ptr);
    free(g->col_idx);
    free(g);
}

int32_t kg_n(const kg_graph *g) { return g->n; }
int64_t kg_nnz(const kg_graph *g) { return g->nnz; }
void kg_copy(const kg_graph *g, int64_t *row_ptr, int32_t *col_idx)
{
    memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * ((size_t)g->n + 1));
    memcpy(col_idx, g->col_idx, sizeof(int32_t) * (size_t)g->nnz);
}

/* Graph from directed keys src << scale | dst over 2^scale ids (UINT64_MAX
 * marks a dropped entry; keys is freed): loops dropped, sorted, duplicates
 * dropped, CSR, the largest component kept (ties: the component of the
 * smallest id), ids renumbered in ascending order. */
static kg_graph *graph_from_keys(uint64_t *keys, int64_t nk, int scale, int threads)
{
    const int64_t N = (int64_t)1 << scale;
    /* drop loops (stable compaction), then sort */
    int64_t m = 0;
    for (int64_t i = 0; i < nk; ++i)
        if (keys[i] != UINT64_MAX) keys[m++] = keys[i];
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m ? m : 1));
    if (!tmp) {
        free(keys);
        return NULL;
    }
    uint64_t *s = radix_sort(keys, tmp, m, 2 * scale, threads);
    uint64_t *other = (s == keys) ? tmp : keys;
    free(other);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i)
        if (u == 0 || s[i] != s[u - 1]) s[u++] = s[i];

    /* CSR over all ids */
    const uint64_t mask = (uint64_t)N - 1;
    int64_t *rp = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(u ? u : 1));
    if (!rp || !ci) {
        free(s);
        free(rp);
        free(ci);
        return NULL;
    }
    for (int64_t i = 0; i < u; ++i) {
        rp[(s[i] >> scale) + 1]++;
        ci[i] = (int32_t)(s[i] & mask);
    }
    free(s);
    for (int64_t v = 0; v < N; ++v) rp[v + 1] += rp[v];

    /* components by BFS in ascending id order */
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!comp || !q) {
        free(rp);
        free(ci);
        free(comp);
        free(q);
        return NULL;
    }
    for (int64_t v = 0; v < N; ++v) comp[v] = -1;
    int32_t ncomp = 0, best = -1;
    int64_t best_size = 0;
    for (int64_t r = 0; r < N; ++r) {
        if (comp[r] >= 0) continue;
        int64_t h = 0, t = 0;
        q[t++] = (int32_t)r;
        comp[r] = ncomp;
        while (h < t) {
            const int32_t x = q[h++];
            for (int64_t e = rp[x]; e < rp[x + 1]; ++e) {
                const int32_t y = ci[e];
                if (comp[y] < 0) {
                    comp[y] = ncomp;
                    q[t++] = y;
                }
            }
        }
        if (t > best_size) {
            best_size = t;
            best = ncomp;
        }
        ncomp++;
    }
    /* renumber the kept component in ascending id order */
    int32_t *newid = q;
    int32_t nn = 0;
    for (int64_t v = 0; v < N; ++v) newid[v] = (comp[v] == best) ? nn++ : -1;
    kg_graph *g = (kg_graph *)calloc(1, sizeof(kg_graph));
    int64_t nnz = 0;
    for (int64_t v = 0; v < N; ++v)
        if (comp[v] == best) nnz += rp[v + 1] - rp[v];
    g->n = nn;
    g->nnz = nnz;
    g->row_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nn + 1));
    g->col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    if (!g->row_ptr || !g->col_idx) {
        kg_free(g);
        free(rp);
        free(ci);
        free(comp);
        free(q);
        return NULL;
    }
    int64_t at = 0;
    g->row_ptr[0] = 0;
    for (int64_t v = 0; v < N; ++v) {
        if (comp[v] != best) continue;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) g->col_idx[at++] = newid[ci[e]];
        g->row_ptr[newid[v] + 1] = at;
    }
    free(rp);
    free(ci);
    free(comp);
    free(q);
    return g;
}

/* Returns NULL on allocation failure or bad arguments. */
kg_graph *kg_rmat(int scale, int edge_factor, uint64_t seed, uint64_t stream, double a, double b, double c,
                  const int64_t *perm, int threads)
{
    if (scale < 1 || scale > 30 || edge_factor < 1 || threads < 1) return NULL;
    if (threads > 64) threads = 64;
    const int64_t N = (int64_t)1 << scale;
    const int64_t total = N * edge_factor;
    const int64_t nk = 2 * total;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nk);
    if (!keys) return NULL;

    draw_job dj[64];
    const double ab = a + b, abc = a + b + c;
    for (int t = 0; t < threads; ++t) {
        dj[t].scale = scale;
        dj[t].ef = edge_factor;
        dj[t].key0 = seed;
        dj[t].key1 = stream;
        dj[t].a = a;
        dj[t].ab = ab;
        dj[t].abc = abc;
        dj[t].perm = perm;
        dj[t].keys = keys;
        dj[t].e0 = total * t / threads;
        dj[t].e1 = total * (t + 1) / threads;
    }
    run_threads(threads, draw_worker, dj, sizeof(draw_job));

    return graph_from_keys(keys, nk, scale, threads);
}

/* ---- Random hyperbolic graphs (Krioukov et al., threshold model): n =
 * 2^scale points in a hyperbolic disk of radius R, angle uniform, radius
 * with density alpha sinh(alpha r) / (cosh(alpha R) - 1), alpha = (gamma -
 * 1) / 2 for a power-law degree exponent gamma; two points are adjacent
 * when their hyperbolic distance is at most R:
 *   cosh r1 cosh r2 - sinh r1 sinh r2 cos(t1 - t2) <= cosh R.
 * R is chosen so that the expected average degree is avg_deg (numerical
 * integration of the adjacency probability over the radial law, then
 * bisection on R).  Neighbours are found band by band: the points sorted
 * by radial band and angle, a point scans in each band only the angles its
 * threshold admits at the band's inner radius (the threshold angle shrinks
 * as the other radius grows), then tests each candidate exactly.  Every
 * edge is found from both ends; ids are permuted by `perm`, then the keys
 * go through graph_from_keys (largest component, ascending renumbering).
 * Random numbers: point i takes words 0 (radius) and 1 (angle) of Philox
 * block i of (seed, stream).  Input generation only. */
#include <math.h>

static double hyp_theta_max(double r1, double r2, double R, double coshR)
{
    if (r1 + r2 <= R) return M_PI;
    double c = (cosh(r1) * cosh(r2) - coshR) / (sinh(r1) * sinh(r2));
    if (c <= -1.0) return M_PI;
    if (c >= 1.0) return 0.0;
    return acos(c);
}

/* radius at quantile q of the radial law */
static double hyp_radius(double q, double alpha, double R)
{
    return acosh(1.0 + (cosh(alpha * R) - 1.0) * q) / alpha;
}

/* expected average degree for n points in a disk of radius R: n times the
 * mean over two independent radii of theta_max / pi (midpoint rule on a
 * grid of Q quantiles) */
static double hyp_avg_degree(int64_t n, double alpha, double R)
{
    const int Q = 600;
    double rq[600];
    for (int i = 0; i < Q; ++i) rq[i] = hyp_radius((i + 0.5) / Q, alpha, R);
    const double coshR = cosh(R);
    double s = 0.0;
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) s += hyp_theta_max(rq[i], rq[j], R, coshR);
    return (double)(n - 1) * s / ((double)Q * Q * M_PI);
}

static void philox_one(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t out[4])
{
    uint64_t c[4] = {c0, 0, 0, 0};
    for (int r = 0; r < 10; ++r) {
        const u128 p0 = (u128)0xD2E7470EE14C6C93ull * c[0];
        const u128 p1 = (u128)0xCA5A826395121157ull * c[2];
        const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0, n2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
        c[1] = (uint64_t)p1;
        c[3] = (uint64_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    memcpy(out, c, sizeof(c));
}

#define HYP_MAXB 64

typedef struct {
    int64_t n;
    double R, coshR;
    const double *th, *ch, *sh, *rr;   /* by sorted position */
    const int32_t *id;                 /* original point of a sorted position */
    const int64_t *bstart;             /* band b = sorted positions [bstart[b], bstart[b+1]) */
    const double *binner;              /* inner radius of band b */
    int nb;
    const int64_t *perm;
    int scale;
    int64_t p0, p1;                    /* this thread's sorted positions */
    uint64_t *out;
    int64_t cnt, cap;
    int fail;
} hyp_job;

static void hyp_emit(hyp_job *J, uint64_t k)
{
    if (J->cnt == J->cap) {
        int64_t nc = J->cap ? 2 * J->cap : (1 << 20);
        uint64_t *q = (uint64_t *)realloc(J->out, sizeof(uint64_t) * (size_t)nc);
        if (!q) { J->fail = 1; return; }
        J->out = q;
        J->cap = nc;
    }
    J->out[J->cnt++] = k;
}

/* first sorted position in [lo, hi) whose angle is >= x */
static int64_t hyp_lower(const double *th, int64_t lo, int64_t hi, double x)
{
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (th[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static void hyp_scan(hyp_job *J, int64_t p, int64_t lo, int64_t hi)
{
    const double chp = J->ch[p], shp = J->sh[p], thp = J->th[p];
    const uint64_t src = (uint64_t)J->perm[J->id[p]] << J->scale;
    for (int64_t q = lo; q < hi && !J->fail; ++q) {
        if (q == p) continue;
        if (chp * J->ch[q] - shp * J->sh[q] * cos(thp - J->th[q]) <= J->coshR)
            hyp_emit(J, src | (uint64_t)J->perm[J->id[q]]);
    }
}

static void *hyp_worker(void *arg)
{
    hyp_job *J = (hyp_job *)arg;
    const double margin = 1e-9;
    for (int64_t p = J->p0; p < J->p1 && !J->fail; ++p) {
        for (int b = 0; b < J->nb; ++b) {
            const int64_t lo = J->bstart[b], hi = J->bstart[b + 1];
            if (lo == hi) continue;
            const double d = hyp_theta_max(J->rr[p], J->binner[b], J->R, J->coshR) + margin;
            if (d >= M_PI) {
                hyp_scan(J, p, lo, hi);
                continue;
            }
            const double a = J->th[p] - d, z = J->th[p] + d;
            if (a < 0.0) {
                hyp_scan(J, p, hyp_lower(J->th, lo, hi, a + 2.0 * M_PI), hi);
                hyp_scan(J, p, lo, hyp_lower(J->th, lo, hi, z));
            } else if (z > 2.0 * M_PI) {
                hyp_scan(J, p, hyp_lower(J->th, lo, hi, a), hi);
                hyp_scan(J, p, lo, hyp_lower(J->th, lo, hi, z - 2.0 * M_PI));
            } else {
                hyp_scan(J, p, hyp_lower(J->th, lo, hi, a), hyp_lower(J->th, lo, hi, z));
            }
        }
    }
    return NULL;
}

/* *R_out: the disk radius used. */
kg_graph *kg_hyperbolic(int scale, double avg_deg, double gamma, uint64_t seed, uint64_t stream,
                        const int64_t *perm, int threads, double *R_out)
{
    if (scale < 2 || scale > 26 || !(avg_deg > 0.0) || !(gamma > 2.0) || threads < 1) return NULL;
    if (threads > 64) threads = 64;
    const int64_t N = (int64_t)1 << scale;
    const double alpha = (gamma - 1.0) / 2.0;
    /* R: the expected average degree decreases in R */
    double lo = 0.5, hi = 200.0;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (hyp_avg_degree(N, alpha, mid) > avg_deg) lo = mid; else hi = mid;
    }
    const double R = 0.5 * (lo + hi);
    if (R_out) *R_out = R;
    /* bands of width 1/2 in r (the last one ends at R) */
    int nb = (int)ceil(R / 0.5);
    if (nb > HYP_MAXB) nb = HYP_MAXB;
    const double bw = R / nb;
    double binner[HYP_MAXB + 1];
    for (int b = 0; b <= nb; ++b) binner[b] = bw * b;
    /* points, sorted by (band, angle) through 64-bit keys: band 6 bits,
     * angle 32 bits, point index 26 bits */
    double *r0 = (double *)malloc(sizeof(double) * (size_t)N);
    double *t0 = (double *)malloc(sizeof(double) * (size_t)N);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    if (!r0 || !t0 || !keys || !tmp) { free(r0); free(t0); free(keys); free(tmp); return NULL; }
    for (int64_t i = 0; i < N; ++i) {
        uint64_t w[4];
        philox_one(seed, stream, (uint64_t)i, w);
        const double u = (double)(w[0] >> 11) * 0x1p-53, v = (double)(w[1] >> 11) * 0x1p-53;
        r0[i] = hyp_radius(u, alpha, R);
        t0[i] = 2.0 * M_PI * v;
        int b = (int)(r0[i] / bw);
        if (b >= nb) b = nb - 1;
        const uint64_t tq = (uint64_t)(v * 4294967296.0);
        keys[i] = ((uint64_t)b << 58) | ((tq & 0xffffffffull) << 26) | (uint64_t)i;
    }
    uint64_t *s = radix_sort(keys, tmp, N, 64, threads);
    double *th = (double *)malloc(sizeof(double) * (size_t)N), *ch = (double *)malloc(sizeof(double) * (size_t)N);
    double *sh = (double *)malloc(sizeof(double) * (size_t)N), *rr = (double *)malloc(sizeof(double) * (size_t)N);
    int32_t *id = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int64_t bstart[HYP_MAXB + 1];
    if (!th || !ch || !sh || !rr || !id) {
        free(r0); free(t0); free(keys); free(tmp); free(th); free(ch); free(sh); free(rr); free(id);
        return NULL;
    }
    for (int b = 0; b <= nb; ++b) bstart[b] = N;
    for (int64_t p = N - 1; p >= 0; --p) {
        const int64_t i = (int64_t)(s[p] & ((1ull << 26) - 1));
        const int b = (int)(s[p] >> 58);
        id[p] = (int32_t)i;
        th[p] = t0[i];
        rr[p] = r0[i];
        ch[p] = cosh(r0[i]);
        sh[p] = sinh(r0[i]);
        bstart[b] = p;
    }
    for (int b = nb - 1; b >= 0; --b)
        if (bstart[b] > bstart[b + 1]) bstart[b] = bstart[b + 1];
    /* angles within a band ascend up to the 32-bit quantisation of the key;
     * make them exactly ascending for the binary searches */
    for (int b = 0; b < nb; ++b)
        for (int64_t p = bstart[b] + 1; p < bstart[b + 1]; ++p)
            if (th[p] < th[p - 1]) th[p] = th[p - 1];
    free(r0); free(t0); free(keys); free(tmp);
    hyp_job jobs[64];
    memset(jobs, 0, sizeof(jobs));
    for (int t = 0; t < threads; ++t) {
        jobs[t].n = N;
        jobs[t].R = R;
        jobs[t].coshR = cosh(R);
        jobs[t].th = th;
        jobs[t].ch = ch;
        jobs[t].sh = sh;
        jobs[t].rr = rr;
        jobs[t].id = id;
        jobs[t].bstart = bstart;
        jobs[t].binner = binner;
        jobs[t].nb = nb;
        jobs[t].perm = perm;
        jobs[t].scale = scale;
        jobs[t].p0 = N * t / threads;
        jobs[t].p1 = N * (t + 1) / threads;
    }
    run_threads(threads, hyp_worker, jobs, sizeof(hyp_job));
    int64_t total = 0;
    int fail = 0;
    for (int t = 0; t < threads; ++t) {
        total += jobs[t].cnt;
        fail |= jobs[t].fail;
    }
    free(th); free(ch); free(sh); free(rr); free(id);
    uint64_t *all = fail ? NULL : (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(total ? total : 1));
    int64_t at = 0;
    for (int t = 0; t < threads; ++t) {
        if (all) memcpy(all + at, jobs[t].out, sizeof(uint64_t) * (size_t)jobs[t].cnt);
        at += jobs[t].cnt;
        free(jobs[t].out);
    }
    if (!all) return NULL;
    return graph_from_keys(all, total, scale, threads);
}
