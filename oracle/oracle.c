/*
 * Plain CPU oracle for KADABRA-style adaptive-sampling betweenness
 * approximation (van der Grinten & Meyerhenke, "Scaling Betweenness
 * Approximation to Billions of Edges by MPI-based Adaptive Sampling").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP library: it has its own Philox, its own BFS, its own stop
 * rule.  Everything is written for a reader who checks it against the
 * paper, not for speed: one sample at a time, one thread, FP64 wherever
 * floating point appears.
 *
 * What the paper fixes, and what is a reading of this project:
 *   - betweenness of x: sum over ordered pairs s != t of sigma_st(x)/sigma_st,
 *     divided by n(n-1); x counts only as an intermediate vertex (Sec. I).
 *   - a sample draws a pair s != t, samples one shortest s-t path uniformly
 *     and adds one to c~(x) for each vertex x on it; b~ = c~ / tau
 *     (Sec. III-A).  Only interior vertices are counted (reading: the
 *     definition in Sec. I counts intermediate vertices only).
 *   - the path is found by a bidirectional BFS (Sec. III-A).  The balancing
 *     rule, the set-semantics layers and the meet rule are readings
 *     (KADABRA's own paper is cited there, not reproduced).
 *   - stop when f < eps and g < eps for every vertex, or tau reaches omega
 *     (Sec. III-A).  The formulas for f, g and omega are KADABRA's, recalled
 *     here, not printed in the paper ("parity unpinned" against KADABRA's
 *     own text; pinned here by the closed forms in the tests).
 *   - the check runs on a consistent snapshot once per epoch (Sec. III-B,
 *     Alg. 2); this oracle uses fixed epochs of E samples.
 *   - the random numbers: Philox4x64-10 (Salmon et al., SC'11), key =
 *     (seed, stream), counter = (block, sample index, 0, 0); draw j of a
 *     sample is word j mod 4 of block floor(j / 4).
 *
 * Sigma arithmetic (not in the paper).  Integer mode: uint64 with exact
 * overflow detection; any overflow switches the whole sample to FP mode.
 * FP mode: FP64 values summed in ascending CSR position, each evaluated
 * layer rescaled by 2^-400 when its maximum exceeds 2^400.  Path choice:
 * the meet vertex in ascending id, then predecessors in CSR order, each
 * chosen as the first candidate whose inclusive prefix sum exceeds a draw
 * scaled to the total.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ------------------------------------------------------------------ */
/* Philox4x64-10, from its published definition (Salmon, Moraes, Dror,  */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).         */
/* ------------------------------------------------------------------ */

static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c0, &hi0, &lo0);
        mul128(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint64_t orc_draw(uint64_t seed, uint64_t stream, uint64_t sample, uint64_t j)
{
    uint64_t key[2] = {seed, stream};
    uint64_t ctr[4] = {j / 4, sample, 0, 0};
    uint64_t out[4];
    orc_philox4x64_10(key, ctr, out);
    return out[j % 4];
}

static uint64_t mulhi64(uint64_t a, uint64_t b)
{
    uint64_t hi, lo;
    mul128(a, b, &hi, &lo);
    return hi;
}

/* Uniform ordered pair s != t (the estimator samples pairs s != t). */
void orc_pair(uint64_t seed, uint64_t stream, uint64_t sample, int32_t n,
              int32_t *s, int32_t *t)
{
    uint64_t u0 = orc_draw(seed, stream, sample, 0);
    uint64_t u1 = orc_draw(seed, stream, sample, 1);
    int32_t ss = (int32_t)mulhi64(u0, (uint64_t)n);
    int32_t tt = (int32_t)mulhi64(u1, (uint64_t)(n - 1));
    if (tt >= ss) tt += 1;
    *s = ss;
    *t = tt;
}

/* ------------------------------------------------------------------ */
/* Workspace: per-vertex arrays reused between samples.  Entries that a  */
/* sample touched are reset before the next one starts.                 */
/* ------------------------------------------------------------------ */

struct orc_ws {
    int32_t n;
    int32_t *dist[2];        /* BFS depth from s (side 0) and t (side 1), -1 = unseen */
    uint64_t *isig[2];       /* integer-mode sigma                              */
    double *fsig[2];         /* FP-mode sigma                                   */
    int32_t *verts[2];       /* vertices of each side in layer order            */
    int64_t *loff[2];        /* layer j = verts[loff[j] .. loff[j+1])           */
    int32_t nlayers[2];      /* number of layers of each side                   */
    int32_t *meet;           /* meet set                                        */
    int32_t nmeet;
    int32_t *path;           /* s = path[0] .. path[d] = t                      */
    uint8_t *lscaled[2];     /* FP mode: layer j was rescaled by 2^-400         */
};

orc_ws *orc_ws_create(int32_t n)
{
    orc_ws *w = (orc_ws *)calloc(1, sizeof(orc_ws));
    w->n = n;
    for (int side = 0; side < 2; ++side) {
        w->dist[side] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int32_t v = 0; v < n; ++v) w->dist[side][v] = -1;
        w->isig[side] = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
        w->fsig[side] = (double *)calloc((size_t)n, sizeof(double));
        w->verts[side] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        w->loff[side] = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 2));
        w->lscaled[side] = (uint8_t *)calloc((size_t)n + 2, 1);
    }
    w->meet = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    w->path = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    return w;
}

void orc_ws_free(orc_ws *w)
{
    if (!w) return;
    for (int side = 0; side < 2; ++side) {
        free(w->dist[side]); free(w->isig[side]); free(w->fsig[side]);
        free(w->verts[side]); free(w->loff[side]); free(w->lscaled[side]);
    }
    free(w->meet); free(w->path); free(w);
}

static void ws_reset(orc_ws *w)
{
    for (int side = 0; side < 2; ++side) {
        int64_t cnt = w->loff[side][w->nlayers[side]];
        for (int64_t i = 0; i < cnt; ++i) w->dist[side][w->verts[side][i]] = -1;
        w->nlayers[side] = 0;
        w->loff[side][0] = 0;
    }
    /* Meet vertices were marked by the meeting side but not listed there. */
    for (int32_t i = 0; i < w->nmeet; ++i) {
        w->dist[0][w->meet[i]] = -1;
        w->dist[1][w->meet[i]] = -1;
    }
    w->nmeet = 0;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

#define DEG(g, v) ((g)->row_ptr[(v) + 1] - (g)->row_ptr[(v)])

/* sigma of vertex v on one side: sum over neighbours at depth dep, taken in
 * ascending CSR position.  Integer mode flags overflow. */
static uint64_t pull_int(const orc_graph *g, orc_ws *w, int side, int32_t v, int32_t dep, int *ovf)
{
    uint64_t acc = 0;
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
        int32_t u = g->col_idx[e];
        if (w->dist[side][u] == dep) {
            if (__builtin_add_overflow(acc, w->isig[side][u], &acc)) *ovf = 1;
        }
    }
    return acc;
}

static double pull_fp(const orc_graph *g, orc_ws *w, int side, int32_t v, int32_t dep)
{
    double acc = 0.0;
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
        int32_t u = g->col_idx[e];
        if (w->dist[side][u] == dep) acc = acc + w->fsig[side][u];
    }
    return acc;
}

/* sigma for every vertex of layers 1 .. upto of one side (the layers that
 * were expanded).  Returns 1 on integer overflow. */
static int sigma_layers_int(const orc_graph *g, orc_ws *w, int side, int32_t upto)
{
    int ovf = 0;
    w->isig[side][w->verts[side][0]] = 1;
    for (int32_t j = 1; j <= upto; ++j)
        for (int64_t i = w->loff[side][j]; i < w->loff[side][j + 1]; ++i) {
            int32_t v = w->verts[side][i];
            w->isig[side][v] = pull_int(g, w, side, v, j - 1, &ovf);
        }
    return ovf;
}

static void sigma_layers_fp(const orc_graph *g, orc_ws *w, int side, int32_t upto)
{
    const double BIG = 0x1p400, SHRINK = 0x1p-400;
    w->fsig[side][w->verts[side][0]] = 1.0;
    for (int32_t j = 1; j <= upto; ++j) {
        double mx = 0.0;
        for (int64_t i = w->loff[side][j]; i < w->loff[side][j + 1]; ++i) {
            int32_t v = w->verts[side][i];
            double x = pull_fp(g, w, side, v, j - 1);
            w->fsig[side][v] = x;
            if (x > mx) mx = x;
        }
        w->lscaled[side][j] = 0;
        if (mx > BIG) {
            for (int64_t i = w->loff[side][j]; i < w->loff[side][j + 1]; ++i)
                w->fsig[side][w->verts[side][i]] *= SHRINK;
            w->lscaled[side][j] = 1;
        }
    }
}

/* One predecessor pick while walking back towards the root of `side`. */
static int32_t pick_pred_int(const orc_graph *g, orc_ws *w, int side, int32_t v, int32_t dep, uint64_t u)
{
    uint64_t total = 0;
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
        int32_t x = g->col_idx[e];
        if (w->dist[side][x] == dep) total += w->isig[side][x];
    }
    uint64_t r = mulhi64(u, total);
    uint64_t pre = 0;
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
        int32_t x = g->col_idx[e];
        if (w->dist[side][x] == dep) {
            pre += w->isig[side][x];
            if (pre > r) return x;
        }
    }
    return -1; /* unreachable: pre reaches total > r */
}

static double unit53(uint64_t u) { return (double)(u >> 11) * 0x1p-53; }

static int32_t pick_pred_fp(const orc_graph *g, orc_ws *w, int side, int32_t v, int32_t dep, uint64_t u)
{
    double total = 0.0;
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
        int32_t x = g->col_idx[e];
        if (w->dist[side][x] == dep) total = total + w->fsig[side][x];
    }
    double r = unit53(u) * total;
    double pre = 0.0;
    int32_t last_nz = -1;
    for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
        int32_t x = g->col_idx[e];
        if (w->dist[side][x] == dep) {
            double a = w->fsig[side][x];
            pre = pre + a;
            if (a != 0.0) last_nz = x;
            if (pre > r) return x;
        }
    }
    return last_nz;
}

/* Number of layers among 1 .. upto of one side that were rescaled in FP mode. */
static int32_t scaled_layers(const orc_graph *g, orc_ws *w, int side, int32_t upto)
{
    (void)g;
    int32_t m = 0;
    for (int32_t j = 1; j <= upto; ++j) m += w->lscaled[side][j];
    return m;
}

static int sample_pair_given(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream,
                             uint64_t sample, int sigma_mode, int32_t s, int32_t t,
                             orc_sample_info *info);

int orc_sample(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream, uint64_t sample,
               int sigma_mode, orc_sample_info *info)
{
    int32_t s, t;
    orc_pair(seed, stream, sample, g->n, &s, &t);
    return sample_pair_given(g, w, seed, stream, sample, sigma_mode, s, t, info);
}

/* The same sampling step for a given pair (s, t): used by the tests that
 * check the path distribution of one pair.  Draws 2, 3, ... of the sample
 * are consumed exactly as in orc_sample. */
int orc_sample_fixed(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream, uint64_t sample,
                     int sigma_mode, int32_t s, int32_t t, int32_t *path_out, orc_sample_info *info)
{
    int rc = sample_pair_given(g, w, seed, stream, sample, sigma_mode, s, t, info);
    if (rc != ORC_OK) return rc;
    memcpy(path_out, w->path, sizeof(int32_t) * ((size_t)info->d + 1));
    return ORC_OK;
}

static int sample_pair_given(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream,
                             uint64_t sample, int sigma_mode, int32_t s, int32_t t,
                             orc_sample_info *info)
{
    int32_t root[2] = {s, t};
    memset(info, 0, sizeof(*info));
    if (s < 0 || t < 0 || s >= g->n || t >= g->n || s == t) return ORC_EINVAL;
    info->s = root[0];
    info->t = root[1];

    for (int side = 0; side < 2; ++side) {
        w->verts[side][0] = root[side];
        w->dist[side][root[side]] = 0;
        w->loff[side][0] = 0;
        w->loff[side][1] = 1;
        w->nlayers[side] = 1;
    }
    w->nmeet = 0;

    /* Balanced bidirectional BFS: grow the side whose newest layer has the
     * smaller degree sum (ties: the s side); each step adds a whole layer. */
    int X = 0;
    int64_t edges = 0;
    for (;;) {
        int64_t sum[2];
        for (int side = 0; side < 2; ++side) {
            sum[side] = 0;
            int32_t j = w->nlayers[side] - 1;
            for (int64_t i = w->loff[side][j]; i < w->loff[side][j + 1]; ++i)
                sum[side] += DEG(g, w->verts[side][i]);
        }
        X = (sum[0] <= sum[1]) ? 0 : 1;
        int Y = 1 - X;
        int32_t k = w->nlayers[X] - 1;
        edges += sum[X];
        info->steps += 1;
        int64_t lo = w->loff[X][k], hi = w->loff[X][k + 1];
        int64_t tail = hi;
        for (int64_t i = lo; i < hi; ++i) {
            int32_t u = w->verts[X][i];
            for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                int32_t x = g->col_idx[e];
                if (w->dist[X][x] >= 0) continue;
                w->dist[X][x] = k + 1;
                if (w->dist[Y][x] >= 0) {
                    w->meet[w->nmeet++] = x;       /* met the other side */
                } else {
                    w->verts[X][tail++] = x;
                }
            }
        }
        /* The new layer is recorded even on the meeting step (so that the
         * reset finds it); the meet vertices themselves are listed apart. */
        w->loff[X][k + 2] = tail;
        w->nlayers[X] = k + 2;
        if (w->nmeet > 0) break;
        if (tail == hi) {                          /* other side unreachable */
            ws_reset(w);
            return ORC_EDISCONNECTED;
        }
    }
    int Y = 1 - X;
    int32_t kX = w->nlayers[X] - 2;     /* the layer expanded in the last step */
    int32_t kY = w->nlayers[Y] - 1;     /* the meet set lies in this layer of Y */
    int32_t d = kX + 1 + kY;
    info->d = d;
    info->edges = edges;
    info->meet_size = w->nmeet;
    info->side = X;
    info->visited = (int32_t)(w->loff[0][w->nlayers[0]] + w->loff[1][w->nlayers[1]] + w->nmeet);
    qsort(w->meet, (size_t)w->nmeet, sizeof(int32_t), cmp_i32);

    /* Sigma: every expanded layer of both sides, then the meet set. */
    int fp = (sigma_mode == ORC_SIGMA_FP);
    uint64_t isX = 0, isY = 0, ist = 0;
    if (!fp) {
        int ovf = sigma_layers_int(g, w, X, kX);
        ovf |= sigma_layers_int(g, w, Y, kY - 1);
        for (int32_t i = 0; i < w->nmeet && !ovf; ++i) {
            int32_t x = w->meet[i];
            isX = pull_int(g, w, X, x, kX, &ovf);
            isY = (kY == 0) ? 1 : pull_int(g, w, Y, x, kY - 1, &ovf);
            uint64_t a;
            if (__builtin_mul_overflow(isX, isY, &a)) ovf = 1;
            if (__builtin_add_overflow(ist, a, &ist)) ovf = 1;
        }
        if (ovf) fp = 1;
    }
    info->fp_mode = fp;
    if (!fp) { info->sigma_st_int = ist; info->sigma_st = (double)ist; }

    /* Meet vertex: first in ascending id whose inclusive prefix exceeds
     * the draw scaled to sigma_st. */
    uint64_t u2 = orc_draw(seed, stream, sample, 2);
    int32_t wv = -1;
    if (!fp) {
        uint64_t r = mulhi64(u2, ist);
        uint64_t pre = 0;
        for (int32_t i = 0; i < w->nmeet; ++i) {
            int32_t x = w->meet[i];
            int ovf = 0;
            uint64_t a = pull_int(g, w, X, x, kX, &ovf) *
                         ((kY == 0) ? 1 : pull_int(g, w, Y, x, kY - 1, &ovf));
            pre += a;
            if (pre > r) { wv = x; break; }
        }
    } else {
        sigma_layers_fp(g, w, X, kX);
        sigma_layers_fp(g, w, Y, kY - 1);
        double tot = 0.0;
        double *wt = (double *)malloc(sizeof(double) * (size_t)w->nmeet);
        for (int32_t i = 0; i < w->nmeet; ++i) {
            int32_t x = w->meet[i];
            double sx = pull_fp(g, w, X, x, kX);
            double sy = (kY == 0) ? 1.0 : pull_fp(g, w, Y, x, kY - 1);
            wt[i] = sx * sy;
            tot = tot + wt[i];
        }
        info->sigma_st = tot;
        info->sigma_exp = 400 * (scaled_layers(g, w, X, kX) + scaled_layers(g, w, Y, kY - 1));
        double r = unit53(u2) * tot;
        double pre = 0.0;
        for (int32_t i = 0; i < w->nmeet; ++i) {
            pre = pre + wt[i];
            if (wt[i] != 0.0) wv = w->meet[i];
            if (pre > r) { wv = w->meet[i]; break; }
        }
        free(wt);
    }
    info->w = wv;

    /* Depths of the meet vertex from s and from t. */
    int32_t dep[2];
    dep[X] = kX + 1;
    dep[Y] = kY;

    /* Walk back from w to s, then from w to t; one draw per pick. */
    uint64_t j = 3;
    int32_t *path = w->path;
    path[dep[0]] = wv;
    for (int side = 0; side < 2; ++side) {
        int32_t v = wv;
        for (int32_t l = dep[side]; l >= 2; --l) {
            uint64_t u = orc_draw(seed, stream, sample, j++);
            int32_t p = fp ? pick_pred_fp(g, w, side, v, l - 1, u)
                           : pick_pred_int(g, w, side, v, l - 1, u);
            /* side 0 walks towards s = path[0], side 1 towards t = path[d] */
            path[side == 0 ? (l - 1) : (d - (l - 1))] = p;
            v = p;
        }
    }
    path[0] = root[0];
    path[d] = root[1];
    info->draws = j;
    ws_reset(w);
    return ORC_OK;
}

int orc_sample_path(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream, uint64_t sample,
                    int sigma_mode, int32_t *path_out, orc_sample_info *info)
{
    int rc = orc_sample(g, w, seed, stream, sample, sigma_mode, info);
    if (rc != ORC_OK) return rc;
    memcpy(path_out, w->path, sizeof(int32_t) * ((size_t)info->d + 1));
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Stop rule (Sec. III-A): per vertex f(b~, delta_L, omega, tau) and     */
/* g(b~, delta_U, omega, tau), both below eps for every vertex.  The     */
/* formulas are KADABRA's Bernstein-type bounds with L = ln(1/delta):    */
/*   f = L/tau * ((1/3 - omega/tau) + sqrt((1/3 - omega/tau)^2 + 2 b~ omega / L))
 *   g = L/tau * ((1/3 + omega/tau) + sqrt((1/3 + omega/tau)^2 + 2 b~ omega / L))
 * clamped to b~ and 1 - b~ (betweenness lies in [0, 1]).                */
/* ------------------------------------------------------------------ */

double orc_f(double bt, double L, double omega, double tau)
{
    double a = (1.0 / 3.0) - omega / tau;
    double q = a * a + ((2.0 * bt) * omega) / L;
    double f = (L / tau) * (a + sqrt(q));
    return f < bt ? f : bt;
}

double orc_g(double bt, double L, double omega, double tau)
{
    double a = (1.0 / 3.0) + omega / tau;
    double q = a * a + ((2.0 * bt) * omega) / L;
    double g = (L / tau) * (a + sqrt(q));
    double cap = 1.0 - bt;
    return g < cap ? g : cap;
}

/* omega = c / eps^2 * (floor(log2(VD - 2)) + 1 + ln(2 / delta)), c = 1/2,
 * VD = vertex diameter; the log term is 0 when VD - 2 < 1. */
double orc_omega(int64_t vd, double eps, double delta)
{
    double lg = 0.0;
    if (vd - 2 >= 1) {
        int64_t x = vd - 2, fl = 0;
        while (x > 1) { x >>= 1; ++fl; }
        lg = (double)fl;
    }
    return 0.5 / (eps * eps) * (lg + 1.0 + log(2.0 / delta));
}

/* ------------------------------------------------------------------ */
/* Epoch loop: samples kE .. min((k+1)E, ceil(omega)) - 1 form epoch k;  */
/* after each epoch the counters are summed and the rule is checked on  */
/* exactly those samples (a consistent snapshot, Sec. III-B).           */
/* ------------------------------------------------------------------ */

int orc_check(int32_t n, const uint32_t *c, uint64_t tau, double omega, double eps,
              const double *LL, const double *LU, orc_check_info *ci)
{
    int all = 1;
    double mf = 0.0, mg = 0.0, mm = INFINITY;
    for (int32_t v = 0; v < n; ++v) {
        double bt = (double)c[v] / (double)tau;
        double f = orc_f(bt, LL[v], omega, (double)tau);
        double gg = orc_g(bt, LU[v], omega, (double)tau);
        if (!(f < eps && gg < eps)) all = 0;
        if (f > mf) mf = f;
        if (gg > mg) mg = gg;
        double mar = eps - (f > gg ? f : gg);
        if (mar < 0) mar = -mar;
        if (mar < mm) mm = mar;
    }
    if (ci) { ci->max_f = mf; ci->max_g = mg; ci->min_abs_margin = mm; }
    return all;
}

int orc_run(const orc_graph *g, const orc_run_opts *o, const double *LL, const double *LU,
            uint32_t *c, orc_run_result *res, orc_check_info *per_epoch, int32_t max_epochs)
{
    const int32_t n = g->n;
    uint64_t cap = (uint64_t)ceil(o->omega);
    orc_ws *w = orc_ws_create(n);
    int32_t *path = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t k = o->start_epoch;
    if (k == 0) memset(c, 0, sizeof(uint32_t) * (size_t)n);
    int64_t edges = 0;
    uint64_t tau = 0;
    int reason = 0;
    for (;; ++k) {
        uint64_t lo = (uint64_t)k * o->epoch;
        uint64_t hi = lo + o->epoch;
        if (hi > cap) hi = cap;
        for (uint64_t i = lo; i < hi; ++i) {
            orc_sample_info info;
            int rc = orc_sample_path(g, w, o->seed, o->stream, i, o->sigma_mode, path, &info);
            if (rc != ORC_OK) { free(path); orc_ws_free(w); return rc; }
            for (int32_t q = 1; q < info.d; ++q) c[path[q]] += 1;
            edges += info.edges;
        }
        tau = hi;
        orc_check_info ci;
        int ok = orc_check(n, c, tau, o->omega, o->eps, LL, LU, &ci);
        if (per_epoch && k < max_epochs) per_epoch[k] = ci;
        if (ok) { reason = ORC_STOP_COND; break; }
        if (tau >= cap) { reason = ORC_STOP_OMEGA; break; }
        if (o->stop_after_epochs > 0 && k + 1 >= o->start_epoch + o->stop_after_epochs) {
            reason = ORC_STOP_PAUSED;
            break;
        }
    }
    res->tau = tau;
    res->epochs = k + 1;
    res->reason = reason;
    res->edges = edges;
    free(path);
    orc_ws_free(w);
    return ORC_OK;
}

/* Non-adaptive samples on any stream: counters of samples [first, first+count). */
int orc_count(const orc_graph *g, uint64_t seed, uint64_t stream, uint64_t first, uint64_t count,
              int sigma_mode, uint32_t *c, int64_t *edges_out)
{
    orc_ws *w = orc_ws_create(g->n);
    int32_t *path = (int32_t *)malloc(sizeof(int32_t) * ((size_t)g->n + 1));
    int64_t edges = 0;
    for (uint64_t i = first; i < first + count; ++i) {
        orc_sample_info info;
        int rc = orc_sample_path(g, w, seed, stream, i, sigma_mode, path, &info);
        if (rc != ORC_OK) { free(path); orc_ws_free(w); return rc; }
        for (int32_t q = 1; q < info.d; ++q) c[path[q]] += 1;
        edges += info.edges;
    }
    if (edges_out) *edges_out = edges;
    free(path);
    orc_ws_free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Calibration of delta_L, delta_U (Sec. III-A, phase 2).  The paper     */
/* leaves the heuristic out; reading: tau0 = ceil(omega / 100) samples on */
/* stream 1 give b' = c' / tau0; delta(v) = (1 - beta) exp(-C / b'(v)) +  */
/* beta delta / (4n), with C the smallest value (by bisection) at which  */
/* the sum over vertices with c' > 0 of exp(-C / b'(v)) stays below       */
/* delta / 4 (shrunk by a 1e-9 relative safety margin).  Hence the sum of */
/* delta_L + delta_U stays below delta / 2.                              */
/* ------------------------------------------------------------------ */

static double alloc_sum(int32_t n, const double *prior, double C)
{
    double s = 0.0;
    for (int32_t v = 0; v < n; ++v)
        if (prior[v] > 0.0) s = s + exp(-C / prior[v]);
    return s;
}

double orc_alloc_constant(int32_t n, const double *prior, double delta)
{
    const double target = 0.25 * delta * (1.0 - 1e-9);
    int64_t K = 0;
    for (int32_t v = 0; v < n; ++v) if (prior[v] > 0.0) ++K;
    if (K == 0) return 0.0;
    double lo = 0.0, hi = log((double)K / target);
    if (hi < 0.0) hi = 0.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;   /* interval cannot shrink further */
        if (alloc_sum(n, prior, mid) <= target) hi = mid; else lo = mid;
    }
    return hi;
}

void orc_alloc_delta(int32_t n, const double *prior, double C, double delta, double beta,
                     double *LL, double *LU)
{
    const double floor_d = beta * delta / (4.0 * (double)n);
    for (int32_t v = 0; v < n; ++v) {
        double dv = floor_d;
        if (prior[v] > 0.0) dv = (1.0 - beta) * exp(-C / prior[v]) + floor_d;
        LL[v] = -log(dv);
        LU[v] = LL[v];
    }
}

int orc_count_mt(const orc_graph *g, uint64_t seed, uint64_t stream, uint64_t first, uint64_t count,
                 int sigma_mode, uint32_t *c, int64_t *edges_out, int nthreads);

int orc_calibrate_mt(const orc_graph *g, uint64_t seed, double omega, double delta, int sigma_mode,
                     uint32_t *cprime, double *C_out, double *LL, double *LU, int nthreads)
{
    const int32_t n = g->n;
    uint64_t tau0 = (uint64_t)ceil(omega / 100.0);
    memset(cprime, 0, sizeof(uint32_t) * (size_t)n);
    int rc = nthreads > 1 ? orc_count_mt(g, seed, ORC_STREAM_CALIB, 0, tau0, sigma_mode, cprime, NULL, nthreads)
                          : orc_count(g, seed, ORC_STREAM_CALIB, 0, tau0, sigma_mode, cprime, NULL);
    if (rc != ORC_OK) return rc;
    double *prior = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) prior[v] = (double)cprime[v] / (double)tau0;
    double C = orc_alloc_constant(n, prior, delta);
    orc_alloc_delta(n, prior, C, delta, 1e-3, LL, LU);
    free(prior);
    *C_out = C;
    return ORC_OK;
}

int orc_calibrate(const orc_graph *g, uint64_t seed, double omega, double delta, int sigma_mode,
                  uint32_t *cprime, double *C_out, double *LL, double *LU)
{
    return orc_calibrate_mt(g, seed, omega, delta, sigma_mode, cprime, C_out, LL, LU, 1);
}

/* ------------------------------------------------------------------ */
/* Vertex diameter bracket for omega: BFS from the vertex of highest     */
/* degree r, then from its farthest vertex a, then from a's farthest b;  */
/* eccentricities give LB = max(ecc a, ecc b) <= D <= UB = 2 min(ecc).   */
/* ------------------------------------------------------------------ */

static int32_t bfs_ecc(const orc_graph *g, int32_t src, int32_t *dist, int32_t *queue, int32_t *far)
{
    for (int32_t v = 0; v < g->n; ++v) dist[v] = -1;
    int64_t head = 0, tail = 0;
    queue[tail++] = src;
    dist[src] = 0;
    int32_t ecc = 0, fv = src;
    while (head < tail) {
        int32_t u = queue[head++];
        if (dist[u] > ecc || (dist[u] == ecc && u < fv)) { ecc = dist[u]; fv = u; }
        for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
            int32_t x = g->col_idx[e];
            if (dist[x] < 0) { dist[x] = dist[u] + 1; queue[tail++] = x; }
        }
    }
    *far = fv;
    return ecc;
}

void orc_vd_bracket(const orc_graph *g, int64_t *vd_lo, int64_t *vd_hi)
{
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t r = 0;
    for (int32_t v = 1; v < g->n; ++v) if (DEG(g, v) > DEG(g, r)) r = v;
    int32_t a, b, c;
    int32_t er = bfs_ecc(g, r, dist, queue, &a);
    int32_t ea = bfs_ecc(g, a, dist, queue, &b);
    int32_t eb = bfs_ecc(g, b, dist, queue, &c);
    int32_t lb = ea > eb ? ea : eb;
    int32_t m = er < ea ? er : ea;
    if (eb < m) m = eb;
    *vd_lo = (int64_t)lb + 1;
    *vd_hi = 2 * (int64_t)m + 1;
    free(dist);
    free(queue);
}

/* Eccentricity of v (BFS). */
int32_t orc_eccentricity(const orc_graph *g, int32_t v)
{
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t far;
    int32_t e = bfs_ecc(g, v, dist, queue, &far);
    free(dist);
    free(queue);
    return e;
}

/* Exact vertex diameter: one BFS per vertex (the definition; small graphs). */
int64_t orc_exact_vd(const orc_graph *g)
{
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t best = 0, far;
    for (int32_t v = 0; v < g->n; ++v) {
        int32_t e = bfs_ecc(g, v, dist, queue, &far);
        if (e > best) best = e;
    }
    free(dist);
    free(queue);
    return (int64_t)best + 1;
}

/* omega from the bracket: exact when both ends give the same floor(log2(VD-2)),
 * otherwise the (valid, larger) value of the upper end. */
double orc_omega_bracket(int64_t vd_lo, int64_t vd_hi, double eps, double delta)
{
    double lo = orc_omega(vd_lo, eps, delta), hi = orc_omega(vd_hi, eps, delta);
    return lo == hi ? lo : hi;
}

/* ------------------------------------------------------------------ */
/* Exact betweenness by Brandes' algorithm (Sec. I / II), normalised by  */
/* n(n-1) over ordered pairs.                                            */
/* ------------------------------------------------------------------ */

void orc_brandes(const orc_graph *g, double *bc)
{
    const int32_t n = g->n;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *sig = (double *)malloc(sizeof(double) * (size_t)n);
    double *dep = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;
    for (int32_t s = 0; s < n; ++s) {
        for (int32_t v = 0; v < n; ++v) { dist[v] = -1; sig[v] = 0.0; dep[v] = 0.0; }
        int64_t head = 0, tail = 0;
        order[tail++] = s;
        dist[s] = 0;
        sig[s] = 1.0;
        while (head < tail) {
            int32_t u = order[head++];
            for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                int32_t x = g->col_idx[e];
                if (dist[x] < 0) { dist[x] = dist[u] + 1; order[tail++] = x; }
                if (dist[x] == dist[u] + 1) sig[x] += sig[u];
            }
        }
        for (int64_t i = tail - 1; i >= 0; --i) {
            int32_t x = order[i];
            for (int64_t e = g->row_ptr[x]; e < g->row_ptr[x + 1]; ++e) {
                int32_t u = g->col_idx[e];
                if (dist[u] == dist[x] - 1) dep[u] += sig[u] / sig[x] * (1.0 + dep[x]);
            }
            if (x != s) bc[x] += dep[x];
        }
    }
    double norm = (double)n * (double)(n - 1);
    for (int32_t v = 0; v < n; ++v) bc[v] /= norm;
    free(dist); free(order); free(sig); free(dep);
}

/* ------------------------------------------------------------------ */
/* Learned prior: per-vertex features and the 3-64-64-1 ReLU MLP in FP64 */
/* (not in the paper; a learned replacement for the calibration phase).  */
/* ------------------------------------------------------------------ */

void orc_features(const orc_graph *g, double *x /* n x 3, row-major */)
{
    for (int32_t v = 0; v < g->n; ++v) {
        int64_t dv = DEG(g, v);
        double acc = 0.0;
        double sumdeg = 0.0;
        for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            int32_t u = g->col_idx[e];
            double du = (double)DEG(g, u);
            acc += log1p(du);
            sumdeg += du;
        }
        x[3 * v + 0] = log1p((double)dv);
        x[3 * v + 1] = dv > 0 ? acc / (double)dv : 0.0;
        x[3 * v + 2] = log1p(sumdeg);
    }
}

/* Parameter layout (4481 values): W1[64][3], b1[64], W2[64][64], b2[64],
 * W3[64], b3.  Row-major, out x in. */
/* Learned prior from the network output y = ln(b + 1/omega) (the
 * regression target): b = e^y - 1/omega, clamped to [0, 1], the range of
 * betweenness (Sec. I); a non-finite b is left as it is. */
void orc_prior_from_output(int64_t n, const double *y, double omega, double *prior)
{
    for (int64_t v = 0; v < n; ++v) {
        double b = exp(y[v]) - 1.0 / omega;
        if (isfinite(b)) {   /* a non-finite output is left as it is */
            if (b < 0.0) b = 0.0;
            if (b > 1.0) b = 1.0;
        }
        prior[v] = b;
    }
}

void orc_mlp_forward(const double *p, const double *x, int64_t rows, double *y)
{
    const double *W1 = p, *b1 = p + 192, *W2 = p + 256, *b2 = p + 4352, *W3 = p + 4416, *b3 = p + 4480;
    double h1[64], h2[64];
    for (int64_t r = 0; r < rows; ++r) {
        const double *xr = x + 3 * r;
        for (int i = 0; i < 64; ++i) {
            double a = b1[i];
            for (int j = 0; j < 3; ++j) a += W1[3 * i + j] * xr[j];
            h1[i] = a > 0 ? a : 0;
        }
        for (int i = 0; i < 64; ++i) {
            double a = b2[i];
            for (int j = 0; j < 64; ++j) a += W2[64 * i + j] * h1[j];
            h2[i] = a > 0 ? a : 0;
        }
        double a = b3[0];
        for (int j = 0; j < 64; ++j) a += W3[j] * h2[j];
        y[r] = a;
    }
}

/* Mean squared error over the rows and its gradient w.r.t. every parameter. */
double orc_mlp_loss_grad(const double *p, const double *x, const double *target, int64_t rows,
                         double *grad)
{
    const double *W1 = p, *b1 = p + 192, *W2 = p + 256, *b2 = p + 4352, *W3 = p + 4416, *b3 = p + 4480;
    double *gW1 = grad, *gb1 = grad + 192, *gW2 = grad + 256, *gb2 = grad + 4352, *gW3 = grad + 4416,
           *gb3 = grad + 4480;
    memset(grad, 0, sizeof(double) * ORC_MLP_PARAMS);
    double loss = 0.0;
    double z1[64], h1[64], z2[64], h2[64], d2[64], d1[64];
    for (int64_t r = 0; r < rows; ++r) {
        const double *xr = x + 3 * r;
        for (int i = 0; i < 64; ++i) {
            double a = b1[i];
            for (int j = 0; j < 3; ++j) a += W1[3 * i + j] * xr[j];
            z1[i] = a; h1[i] = a > 0 ? a : 0;
        }
        for (int i = 0; i < 64; ++i) {
            double a = b2[i];
            for (int j = 0; j < 64; ++j) a += W2[64 * i + j] * h1[j];
            z2[i] = a; h2[i] = a > 0 ? a : 0;
        }
        double yv = b3[0];
        for (int j = 0; j < 64; ++j) yv += W3[j] * h2[j];
        double diff = yv - target[r];
        loss += diff * diff;
        double dy = 2.0 * diff / (double)rows;
        gb3[0] += dy;
        for (int j = 0; j < 64; ++j) {
            gW3[j] += dy * h2[j];
            d2[j] = z2[j] > 0 ? dy * W3[j] : 0.0;
        }
        for (int i = 0; i < 64; ++i) {
            gb2[i] += d2[i];
            for (int j = 0; j < 64; ++j) gW2[64 * i + j] += d2[i] * h1[j];
        }
        for (int j = 0; j < 64; ++j) {
            double a = 0.0;
            for (int i = 0; i < 64; ++i) a += W2[64 * i + j] * d2[i];
            d1[j] = z1[j] > 0 ? a : 0.0;
        }
        for (int i = 0; i < 64; ++i) {
            gb1[i] += d1[i];
            for (int j = 0; j < 3; ++j) gW1[3 * i + j] += d1[i] * xr[j];
        }
    }
    return loss / (double)rows;
}

/* One Adam step (Kingma & Ba): bias-corrected first and second moments. */
void orc_adam_step(double *p, const double *grad, double *m, double *v, int64_t count, int64_t step,
                   double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < count; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------ */
/* -ln(delta) per vertex: the stop rule takes L = ln(1/delta_L) and      */
/* ln(1/delta_U) (Sec. III-A); the oracle computes them itself from the  */
/* delta arrays a run is given.                                          */
/* ------------------------------------------------------------------ */

void orc_neglog(int32_t n, const double *delta, double *L)
{
    for (int32_t v = 0; v < n; ++v) L[v] = -log(delta[v]);
}

/* ------------------------------------------------------------------ */
/* Threaded runner.  The shared-memory layout of the sampling phase      */
/* (Sec. IV-A): every thread samples into a state frame of its own, and  */
/* the frames are summed into the counters at each epoch boundary (the   */
/* aggregation of Alg. 1 / Alg. 2, here without MPI).  The samples of an */
/* epoch are split into contiguous index slices, one per thread.  The    */
/* counters are integer sums, so the result is the single-threaded       */
/* run's, bit for bit; the check's maxima, minimum and AND do not depend */
/* on the order either.                                                  */
/* ------------------------------------------------------------------ */

typedef struct {
    const orc_graph *g;
    uint64_t seed, stream;
    int sigma_mode;
    uint64_t lo, hi;          /* sample indices [lo, hi) of this thread     */
    uint32_t *frame;          /* thread-local state frame, n counters       */
    orc_ws *ws;
    int32_t *path;
    int64_t edges;
    int rc;
    /* frame sum and check over vertices [v0, v1) */
    int32_t v0, v1;
    uint32_t *const *frames;
    int nframes;
    uint32_t *c;
    uint64_t tau;
    double omega, eps;
    const double *LL, *LU;
    int all;
    orc_check_info ci;
} mt_job;

static void *mt_sample(void *arg)
{
    mt_job *j = (mt_job *)arg;
    j->rc = ORC_OK;
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        orc_sample_info info;
        int rc = orc_sample_path(j->g, j->ws, j->seed, j->stream, i, j->sigma_mode, j->path, &info);
        if (rc != ORC_OK) { j->rc = rc; return NULL; }
        for (int32_t q = 1; q < info.d; ++q) j->frame[j->path[q]] += 1;
        j->edges += info.edges;
    }
    return NULL;
}

/* c[v] += sum of the frames at v, frames cleared; then the stop rule on
 * the slice's vertices when LL is set. */
static void *mt_merge_check(void *arg)
{
    mt_job *j = (mt_job *)arg;
    for (int f = 0; f < j->nframes; ++f) {
        uint32_t *fr = j->frames[f];
        for (int32_t v = j->v0; v < j->v1; ++v) {
            j->c[v] += fr[v];
            fr[v] = 0;
        }
    }
    if (j->LL) {
        j->all = orc_check(j->v1 - j->v0, j->c + j->v0, j->tau, j->omega, j->eps, j->LL + j->v0,
                           j->LU + j->v0, &j->ci);
    }
    return NULL;
}

static int mt_for(int nthreads, mt_job *jobs, void *(*fn)(void *))
{
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int i = 1; i < nthreads; ++i) {
        if (pthread_create(&th[i], NULL, fn, &jobs[i]) != 0) break;
        started = i;
    }
    /* thread 0's share runs here; shares whose thread did not start too */
    fn(&jobs[0]);
    for (int i = started + 1; i < nthreads; ++i) fn(&jobs[i]);
    for (int i = 1; i <= started; ++i) pthread_join(th[i], NULL);
    free(th);
    return ORC_OK;
}

typedef struct {
    int nthreads;
    mt_job *jobs;
    uint32_t **frames;
} mt_pool;

static void mt_pool_init(mt_pool *p, const orc_graph *g, uint64_t seed, uint64_t stream, int sigma_mode,
                         int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    p->nthreads = nthreads;
    p->jobs = (mt_job *)calloc((size_t)nthreads, sizeof(mt_job));
    p->frames = (uint32_t **)malloc(sizeof(uint32_t *) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i) {
        mt_job *j = &p->jobs[i];
        j->g = g;
        j->seed = seed;
        j->stream = stream;
        j->sigma_mode = sigma_mode;
        j->frame = (uint32_t *)calloc((size_t)g->n, sizeof(uint32_t));
        j->ws = orc_ws_create(g->n);
        j->path = (int32_t *)malloc(sizeof(int32_t) * ((size_t)g->n + 1));
        p->frames[i] = j->frame;
    }
}

static void mt_pool_free(mt_pool *p)
{
    for (int i = 0; i < p->nthreads; ++i) {
        free(p->jobs[i].frame);
        orc_ws_free(p->jobs[i].ws);
        free(p->jobs[i].path);
    }
    free(p->jobs);
    free(p->frames);
}

/* Samples [lo, hi) on the pool's threads, frames summed into c; when LL is
 * set, the stop rule at tau is evaluated (returns 1 when it holds). */
static int mt_epoch(mt_pool *p, uint64_t lo, uint64_t hi, uint32_t *c, int64_t *edges, uint64_t tau,
                    double omega, double eps, const double *LL, const double *LU, orc_check_info *ci,
                    int *rc_out)
{
    const int T = p->nthreads;
    const int32_t n = p->jobs[0].g->n;
    const uint64_t cnt = hi - lo;
    for (int i = 0; i < T; ++i) {
        mt_job *j = &p->jobs[i];
        j->lo = lo + cnt * (uint64_t)i / (uint64_t)T;
        j->hi = lo + cnt * (uint64_t)(i + 1) / (uint64_t)T;
        j->edges = 0;
    }
    mt_for(T, p->jobs, mt_sample);
    *rc_out = ORC_OK;
    for (int i = 0; i < T; ++i) {
        if (p->jobs[i].rc != ORC_OK) *rc_out = p->jobs[i].rc;
        *edges += p->jobs[i].edges;
    }
    for (int i = 0; i < T; ++i) {
        mt_job *j = &p->jobs[i];
        j->v0 = (int32_t)((int64_t)n * i / T);
        j->v1 = (int32_t)((int64_t)n * (i + 1) / T);
        j->frames = p->frames;
        j->nframes = T;
        j->c = c;
        j->tau = tau;
        j->omega = omega;
        j->eps = eps;
        j->LL = LL;
        j->LU = LU;
    }
    mt_for(T, p->jobs, mt_merge_check);
    if (!LL) return 0;
    int all = 1;
    double mf = 0.0, mg = 0.0, mm = INFINITY;
    for (int i = 0; i < T; ++i) {
        const mt_job *j = &p->jobs[i];
        if (j->v1 <= j->v0) continue;
        if (!j->all) all = 0;
        if (j->ci.max_f > mf) mf = j->ci.max_f;
        if (j->ci.max_g > mg) mg = j->ci.max_g;
        if (j->ci.min_abs_margin < mm) mm = j->ci.min_abs_margin;
    }
    if (ci) { ci->max_f = mf; ci->max_g = mg; ci->min_abs_margin = mm; }
    return all;
}

int orc_count_mt(const orc_graph *g, uint64_t seed, uint64_t stream, uint64_t first, uint64_t count,
                 int sigma_mode, uint32_t *c, int64_t *edges_out, int nthreads)
{
    mt_pool p;
    mt_pool_init(&p, g, seed, stream, sigma_mode, nthreads);
    int64_t edges = 0;
    int rc = ORC_OK;
    mt_epoch(&p, first, first + count, c, &edges, 0, 0.0, 0.0, NULL, NULL, NULL, &rc);
    mt_pool_free(&p);
    if (edges_out) *edges_out = edges;
    return rc;
}

/* orc_run with every epoch's samples split over nthreads threads. */
int orc_run_mt(const orc_graph *g, const orc_run_opts *o, const double *LL, const double *LU,
               uint32_t *c, orc_run_result *res, orc_check_info *per_epoch, int32_t max_epochs,
               int nthreads)
{
    const int32_t n = g->n;
    uint64_t cap = (uint64_t)ceil(o->omega);
    mt_pool p;
    mt_pool_init(&p, g, o->seed, o->stream, o->sigma_mode, nthreads);
    int32_t k = o->start_epoch;
    if (k == 0) memset(c, 0, sizeof(uint32_t) * (size_t)n);
    int64_t edges = 0;
    uint64_t tau = 0;
    int reason = 0;
    for (;; ++k) {
        uint64_t lo = (uint64_t)k * o->epoch;
        uint64_t hi = lo + o->epoch;
        if (hi > cap) hi = cap;
        orc_check_info ci;
        int rc = ORC_OK;
        int ok = mt_epoch(&p, lo, hi, c, &edges, hi, o->omega, o->eps, LL, LU, &ci, &rc);
        if (rc != ORC_OK) { mt_pool_free(&p); return rc; }
        tau = hi;
        if (per_epoch && k < max_epochs) per_epoch[k] = ci;
        if (ok) { reason = ORC_STOP_COND; break; }
        if (tau >= cap) { reason = ORC_STOP_OMEGA; break; }
        if (o->stop_after_epochs > 0 && k + 1 >= o->start_epoch + o->stop_after_epochs) {
            reason = ORC_STOP_PAUSED;
            break;
        }
    }
    res->tau = tau;
    res->epochs = k + 1;
    res->reason = reason;
    res->edges = edges;
    mt_pool_free(&p);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Training loop of the prior network (not in the paper).  Weights drawn */
/* uniformly in [-sqrt(6/fan_in), sqrt(6/fan_in)) (He), biases zero:     */
/* parameter i takes draw 0 of Philox sample i of stream 2.  Adam step j */
/* (counted over all epochs) takes `batch` rows drawn uniformly with     */
/* replacement: row b is floor(u rows / 2^64), u = draw b of sample      */
/* 2^32 + j of stream 2.  The step size halves every `halve_every`       */
/* epochs.  losses[e] = mean over epoch e's steps of the batch loss.     */
/* ------------------------------------------------------------------ */

static double orc_unit53(uint64_t u) { return (double)(u >> 11) * 0x1p-53; }

void orc_mlp_init(uint64_t seed, double *p)
{
    for (int i = 0; i < ORC_MLP_PARAMS; ++i) {
        double bound = 0.0;
        if (i < 192) bound = sqrt(6.0 / 3.0);                 /* W1 */
        else if (i >= 256 && i < 4352) bound = sqrt(6.0 / 64.0);   /* W2 */
        else if (i >= 4416 && i < 4480) bound = sqrt(6.0 / 64.0);  /* W3 */
        p[i] = bound > 0.0 ? (2.0 * orc_unit53(orc_draw(seed, 2, (uint64_t)i, 0)) - 1.0) * bound : 0.0;
    }
}

void orc_batch_rows(uint64_t seed, uint64_t step, int32_t batch, int64_t rows, int64_t *out)
{
    for (int32_t b = 0; b < batch; ++b)
        out[b] = (int64_t)mulhi64(orc_draw(seed, 2, (1ull << 32) + step, (uint64_t)b), (uint64_t)rows);
}

void orc_mlp_train(const double *x, const double *y, int64_t rows, int32_t epochs, int32_t batch, double lr,
                   int32_t halve_every, uint64_t seed, double *p, double *losses)
{
    double *grad = (double *)malloc(sizeof(double) * ORC_MLP_PARAMS);
    double *m = (double *)calloc(ORC_MLP_PARAMS, sizeof(double));
    double *v = (double *)calloc(ORC_MLP_PARAMS, sizeof(double));
    double *xb = (double *)malloc(sizeof(double) * 3 * (size_t)batch);
    double *yb = (double *)malloc(sizeof(double) * (size_t)batch);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)batch);
    orc_mlp_init(seed, p);
    const int64_t steps = (rows + batch - 1) / batch;
    uint64_t j = 0;
    for (int32_t e = 0; e < epochs; ++e) {
        const double lr_e = lr * pow(0.5, (double)(halve_every > 0 ? e / halve_every : 0));
        double sum = 0.0;
        for (int64_t s = 0; s < steps; ++s, ++j) {
            orc_batch_rows(seed, j, batch, rows, idx);
            for (int32_t b = 0; b < batch; ++b) {
                for (int k = 0; k < 3; ++k) xb[3 * b + k] = x[3 * idx[b] + k];
                yb[b] = y[idx[b]];
            }
            sum += orc_mlp_loss_grad(p, xb, yb, batch, grad);
            orc_adam_step(p, grad, m, v, ORC_MLP_PARAMS, (int64_t)j + 1, lr_e, 0.9, 0.999, 1e-8);
        }
        if (losses) losses[e] = sum / (double)steps;
    }
    free(grad); free(m); free(v); free(xb); free(yb); free(idx);
}
