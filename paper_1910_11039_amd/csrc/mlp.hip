// Learned prior for the delta allocation (not in the paper; the paper's
// calibration phase, Sec. III-A phase 2, picks delta_L/delta_U from a few
// samples, and any split with sum below delta is valid -- so a predicted
// prior may replace those samples without touching the guarantee).
//
//  * features of vertex v: ln(1 + deg v), mean over neighbours u of
//    ln(1 + deg u), ln(1 + sum over neighbours of deg u) -- one wave per
//    vertex, lanes stride the adjacency, FP64 inside, FP32 out;
//  * MLP 3 -> 64 -> 64 -> 1 with ReLU, FP32.  A workgroup of four waves
//    takes 64 rows at a time; the three dense 64x64 contractions (hidden
//    layer forward, its weight gradient, and the back-propagated signal)
//    run on the FP32 matrix cores (v_mfma_f32_16x16x4f32, one 16-row strip
//    per wave); the 3-wide input layer and the 64-wide output dot product
//    are plain FMAs.  Gradients are reduced per workgroup and then summed
//    over workgroups in a fixed order.
#include <math.h>

#include "kad_internal.h"
#include "philox.h"

namespace kad {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int TR = 64;          // rows per tile
constexpr int LD = 68;          // padded row stride in LDS (floats)
constexpr int NP = 4481;        // parameters
constexpr int PSTRIDE = NP + 1; // per-block partial: gradient then loss
constexpr int OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 256, OFF_B2 = 4352, OFF_W3 = 4416, OFF_B3 = 4480;

// ln(1 + deg u) and deg u (FP64) of a neighbour u: the 4-byte degree is
// gathered and the logarithm read from a table indexed by degree, lt[d] =
// ln(1 + d) for d = 0 .. max degree, filled once per pass.  The FP64
// logarithm is about 120 FP64 instructions, which over the 2 nnz entries
// of a large graph cost more than the whole gather; the table's hot part
// (the small degrees, and the few hubs' entries) stays in cache, and a
// 16-byte table per vertex would not.
__device__ __forceinline__ double2 logdeg(const DevGraph &g, const double *lt, int32_t u)
{
    const uint32_t d = g.deg[u];
    // (a degree of n or more, possible only with repeated entries, is
    // beyond the table)
    return make_double2(d < (uint32_t)g.n ? lt[d] : log1p((double)d), (double)d);
}

// The degree-run table in LDS.  Vertices are numbered by descending degree,
// so a vertex's degree is a step function of its id with one step per
// distinct degree (3 139 steps on R-MAT 26 against 32.8 M vertices).  The
// feature kernels hold the last `cnt` runs (the smallest degrees) in LDS:
// key[] the first vertex of each run (padded with INT32_MAX to a power of
// two, `half` is half of that), lg[] = ln(1 + d) and dg[] = d.  A neighbour
// u at or above key[0] is resolved by a binary search, which needs no global
// load; a neighbour below key[0] (a hub, only when the graph has more
// distinct degrees than the table holds) is gathered as above.  On R-MAT 26
// 28 % of the adjacency entries point at the 31.8 M vertices of degree
// under 256, scattered over a 131 MB degree array that misses L2; the
// search turns those into LDS reads.
constexpr int RUNCAP = 4096;      // runs held in LDS (16 B each)

struct RunArgs {
    const int32_t *start;   // run starts (global)
    const uint32_t *deg;    // run degrees (global)
    int32_t first;          // first run held in LDS
    int32_t cnt;            // runs held
    int32_t pow2;           // cnt rounded up to a power of two
};

struct RunLds {
    const double *lg;
    const int32_t *key;
    const uint32_t *dg;
    int32_t half;
};

size_t run_lds_bytes(int32_t cnt, int32_t pow2) { return 8 * (size_t)cnt + 4 * (size_t)pow2 + 4 * (size_t)cnt; }

// Fills the block's LDS table (every thread of the block must call this
// before any lookup; it ends with a barrier).  lt must hold ln(1 + d) for
// the degrees below n.
__device__ RunLds load_runs(const DevGraph &g, const double *lt, const RunArgs &r)
{
    extern __shared__ double s_runs[];
    double *lg = s_runs;
    int32_t *key = (int32_t *)(lg + r.cnt);
    uint32_t *dg = (uint32_t *)(key + r.pow2);
    for (int i = threadIdx.x; i < r.pow2; i += blockDim.x) {
        key[i] = i < r.cnt ? r.start[r.first + i] : INT32_MAX;
        if (i < r.cnt) {
            const uint32_t d = r.deg[r.first + i];
            dg[i] = d;
            lg[i] = d < (uint32_t)g.n ? lt[d] : log1p((double)d);
        }
    }
    __syncthreads();
    return RunLds{lg, key, dg, r.pow2 >> 1};
}

// (ln(1 + deg u), deg u) of B neighbours (u < 0: an empty position, 0).
// The B searches are interleaved step by step so that their LDS reads
// overlap.
template <int B>
__device__ __forceinline__ void run_lookup(const DevGraph &g, const double *lt, const RunLds &L,
                                           const int32_t (&u)[B], double2 (&p)[B])
{
    int k[B];
#pragma unroll
    for (int j = 0; j < B; ++j) k[j] = 0;
    for (int h = L.half; h > 0; h >>= 1) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int c = k[j] + h;
            if (L.key[c] <= u[j]) k[j] = c;
        }
    }
    const int32_t lo = L.key[0];
#pragma unroll
    for (int j = 0; j < B; ++j) {
        if (u[j] < 0) p[j] = make_double2(0.0, 0.0);
        else if (u[j] < lo) p[j] = logdeg(g, lt, u[j]);
        else p[j] = make_double2(L.lg[k[j]], (double)L.dg[k[j]]);
    }
}

// lt[d] = ln(1 + d) for d = 0 .. min(deg[0], n - 1) (vertex 0 has the
// largest degree in the internal numbering).
__global__ void k_logtab(DevGraph g, double *lt)
{
    const int64_t top = min((int64_t)g.deg[0], (int64_t)g.n - 1);
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d <= top;
         d += (int64_t)gridDim.x * blockDim.x)
        lt[d] = log1p((double)d);
}

constexpr int64_t FPIECE = 8192;   // rows longer than this are summed in pieces

__device__ __forceinline__ void write_features(float *out, int64_t v, double dv, double acc, double sd)
{
    out[3 * v + 0] = (float)log1p(dv);
    out[3 * v + 1] = (float)(dv > 0 ? acc / dv : 0.0);
    out[3 * v + 2] = (float)log1p(sd);
}

constexpr int64_t FSHORT = 32;     // rows up to this long: a thread per vertex

// Short rows (most vertices of a power-law graph): a thread per vertex, its
// entries eight at a time.
// (Vertices are numbered by descending degree: the short rows are those of
// vertices bnd[1] .. n-1.)
__global__ __launch_bounds__(512) void k_features_short(DevGraph g, const int32_t *bnd, const double *lt,
                                                        RunArgs ra, float *out)
{
    const RunLds L = load_runs(g, lt, ra);
    const int64_t first = bnd[1];
    for (int64_t v = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t beg = g.rp[v], end = g.rp[v + 1];
        double acc = 0.0, sd = 0.0;
        constexpr int B = 8;
        for (int64_t e0 = beg; e0 < end; e0 += B) {
            int32_t u[B];
#pragma unroll
            for (int j = 0; j < B; ++j) u[j] = (e0 + j < end) ? g.ci[e0 + j] : -1;
            double2 p[B];
            run_lookup<B>(g, lt, L, u, p);
#pragma unroll
            for (int j = 0; j < B; ++j) {
                if (u[j] < 0) continue;
                acc += p[j].x;
                sd += p[j].y;
            }
        }
        write_features(out, v, (double)(end - beg), acc, sd);
    }
}

constexpr int64_t FMID = 256;      // rows up to this long: eight lanes per vertex

// Rows of medium length: a group of G lanes per vertex (G = 8 for rows of
// FSHORT + 1 .. FMID entries, vertices bnd[2] .. bnd[1]-1; G = 64 for rows
// of FMID + 1 .. FPIECE, vertices bnd[0] .. bnd[2]-1; the longer rows,
// vertices 0 .. bnd[0]-1, go in pieces).  A lane keeps eight entries in
// flight; G is matched to the row length so that most lanes have loads
// to issue (a wave per vertex left seven of eight batches empty on rows
// of a few dozen entries).
template <int G>
__global__ __launch_bounds__(512) void k_features_group(DevGraph g, const int32_t *bnd, const double *lt,
                                                        RunArgs ra, float *out)
{
    const RunLds L = load_runs(g, lt, ra);
    const int sub = threadIdx.x & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t grps = ((int64_t)gridDim.x * blockDim.x) / G;
    const int64_t lo = G == 64 ? bnd[0] : bnd[2], hi = G == 64 ? bnd[2] : bnd[1];
    // every lane of a wave runs the same number of iterations (the row's
    // sum needs all G lanes of its group at the shuffles)
    const int64_t span = hi - lo, iters = (span + grps - 1) / grps;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t v = lo + grp + it * grps;
        const bool own = v < hi;
        const int64_t beg = own ? g.rp[v] : 0, end = own ? g.rp[v + 1] : 0;
        double acc = 0.0, sd = 0.0;
        constexpr int B = 8;
        for (int64_t e0 = beg + sub; e0 < end; e0 += G * B) {
            int32_t u[B];
#pragma unroll
            for (int j = 0; j < B; ++j) u[j] = (e0 + G * j < end) ? g.ci[e0 + G * j] : -1;
            double2 p[B];
            run_lookup<B>(g, lt, L, u, p);
#pragma unroll
            for (int j = 0; j < B; ++j) {
                if (u[j] < 0) continue;
                acc += p[j].x;
                sd += p[j].y;
            }
        }
        for (int o = G / 2; o > 0; o >>= 1) {
            acc += __shfl_xor(acc, o);
            sd += __shfl_xor(sd, o);
        }
        if (own && sub == 0) write_features(out, v, (double)(end - beg), acc, sd);
    }
}

// Long rows, in three steps: (1) one workgroup finds H, the number of
// vertices with more than FPIECE entries, and the prefix of their piece
// counts; (2) a wave per piece sums its entries; (3) a thread per long row
// adds its pieces in order.
__global__ __launch_bounds__(1024) void k_feat_pieces(DevGraph g, int64_t *pref, int32_t *H_out)
{
    __shared__ int32_t sH;
    __shared__ int64_t s_run;
    __shared__ int64_t s_w[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        int32_t lo = 0, hi = g.n;      // first vertex with at most FPIECE entries
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if ((int64_t)g.deg[mid] > FPIECE) lo = mid + 1; else hi = mid;
        }
        sH = lo;
        s_run = 0;
        H_out[0] = lo;
        hi = g.n;                      // first vertex with at most FMID entries
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if ((int64_t)g.deg[mid] > FMID) lo = mid + 1; else hi = mid;
        }
        H_out[2] = lo;
        hi = g.n;                      // first vertex with at most FSHORT entries
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if ((int64_t)g.deg[mid] > FSHORT) lo = mid + 1; else hi = mid;
        }
        H_out[1] = lo;
    }
    __syncthreads();
    const int32_t H = sH;
    for (int32_t b0 = 0; b0 < H; b0 += 1024) {
        const int32_t v = b0 + tid;
        int64_t x = v < H ? ((int64_t)g.deg[v] + FPIECE - 1) / FPIECE : 0;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[wid] = x;
        __syncthreads();
        int64_t before = s_run;
        for (int i = 0; i < wid; ++i) before += s_w[i];
        if (v < H) pref[v + 1] = before + x;
        __syncthreads();
        if (tid == 1023) s_run = before + x;
        __syncthreads();
    }
    if (tid == 0) pref[0] = 0;
}

__global__ __launch_bounds__(512) void k_feat_sum(DevGraph g, const int64_t *pref, const int32_t *H_in,
                                                  const double *lt, RunArgs ra, double2 *part)
{
    const RunLds L = load_runs(g, lt, ra);
    const int lane = threadIdx.x & 63;
    const int32_t H = *H_in;
    if (H == 0) return;
    const int64_t total = pref[H];
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < total; q += waves) {
        int32_t lo = 0, hi = H - 1;     // the row v with pref[v] <= q < pref[v + 1]
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (pref[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int64_t b = g.rp[lo] + (q - pref[lo]) * FPIECE;
        const int64_t e = min(b + FPIECE, g.rp[lo + 1]);
        double acc = 0.0, sd = 0.0;
        constexpr int B = 8;
        for (int64_t e0 = b + lane; e0 < e; e0 += 64 * B) {
            int32_t u[B];
#pragma unroll
            for (int j = 0; j < B; ++j) u[j] = (e0 + 64 * j < e) ? g.ci[e0 + 64 * j] : -1;
            double2 p[B];
            run_lookup<B>(g, lt, L, u, p);
#pragma unroll
            for (int j = 0; j < B; ++j) {
                if (u[j] < 0) continue;
                acc += p[j].x;
                sd += p[j].y;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            acc += __shfl_xor(acc, o);
            sd += __shfl_xor(sd, o);
        }
        if (lane == 0) part[q] = make_double2(acc, sd);
    }
}

__global__ void k_feat_combine(DevGraph g, const int64_t *pref, const int32_t *H_in, const double2 *part,
                               float *out)
{
    const int32_t H = *H_in;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < H; v += gridDim.x * blockDim.x) {
        double acc = 0.0, sd = 0.0;
        for (int64_t q = pref[v]; q < pref[v + 1]; ++q) {
            acc += part[q].x;
            sd += part[q].y;
        }
        write_features(out, v, (double)(g.rp[v + 1] - g.rp[v]), acc, sd);
    }
}

__global__ void k_normalize(int32_t n, float *x, const float *norm)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3ll * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % 3);
        x[i] = (x[i] - norm[j]) / norm[3 + j];
    }
}

// C[16x16] += A[16 x K] * B[K x 16] on the matrix cores; a(m, k), b(k, n)
// fetch operands.  Lane l supplies A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16]; the result element (row, col) of accumulator i
// is row = (l / 16) * 4 + i, col = l % 16.
template <typename FA, typename FB>
__device__ __forceinline__ floatx4 mfma_tile(floatx4 c, int K, FA a, FB b)
{
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 4) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a(m, k0 + kk), b(k0 + kk, m), c, 0, 0, 0);
    return c;
}

// Forward (and, when train != 0, backward) over all rows.
__global__ __launch_bounds__(256) void k_mlp(const float *P, const float *X, const float *Yt, int64_t rows,
                                             float *Yout, float *partial, int train)
{
    __shared__ float sW1[192], sb1[64], sb2[64], sW3[64];
    __shared__ float sW2[64 * LD];
    __shared__ float sX[TR * 3];
    __shared__ float sH1[TR * LD];
    __shared__ float sH2[TR * LD];   // H2, then D1
    __shared__ float sD2[TR * LD];
    __shared__ float sdy[TR];
    __shared__ float gW1[192], gb1[64], gb2[64], gW3[64];
    __shared__ float sgb3, sloss;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < 192; i += 256) { sW1[i] = P[OFF_W1 + i]; gW1[i] = 0.f; }
    for (int i = tid; i < 64; i += 256) {
        sb1[i] = P[OFF_B1 + i];
        sb2[i] = P[OFF_B2 + i];
        sW3[i] = P[OFF_W3 + i];
        gb1[i] = gb2[i] = gW3[i] = 0.f;
    }
    for (int i = tid; i < 4096; i += 256) sW2[(i >> 6) * LD + (i & 63)] = P[OFF_W2 + i];
    if (tid == 0) { sgb3 = 0.f; sloss = 0.f; }
    const float b3 = P[OFF_B3];
    floatx4 gacc[4];
    for (int t = 0; t < 4; ++t) gacc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    const float scale = 2.0f / (float)rows;

    for (int64_t r0 = (int64_t)blockIdx.x * TR; r0 < rows; r0 += (int64_t)gridDim.x * TR) {
        const int cnt = (int)min<int64_t>(TR, rows - r0);
        for (int i = tid; i < TR * 3; i += 256) sX[i] = (i / 3 < cnt) ? X[r0 * 3 + i] : 0.f;
        __syncthreads();
        // hidden layer 1 (K = 3): thread -> row tid/4, 16 outputs
        {
            const int r = tid >> 2, o0 = (tid & 3) * 16;
            const float x0 = sX[3 * r], x1 = sX[3 * r + 1], x2 = sX[3 * r + 2];
            for (int o = o0; o < o0 + 16; ++o) {
                float z = sb1[o];
                z = fmaf(sW1[3 * o + 0], x0, z);
                z = fmaf(sW1[3 * o + 1], x1, z);
                z = fmaf(sW1[3 * o + 2], x2, z);
                sH1[r * LD + o] = z > 0.f ? z : 0.f;
            }
        }
        __syncthreads();
        // hidden layer 2: Z2[r][o] = sum_k H1[r][k] W2[o][k]; wave w owns rows 16w..16w+15
        for (int ct = 0; ct < 4; ++ct) {
            floatx4 c = mfma_tile(floatx4{0.f, 0.f, 0.f, 0.f}, 64,
                                  [&](int m, int k) { return sH1[(16 * w + m) * LD + k]; },
                                  [&](int k, int nn) { return sW2[(16 * ct + nn) * LD + k]; });
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * w + (lane >> 4) * 4 + i, col = 16 * ct + (lane & 15);
                const float z = c[i] + sb2[col];
                sH2[row * LD + col] = z > 0.f ? z : 0.f;
            }
        }
        __syncthreads();
        // output layer and loss
        if (tid < TR) {
            float y = b3;
            for (int k = 0; k < 64; ++k) y = fmaf(sW3[k], sH2[tid * LD + k], y);
            if (tid < cnt) {
                if (Yout) Yout[r0 + tid] = y;
                if (train) {
                    const float d = y - Yt[r0 + tid];
                    atomicAdd(&sloss, d * d);
                    sdy[tid] = scale * d;
                }
            } else {
                sdy[tid] = 0.f;
            }
        }
        if (!train) { __syncthreads(); continue; }
        __syncthreads();
        // D2 = dy W3 masked by H2 > 0; gW3, gb3
        for (int i = tid; i < TR * 64; i += 256) {
            const int r = i >> 6, o = i & 63;
            const float h = sH2[r * LD + o];
            sD2[r * LD + o] = h > 0.f ? sdy[r] * sW3[o] : 0.f;
        }
        if (tid < 64) {
            float gw = 0.f, gb = 0.f;
            for (int r = 0; r < TR; ++r) gw = fmaf(sdy[r], sH2[r * LD + tid], gw);
            gW3[tid] += gw;
            if (tid == 0) {
                for (int r = 0; r < TR; ++r) gb += sdy[r];
                sgb3 += gb;
            }
        }
        __syncthreads();
        // gW2[o][k] += sum_r D2[r][o] H1[r][k]  (wave w owns o in 16w..16w+15)
        for (int kt = 0; kt < 4; ++kt)
            gacc[kt] = mfma_tile(gacc[kt], TR,
                                 [&](int m, int r) { return sD2[r * LD + 16 * w + m]; },
                                 [&](int r, int nn) { return sH1[r * LD + 16 * kt + nn]; });
        if (tid < 64) {
            float gb = 0.f;
            for (int r = 0; r < TR; ++r) gb += sD2[r * LD + tid];
            gb2[tid] += gb;
        }
        // D1[r][k] = sum_o D2[r][o] W2[o][k], masked by H1 > 0 (into sH2)
        for (int kt = 0; kt < 4; ++kt) {
            floatx4 c = mfma_tile(floatx4{0.f, 0.f, 0.f, 0.f}, 64,
                                  [&](int m, int o) { return sD2[(16 * w + m) * LD + o]; },
                                  [&](int o, int nn) { return sW2[o * LD + 16 * kt + nn]; });
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * w + (lane >> 4) * 4 + i, col = 16 * kt + (lane & 15);
                sH2[row * LD + col] = sH1[row * LD + col] > 0.f ? c[i] : 0.f;
            }
        }
        __syncthreads();
        // gW1[o][j] += sum_r D1[r][o] X[r][j]; gb1
        if (tid < 64) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, gb = 0.f;
            for (int r = 0; r < TR; ++r) {
                const float d = sH2[r * LD + tid];
                a0 = fmaf(d, sX[3 * r], a0);
                a1 = fmaf(d, sX[3 * r + 1], a1);
                a2 = fmaf(d, sX[3 * r + 2], a2);
                gb += d;
            }
            gW1[3 * tid] += a0;
            gW1[3 * tid + 1] += a1;
            gW1[3 * tid + 2] += a2;
            gb1[tid] += gb;
        }
        __syncthreads();
    }
    if (!train) return;
    float *out = partial + (size_t)blockIdx.x * PSTRIDE;
    for (int kt = 0; kt < 4; ++kt)
        for (int i = 0; i < 4; ++i) {
            const int o = 16 * w + (lane >> 4) * 4 + i, k = 16 * kt + (lane & 15);
            out[OFF_W2 + o * 64 + k] = gacc[kt][i];
        }
    __syncthreads();
    for (int i = tid; i < 192; i += 256) out[OFF_W1 + i] = gW1[i];
    for (int i = tid; i < 64; i += 256) {
        out[OFF_B1 + i] = gb1[i];
        out[OFF_B2 + i] = gb2[i];
        out[OFF_W3 + i] = gW3[i];
    }
    if (tid == 0) {
        out[OFF_B3] = sgb3;
        out[NP] = sloss;
    }
}

// Forward pass alone (the learned prior's inference over every vertex).
// Each wave takes 16-row strips on its own, with no LDS and no barrier, and
// works on transposed activations so that one layer's MFMA output is laid
// out as the next layer's B operand.  With v_mfma_f32_16x16x4f32, lane
// l = 16 g + r (g = 0..3, r = 0..15) supplies A[r][g] and B[g][r] and gets
// C[4 g + i][r], i = 0..3.
//  * layer 1: Z1^T (16 hidden x 16 rows, four tiles) = W1' X'^T, where W1'
//    is W1 with the bias as a fourth column and X' the rows with a fourth
//    input fixed at 1, so lane (g, r) gives input g of row r (the bias's 1
//    for g = 3) and weight W1'[16 t + r][g];
//  * layer 2: Z2^T = W2 H1^T summed over the 64 hidden inputs k in the
//    order k = 16 t + 4 g + i of step q = 4 t + i: at that step lane (g, r)
//    holds exactly H1^T[16 t + 4 g + i][r] (its layer-1 output), and gives
//    W2[16 u + r][16 t + 4 g + i] as A for output tile u;
//  * layer 3: each lane's 16 outputs times W3, then a sum over the four
//    lanes of a row (shuffles by 16 and 32).
// With norm (the training mean and standard deviation of each feature) the
// inputs are standardised on load.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *P, const float *X, const float *norm, int64_t rows,
                                                 float *Y)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    float a1[4], a2[4][16], b2[4][4], w3[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) a1[t] = g < 3 ? P[OFF_W1 + (16 * t + r) * 3 + g] : P[OFF_B1 + 16 * t + r];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int q = 0; q < 16; ++q) a2[u][q] = P[OFF_W2 + (16 * u + r) * 64 + 16 * (q >> 2) + 4 * g + (q & 3)];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b2[u][i] = P[OFF_B2 + 16 * u + 4 * g + i];
            w3[u][i] = P[OFF_W3 + 16 * u + 4 * g + i];
        }
    }
    const float b3 = P[OFF_B3];
    const float mu = (norm && g < 3) ? norm[g] : 0.f, sd = (norm && g < 3) ? norm[3 + g] : 1.f;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t s0 = wave * 16; s0 < rows; s0 += waves * 16) {
        const int64_t row = s0 + r;
        float x = 1.f;
        if (g < 3) {
            x = row < rows ? X[row * 3 + g] : 0.f;
            if (norm) x = (x - mu) / sd;
        }
        floatx4 h1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            h1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[t], x, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) h1[t][i] = h1[t][i] > 0.f ? h1[t][i] : 0.f;
        }
        floatx4 z2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z2[u] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 16; ++q)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                z2[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[u][q], h1[q >> 2][q & 3], z2[u], 0, 0, 0);
        float y = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = z2[u][i] + b2[u][i];
                y = fmaf(w3[u][i], z > 0.f ? z : 0.f, y);
            }
        y += __shfl_xor(y, 16);
        y += __shfl_xor(y, 32);
        if (g == 0 && row < rows) Y[row] = y + b3;
    }
}

__global__ void k_reduce_partials(const float *partial, int nb, float *grad, float *loss, float inv_rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NP) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * PSTRIDE + i];
    if (i < NP) grad[i] = s;
    else *loss = s * inv_rows;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int count, float lr, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_prior(int32_t n, const float *y, double inv_omega, double *prior)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        // betweenness lies in [0, 1] (Sec. I), so the prior is clamped to it;
        // a non-finite output passes through (the budget check rejects it)
        const double b = exp((double)y[v]) - inv_omega;
        prior[v] = isfinite(b) ? (b > 1.0 ? 1.0 : (b > 0.0 ? b : 0.0)) : b;
    }
}

// ---- training (kad_mlp_train) ----

// Regression target of a vertex: y = ln(b~ + 1/omega), in FP64, stored FP32.
__global__ void k_target(int32_t n, const double *b, double inv_omega, float *y)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        y[v] = (float)log(b[v] + inv_omega);
}

constexpr int MOM_BLOCKS = 256;

// Per-block FP64 partial sums of the three feature columns (pass 0) or of
// their squared deviations from `mean` (pass 1); a block's rows are a fixed
// grid-stride set, so the sums do not depend on scheduling.
__global__ __launch_bounds__(256) void k_moments(const float *x, int64_t rows, const double *mean, double *part)
{
    __shared__ double sm[3][256];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const double m0 = mean ? mean[0] : 0.0, m1 = mean ? mean[1] : 0.0, m2 = mean ? mean[2] : 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256) {
        const double x0 = (double)x[3 * r] - m0, x1 = (double)x[3 * r + 1] - m1, x2 = (double)x[3 * r + 2] - m2;
        if (mean) {
            a0 += x0 * x0;
            a1 += x1 * x1;
            a2 += x2 * x2;
        } else {
            a0 += x0;
            a1 += x1;
            a2 += x2;
        }
    }
    sm[0][threadIdx.x] = a0;
    sm[1][threadIdx.x] = a1;
    sm[2][threadIdx.x] = a2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int j = 0; j < 3; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

// Sums the block partials in block order: mean (pass 0) or the population
// standard deviation (pass 1; a zero deviation is taken as 1); writes the
// FP64 value and, for pass 1, the FP32 standardisation vector norm =
// [mean, std].
__global__ void k_moments_finish(const double *part, int nb, int64_t rows, double *out, const double *mean,
                                 float *norm)
{
    const int j = threadIdx.x;
    if (j >= 3) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[3 * b + j];
    if (!mean) {
        out[j] = s / (double)rows;
    } else {
        double sd = sqrt(s / (double)rows);
        if (!(sd > 0.0)) sd = 1.0;
        out[j] = sd;
        norm[j] = (float)mean[j];
        norm[3 + j] = (float)sd;
    }
}

// Uniform initialisation in [-sqrt(6 / fan_in), sqrt(6 / fan_in)) for the
// weights (He), zero biases: parameter i takes draw 0 of Philox sample i of
// stream 2, u = (2 * unit53 - 1) * bound.
__global__ void k_mlp_init(uint64_t seed, float *p)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    double bound = 0.0;
    if (i < OFF_B1) bound = sqrt(6.0 / 3.0);
    else if (i >= OFF_W2 && i < OFF_B2) bound = sqrt(6.0 / 64.0);
    else if (i >= OFF_W3 && i < OFF_B3) bound = sqrt(6.0 / 64.0);
    float v = 0.f;
    if (bound > 0.0) {
        SampleDraws dr;
        dr.init(seed, 2, (uint64_t)i);
        const double u = (double)(dr.get(0) >> 11) * 0x1p-53;
        v = (float)((2.0 * u - 1.0) * bound);
    }
    p[i] = v;
}

// Batch of Adam step j: row b of the batch is row floor(u * rows / 2^64) of
// the training set, u = draw b of Philox sample 2^32 + j of stream 2
// (uniform rows, with replacement).
__global__ void k_gather_batch(uint64_t seed, uint64_t step, int32_t batch, int64_t rows, const float *x,
                               const float *y, float *xb, float *yb)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    uint64_t c[4] = {(uint64_t)b >> 2, (1ull << 32) + step, 0, 0};
    philox4x64_10(seed, 2, c);
    const uint64_t u = c[b & 3];
    const int64_t r = (int64_t)__umul64hi(u, (uint64_t)rows);
    xb[3 * b] = x[3 * r];
    xb[3 * b + 1] = x[3 * r + 1];
    xb[3 * b + 2] = x[3 * r + 2];
    yb[b] = y[r];
}

// acc[e] += loss (the batch loss, a mean over its rows).
__global__ void k_acc_loss(const float *loss, double *acc, int e)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) acc[e] += (double)*loss;
}

int blocks_for_rows(int64_t rows)
{
    int64_t b = (rows + TR - 1) / TR;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 1024);
}

}  // namespace

size_t mlp_scratch_floats(int64_t rows) { return (size_t)blocks_for_rows(rows) * PSTRIDE; }

// Workspace of the feature pass: the prefix of the long rows' pieces, the
// tier boundaries, the pieces' partial sums and the logarithm table (n
// entries at most: no degree reaches n).  Long rows have more than FPIECE
// entries each, so there are at most nnz / FPIECE of them and at most
// 2 nnz / FPIECE + 1 pieces.
size_t features_workspace_bytes(const DevGraph &g)
{
    const int64_t hmax = g.nnz / FPIECE + 1, pmax = 2 * (g.nnz / FPIECE) + 1;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    return up(sizeof(int64_t) * (size_t)(hmax + 1)) + 256 + up(sizeof(double2) * (size_t)pmax) +
           up(sizeof(double) * (size_t)g.n);
}

hipError_t launch_features_ws(const DevGraph &g, const DegreeRuns &runs, float *out, void *ws, hipStream_t st)
{
    if (runs.count < 1) return hipErrorInvalidValue;
    RunArgs ra;
    ra.start = runs.start;
    ra.deg = runs.deg;
    ra.first = std::max(0, runs.count - RUNCAP);
    ra.cnt = runs.count - ra.first;
    ra.pow2 = 1;
    while (ra.pow2 < ra.cnt) ra.pow2 <<= 1;
    const size_t lds = run_lds_bytes(ra.cnt, ra.pow2);
    const int64_t hmax = g.nnz / FPIECE + 1, pmax = 2 * (g.nnz / FPIECE) + 1;
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    int64_t *pref = (int64_t *)ws;
    int32_t *H = (int32_t *)((char *)ws + up(sizeof(int64_t) * (size_t)(hmax + 1)));  // tier boundaries
    double2 *part = (double2 *)((char *)H + 256);
    double *lt = (double *)((char *)part + up(sizeof(double2) * (size_t)pmax));
    const int64_t tblocks = std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_logtab, dim3((unsigned)tblocks), dim3(256), 0, st, g, lt);
    hipLaunchKernelGGL(k_feat_pieces, dim3(1), dim3(1024), 0, st, g, pref, H);
    // each workgroup fills its LDS table once, then strides over its tier
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(((int64_t)g.n + 511) / 512, 2048));
    hipLaunchKernelGGL(k_features_short, dim3((unsigned)blocks), dim3(512), lds, st, g, H, lt, ra, out);
    hipLaunchKernelGGL(k_features_group<8>, dim3((unsigned)blocks), dim3(512), lds, st, g, H, lt, ra, out);
    hipLaunchKernelGGL(k_features_group<64>, dim3((unsigned)blocks), dim3(512), lds, st, g, H, lt, ra, out);
    hipLaunchKernelGGL(k_feat_sum, dim3(1024), dim3(512), lds, st, g, pref, H, lt, ra, part);
    hipLaunchKernelGGL(k_feat_combine, dim3(64), dim3(256), 0, st, g, pref, H, part, out);
    return hipGetLastError();
}

hipError_t launch_features(const DevGraph &g, const DegreeRuns &runs, float *out, hipStream_t st)
{
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, features_workspace_bytes(g), st);
    if (e != hipSuccess) return e;
    e = launch_features_ws(g, runs, out, ws, st);
    const hipError_t f = hipFreeAsync(ws, st);
    return e != hipSuccess ? e : f;
}

hipError_t launch_normalize(int32_t n, float *x, const float *norm, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((3ll * n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_normalize, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, n, x, norm);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const float *x, const float *norm, int64_t rows, float *y,
                              hipStream_t st)
{
    const int64_t strips = (rows + 15) / 16;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((strips + 3) / 4, 2048));
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)blocks), dim3(256), 0, st, params, x, norm, rows, y);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t rows, float *grad,
                                float *loss, float *scratch, hipStream_t st)
{
    const int nb = blocks_for_rows(rows);
    hipLaunchKernelGGL(k_mlp, dim3(nb), dim3(256), 0, st, params, x, y, rows, (float *)nullptr, scratch, 1);
    hipLaunchKernelGGL(k_reduce_partials, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, scratch, nb, grad, loss,
                       1.0f / (float)rows);
    return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int count, int step, float lr,
                       hipStream_t st)
{
    const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, st, params, grad, m, v, count, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_prior_from_mlp(int32_t n, const float *yhat, double omega, double *prior, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_prior, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, n, yhat,
                       1.0 / omega, prior);
    return hipGetLastError();
}

hipError_t launch_target(int32_t n, const double *btilde, double omega, float *y, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_target, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, n, btilde,
                       1.0 / omega, y);
    return hipGetLastError();
}

size_t moments_scratch_doubles() { return 3 * MOM_BLOCKS + 6; }

hipError_t launch_feature_norm(const float *x, int64_t rows, double *scratch, float *norm, hipStream_t st)
{
    const int nb = (int)std::min<int64_t>(MOM_BLOCKS, std::max<int64_t>(1, (rows + 255) / 256));
    double *part = scratch, *mean = scratch + 3 * MOM_BLOCKS, *sd = mean + 3;
    hipLaunchKernelGGL(k_moments, dim3(nb), dim3(256), 0, st, x, rows, (const double *)nullptr, part);
    hipLaunchKernelGGL(k_moments_finish, dim3(1), dim3(64), 0, st, part, nb, rows, mean, (const double *)nullptr,
                       (float *)nullptr);
    hipLaunchKernelGGL(k_moments, dim3(nb), dim3(256), 0, st, x, rows, (const double *)mean, part);
    hipLaunchKernelGGL(k_moments_finish, dim3(1), dim3(64), 0, st, part, nb, rows, sd, (const double *)mean, norm);
    return hipGetLastError();
}

hipError_t launch_mlp_init(uint64_t seed, float *params, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_init, dim3((NP + 255) / 256), dim3(256), 0, st, seed, params);
    return hipGetLastError();
}

hipError_t launch_gather_batch(uint64_t seed, uint64_t step, int32_t batch, int64_t rows, const float *x,
                               const float *y, float *xb, float *yb, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_batch, dim3((batch + 255) / 256), dim3(256), 0, st, seed, step, batch, rows, x, y,
                       xb, yb);
    return hipGetLastError();
}

hipError_t launch_acc_loss(const float *loss, double *acc, int e, hipStream_t st)
{
    hipLaunchKernelGGL(k_acc_loss, dim3(1), dim3(64), 0, st, loss, acc, e);
    return hipGetLastError();
}

}  // namespace kad
