// Epoch boundary, stop rule, delta allocation, diameter bracket, Philox dump.
//
// Epoch boundary (Sec. III-B, Alg. 2 on one GPU): the samples of epoch k
// were counted into state frame SF[k & 1]; the merge kernel adds that frame
// into c~, clears it for epoch k + 2 (two frames suffice: frames of epoch
// e - 2 are never touched again), and evaluates the stop rule on exactly
// the samples [0, tau) -- the consistent snapshot the rule needs because f
// and g are not monotone.
//
// Stop rule (Sec. III-A): stop once f(b~(v), delta_L(v), omega, tau) < eps
// and g(b~(v), delta_U(v), omega, tau) < eps for every vertex, or tau has
// reached ceil(omega).  With L = ln(1/delta) and a = omega / tau (KADABRA's
// Bernstein-type bounds, the reading used throughout):
//   f = L/tau ((1/3 - a) + sqrt((1/3 - a)^2 + 2 b~ omega / L)), capped at b~
//   g = L/tau ((1/3 + a) + sqrt((1/3 + a)^2 + 2 b~ omega / L)), capped at 1 - b~
// evaluated in FP64 (the only FP64 on the sampling path), without FMA
// contraction, in the order written.
#include <math.h>

#include <algorithm>
#include <vector>

#include "kad_internal.h"
#include "philox.h"

namespace kad {
namespace {

constexpr int MB = 256;   // merge block size

__device__ __forceinline__ double fval(double bt, double L, double omega, double tau)
{
    const double a = (1.0 / 3.0) - omega / tau;
    const double q = a * a + ((2.0 * bt) * omega) / L;
    const double f = (L / tau) * (a + sqrt(q));
    return f < bt ? f : bt;
}
__device__ __forceinline__ double gval(double bt, double L, double omega, double tau)
{
    const double a = (1.0 / 3.0) + omega / tau;
    const double q = a * a + ((2.0 * bt) * omega) / L;
    const double g = (L / tau) * (a + sqrt(q));
    const double cap = 1.0 - bt;
    return g < cap ? g : cap;
}
__device__ __forceinline__ uint64_t bits(double d) { return __builtin_bit_cast(uint64_t, d); }
__device__ __forceinline__ double dbl(uint64_t b) { return __builtin_bit_cast(double, b); }

struct EpochHist {
    double max_f, max_g, min_margin;
    int32_t ok;
    int32_t pad;
};

__global__ __launch_bounds__(MB) void k_merge_stop(int32_t n, uint32_t *c, uint32_t *sf0, uint32_t *sf1,
                                                   const double *LL, const double *LU, double omega,
                                                   double eps, unsigned long long cap,
                                                   unsigned long long E, EpochState *es,
                                                   unsigned long long *work_ctr, EpochHist *hist,
                                                   int32_t hist_cap, HostStatus *hs,
                                                   unsigned long long *pool_epoch, int pools,
                                                   unsigned long long *defer_ctr, const uint32_t *lcnt,
                                                   const double *ltab)
{
    if (__hip_atomic_load(&es->stopped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const unsigned long long first = es->range[0], count = es->range[1];
    uint32_t *sf = (es->range[2] & 1) ? sf1 : sf0;
    const unsigned long long tau_u = first + count;
    const double tau = (double)tau_u;
    int ok = 1;
    double mf = 0.0, mg = 0.0, mm = INFINITY;
    // f and g of the thread's previous vertex, reused when the next has the
    // same count and the same L bits (the same inputs give the same FP64
    // results): nearly every vertex of a large graph is never counted, and
    // with the calibrated allocation all uncounted vertices of one
    // calibration count share L, so the divisions and square roots run for
    // a small share of the vertices.  Four vertices a thread per round keep
    // their loads in flight together.  Only the vertices counted in the
    // epoch (sf != 0; about 10 K of R-MAT 26's 32.8 M per epoch) are written
    // back, so the pass over the others only reads.
    uint32_t m_cv = 0xFFFFFFFFu;
    uint64_t m_ll = 0, m_lu = 0;
    double m_f = 0.0, m_g = 0.0;
    constexpr int R = 4;
    const int64_t stride = (int64_t)gridDim.x * MB;
    for (int64_t v0 = (int64_t)blockIdx.x * MB + threadIdx.x; v0 < n; v0 += R * stride) {
        uint32_t cv[R], sv[R];
        double ll[R], lu[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t v = v0 + j * stride;
            cv[j] = 0;
            sv[j] = 0;
            ll[j] = lu[j] = 0.0;
            if (v < n) {
                sv[j] = sf[v];
                cv[j] = c[v] + sv[j];
                // the calibrated allocation by count value (delta_L =
                // delta_U), or the L arrays
                ll[j] = ltab ? ltab[lcnt[v]] : LL[v];
                lu[j] = (ltab || LU == LL) ? ll[j] : LU[v];   // one array when delta_L = delta_U
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t v = v0 + j * stride;
            if (v >= n) continue;
            if (sv[j]) {
                c[v] = cv[j];
                sf[v] = 0;
            }
            double f, g;
            if (cv[j] == m_cv && bits(ll[j]) == m_ll && bits(lu[j]) == m_lu) {
                f = m_f;
                g = m_g;
            } else {
                const double bt = (double)cv[j] / tau;
                f = fval(bt, ll[j], omega, tau);
                g = gval(bt, lu[j], omega, tau);
                m_cv = cv[j];
                m_ll = bits(ll[j]);
                m_lu = bits(lu[j]);
                m_f = f;
                m_g = g;
            }
            ok &= (f < eps && g < eps) ? 1 : 0;
            mf = f > mf ? f : mf;
            mg = g > mg ? g : mg;
            double mar = eps - (f > g ? f : g);
            mar = mar < 0 ? -mar : mar;
            mm = mar < mm ? mar : mm;
        }
    }
    // block reduction
    __shared__ int s_ok;
    __shared__ unsigned long long s_f, s_g, s_m;
    if (threadIdx.x == 0) {
        s_ok = 1;
        s_f = 0;
        s_g = 0;
        s_m = bits(INFINITY);
    }
    __syncthreads();
    if (!ok) atomicAnd(&s_ok, 0);
    atomicMax(&s_f, (unsigned long long)bits(mf));
    atomicMax(&s_g, (unsigned long long)bits(mg));
    atomicMin(&s_m, (unsigned long long)bits(mm));
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (!s_ok) atomicAnd(&es->all_ok, 0);
    atomicMax(&es->max_f_bits, s_f);
    atomicMax(&es->max_g_bits, s_g);
    atomicMin(&es->min_margin_bits, s_m);
    __threadfence();
    const unsigned long long done = atomicAdd(&es->blocks_done, 1ull);
    if (done != gridDim.x - 1) return;
    __threadfence();
    // last block: decide, record, prepare the next epoch's range
    const int all = __hip_atomic_load(&es->all_ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double F = dbl(__hip_atomic_load(&es->max_f_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const double G = dbl(__hip_atomic_load(&es->max_g_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const double M = dbl(__hip_atomic_load(&es->min_margin_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const unsigned long long ep = es->epoch;
    if ((int64_t)ep < hist_cap) {
        hist[ep].max_f = F;
        hist[ep].max_g = G;
        hist[ep].min_margin = M;
        hist[ep].ok = all;
    }
    es->tau = tau_u;
    es->epoch = ep + 1;
    es->max_f = F;
    es->max_g = G;
    es->min_margin = M;
    int stop = 0, reason = KAD_STOP_NONE;
    if (all) { stop = 1; reason = KAD_STOP_COND; }
    else if (tau_u >= cap) { stop = 1; reason = KAD_STOP_OMEGA; }
    es->reason = reason;
    es->all_ok = 1;
    es->max_f_bits = 0;
    es->max_g_bits = 0;
    es->min_margin_bits = bits(INFINITY);
    es->blocks_done = 0;
    const unsigned long long nfirst = tau_u;
    es->range[0] = nfirst;
    es->range[1] = stop ? 0 : ((cap - nfirst) < E ? (cap - nfirst) : E);
    es->range[2] = ep + 1;
    if (work_ctr) *work_ctr = 0;
    if (defer_ctr) {   // the pool's deferred-sample counters, for its next epoch
        defer_ctr[0] = 0;
        defer_ctr[1] = 0;
    }
    if (pool_epoch) *pool_epoch += (unsigned long long)pools;   // this pool's next epoch
    __threadfence();
    __hip_atomic_store(&es->stopped, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hs) {
        hs->reason = reason;
        hs->epoch = ep + 1;
        hs->tau = tau_u;
        hs->stopped = stop;
        __threadfence_system();
    }
}

__global__ void k_fg(int32_t n, const uint32_t *c, double tau, const double *LL, const double *LU,
                     double omega, double *f, double *g)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const double bt = (double)c[v] / tau;
        f[v] = fval(bt, LL[v], omega, tau);
        g[v] = gval(bt, LU[v], omega, tau);
    }
}

__global__ void k_btilde(int32_t n, const uint32_t *c, double tau, double *b)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        b[v] = (double)c[v] / tau;
}

__global__ void k_philox(uint64_t seed, uint64_t stream, uint64_t first, uint32_t count, uint32_t nwords,
                         uint64_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    SampleDraws dr;
    dr.init(seed, stream, first + i);
    for (uint32_t j = 0; j < nwords; ++j) out[i * nwords + j] = dr.get(j);
}

// ---- delta allocation (calibration, Sec. III-A phase 2; reading:
// delta(v) = (1 - beta) exp(-C / prior(v)) + beta delta / (4n), with C the
// smallest value for which the sum over vertices with prior > 0 of
// exp(-C / prior(v)) stays below delta / 4 (shrunk by 1e-9), by bisection).

constexpr int AB = 256;

__device__ __forceinline__ double prior_of(const AllocArgs &a, int32_t v)
{
    return a.counts ? (double)a.counts[v] / a.tau0 : a.dense_prior[v];
}

// A dense prior's constant C: the root of S(C) = T for S(C) = sum over
// p > 0 of exp(-C / p) and T = delta / 4 (1 - 1e-9), i.e. the bisection's
// answer (the smallest C with S(C) <= T) to within 2^-39 relative.  ln S is
// convex and decreasing in C, so Newton's method on ln S - ln T rises
// monotonically from the left; the step is kept inside the bracket
// [lo, hi] of evaluated points (S(lo) > T >= S(hi); hi starts at
// ln(K/T), K = S(0), where S <= T holds), and bisection takes over after
// 60 Newton steps or when a step would leave the bracket.  When Newton
// stalls just left of the root, C is raised by 2^-40 relative until
// S(C) <= T.  One launch per evaluation: each workgroup sums its fixed
// segments of the compacted priors (S, and M = sum exp(-C/p)/p; the
// compaction keeps only the priors whose terms are not exactly zero inside
// the bracket, see k_prior_compact), the last to finish adds the partial
// sums in a fixed order and picks the next point.
struct NewtonState {
    double C, lo, hi;
    int32_t phase;   // 0: Newton, 1: raised just right of a stalled Newton iterate, 2: bisection
    int32_t done;
    unsigned int blocks_done;
    int32_t steps;
};

// Segment s (vertices s * chunk .. s * chunk + chunk - 1) keeps its
// cnt[s] retained priors at packed[s * chunk ...], in vertex order.
__global__ __launch_bounds__(AB) void k_alloc_newton(AllocArgs a, const double *packed, const int32_t *cnt,
                                                     int32_t nseg, int32_t chunk, int32_t seg_per_block,
                                                     double target)
{
    NewtonState *ns = reinterpret_cast<NewtonState *>(a.lo_hi);
    if (__hip_atomic_load(&ns->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const double C = ns->C;
    double sS = 0.0, sM = 0.0;
    // thread t sums positions t, t + AB, ... of each of the block's segments
    // in turn, eight loads in flight at a time
    constexpr int R = 8;
    const int32_t s_end = min(nseg, (int32_t)(blockIdx.x + 1) * seg_per_block);
    for (int32_t sg = blockIdx.x * seg_per_block; sg < s_end; ++sg) {
        const int32_t m = cnt[sg];
        const double *src = packed + (int64_t)sg * chunk;
        for (int32_t i0 = threadIdx.x; i0 < m; i0 += R * AB) {
            double p[R];
#pragma unroll
            for (int j = 0; j < R; ++j) p[j] = i0 + j * AB < m ? src[i0 + j * AB] : 0.0;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (p[j] > 0.0) {
                    const double e = exp(-C / p[j]);
                    sS = sS + e;
                    sM = sM + e / p[j];
                }
            }
        }
    }
    __shared__ double rs[AB], rm[AB];
    __shared__ int last;
    rs[threadIdx.x] = sS;
    rm[threadIdx.x] = sM;
    __syncthreads();
    for (int o = AB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rs[threadIdx.x] = rs[threadIdx.x] + rs[threadIdx.x + o];
            rm[threadIdx.x] = rm[threadIdx.x] + rm[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partials[2 * blockIdx.x] = rs[0];
        a.partials[2 * blockIdx.x + 1] = rm[0];
        __threadfence();
        last = atomicAdd(&ns->blocks_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    // the last workgroup: the partial sums in a fixed order (thread t takes
    // blocks t, t + AB, ... in turn, then a pairwise tree)
    const int32_t nb = (int32_t)gridDim.x;
    sS = 0.0;
    sM = 0.0;
    for (int32_t b = threadIdx.x; b < nb; b += AB) {
        sS = sS + __hip_atomic_load(&a.partials[2 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sM = sM + __hip_atomic_load(&a.partials[2 * b + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    rs[threadIdx.x] = sS;
    rm[threadIdx.x] = sM;
    __syncthreads();
    for (int o = AB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rs[threadIdx.x] = rs[threadIdx.x] + rs[threadIdx.x + o];
            rm[threadIdx.x] = rm[threadIdx.x] + rm[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double S = rs[0], M = rm[0];
    ns->blocks_done = 0;
    ns->steps += 1;
    if (!(S == S) || !(M == M) || ns->steps > 400) {
        ns->done = 1;   // a prior that is not finite: the allocation fails its check
    } else if (ns->steps == 1) {   // C = 0: S is the number of vertices with p > 0
        if (S <= target) {
            ns->done = 1;   // C = 0
        } else {
            ns->lo = 0.0;
            ns->hi = fmax(0.0, log(S / target));
            ns->C = fmin(ns->hi, (log(S) - log(target)) * (S / M));
        }
    } else {
        double lo = ns->lo, hi = ns->hi;
        if (S > target) lo = C; else hi = C;
        ns->lo = lo;
        ns->hi = hi;
        const double mid = 0.5 * (lo + hi);
        if (hi - lo <= hi * 0x1p-39 || mid <= lo || mid >= hi) {
            ns->done = 1;
            ns->C = hi;
        } else if (S > target && ns->phase != 2) {
            const double Cn = C + (log(S) - log(target)) * (S / M);
            if (ns->steps > 60 || Cn >= hi) {
                ns->phase = 2;
                ns->C = mid;
            } else if (Cn > C) {
                ns->phase = 0;
                ns->C = Cn;
            } else {   // stalled left of the root
                ns->phase = 1;
                ns->C = C > 0.0 ? fmin(hi, C * (1.0 + 0x1p-40)) : fmin(hi, 0x1p-1000);
            }
        } else {
            ns->phase = 2;
            ns->C = mid;
        }
    }
    __threadfence();
}

// A bracket of the root before the first Newton step, from a histogram of
// the priors.  Bin 0 holds the priors below 2^-64; bin 1 + 64 (e + 64) + j
// (e = -64 .. -1, j = 0 .. 63) holds [2^e (1 + j/64), 2^e (1 + (j+1)/64)),
// read off the exponent and the top six mantissa bits, so the edges are
// exact; a prior of 1 goes to the last bin, whose upper edge is 1.
// Replacing every prior by its bin's lower edge can only shrink S (each term
// exp(-C/p) grows with p), by the upper edge only raise it; the roots of the
// two bounding sums, found by bisection over the 4 097 bins in one
// workgroup, therefore enclose the root of S, and lie within a factor
// 1 + 1/64 of it.  Newton's method then starts at the lower one (S > T
// there) with the upper one as the right end of its bracket, a few steps
// from the root instead of about twenty from C = 0.
constexpr int PHB = 4097;

__device__ __forceinline__ int prior_bin(double p)
{
    const uint64_t b = bits(p);
    const int e = (int)((b >> 52) & 0x7ff) - 1023;
    if (e < -64) return 0;
    if (e >= 0) return PHB - 1;
    return 1 + (e + 64) * 64 + (int)((b >> 46) & 63);
}

__device__ __forceinline__ void prior_bin_edges(int bin, double *lo, double *up)
{
    if (bin == 0) {
        *lo = 0.0;
        *up = 0x1p-64;
        return;
    }
    const int e = (bin - 1) / 64 - 64, j = (bin - 1) % 64;
    *lo = ldexp(1.0 + j / 64.0, e);
    *up = ldexp(1.0 + (j + 1) / 64.0, e);
}

__global__ __launch_bounds__(256) void k_prior_hist(AllocArgs a, uint32_t *ph)
{
    __shared__ uint32_t sh[PHB];
    for (int i = threadIdx.x; i < PHB; i += blockDim.x) sh[i] = 0;
    __syncthreads();
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        const double p = a.dense_prior[v];
        if (p > 0.0) atomicAdd(&sh[prior_bin(p)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PHB; i += blockDim.x)
        if (sh[i]) atomicAdd(&ph[i], sh[i]);
}

__global__ __launch_bounds__(AB) void k_prior_bracket(AllocArgs a, const uint32_t *ph, double target)
{
    NewtonState *ns = reinterpret_cast<NewtonState *>(a.lo_hi);
    __shared__ double r0[AB], r1[AB];
    const int tid = threadIdx.x;
    double k = 0.0;
    for (int b = tid; b < PHB; b += AB) k += (double)ph[b];
    r0[tid] = k;
    __syncthreads();
    for (int o = AB / 2; o > 0; o >>= 1) {
        if (tid < o) r0[tid] += r0[tid + o];
        __syncthreads();
    }
    const double K = r0[0];   // vertices with a positive prior (exact below 2^53)
    __syncthreads();
    NewtonState st{};
    if (K <= target) {
        st.done = 1;   // S(0) = K <= T: C = 0
        st.C = 0.0;
    } else {
        // every prior is at most 1, so S and both bounds are at most
        // K e^-C, which reaches T at ln(K/T)
        double alo = 0.0, ahi = log(K / target), blo = 0.0, bhi = ahi;
        for (int it = 0; it < 36; ++it) {
            const double am = 0.5 * (alo + ahi), bm = 0.5 * (blo + bhi);
            double sa = 0.0, sb = 0.0;
            for (int b = tid; b < PHB; b += AB) {
                const uint32_t c = ph[b];
                if (!c) continue;
                double lo, up;
                prior_bin_edges(b, &lo, &up);
                if (lo > 0.0) sa += (double)c * exp(-am / lo);
                sb += (double)c * exp(-bm / up);
            }
            r0[tid] = sa;
            r1[tid] = sb;
            __syncthreads();
            for (int o = AB / 2; o > 0; o >>= 1) {
                if (tid < o) {
                    r0[tid] += r0[tid + o];
                    r1[tid] += r1[tid + o];
                }
                __syncthreads();
            }
            if (r0[0] > target) alo = am; else ahi = am;
            if (r1[0] > target) blo = bm; else bhi = bm;
            __syncthreads();
        }
        // S(alo) >= lower sum at alo > T, and S(bhi) <= upper sum at bhi <= T
        st.C = alo;
        st.lo = alo;
        st.hi = bhi;
        st.steps = 1;   // the count at C = 0 is done
    }
    if (tid == 0) *ns = st;
}

// Every point Newton's method or the bisection evaluates lies in the
// bracket, at C >= lo, and a prior p below lo / 750 gives exp(-C/p) below
// e^-750, which is zero in FP64 (the smallest subnormal is e^-744.4); its
// terms in S and M are exactly zero.  Such priors are dropped once: each
// workgroup packs the others of its segment, in vertex order, to
// packed[segment start ...] and stores their number.  On R-MAT 22 about
// 0.1 % of the vertices remain.
__global__ __launch_bounds__(AB) void k_prior_compact(AllocArgs a, int32_t chunk, double *packed, int32_t *cnt)
{
    const NewtonState *ns = reinterpret_cast<const NewtonState *>(a.lo_hi);
    __shared__ int32_t wsum[AB / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (ns->done) return;
    const double thr = ns->lo / 750.0;
    const int32_t beg = blockIdx.x * chunk, end = min(a.n, beg + chunk);
    // rounds of AB consecutive vertices (coalesced loads); within a round the
    // kept priors are packed in vertex order, rounds follow each other
    int32_t base = 0;
    for (int32_t r0 = beg; r0 < end; r0 += AB) {
        const int32_t v = r0 + tid;
        const double p = v < end ? a.dense_prior[v] : 0.0;
        const bool keep = p > 0.0 && p >= thr;
        const uint64_t m = __ballot(keep);
        if (lane == 0) wsum[w] = __popcll(m);
        __syncthreads();
        int32_t off = base + __popcll(m & ((1ull << lane) - 1));
        int32_t tot = 0;
        for (int i = 0; i < AB / 64; ++i) {
            if (i < w) off += wsum[i];
            tot += wsum[i];
        }
        if (keep) packed[beg + off] = p;
        base += tot;
        __syncthreads();
    }
    if (tid == 0) cnt[blockIdx.x] = base;
}

// Calibration priors are counts over tau0, so the sum over vertices is a
// sum over count values c of (vertices with count c) * exp(-mid tau0 / c).
// The whole bisection in one workgroup over the count histogram: per step,
// thread t sums bins t, t + HB, ... in turn, then a pairwise tree (a fixed
// order).  Same interval, step rule and stopping rule as the dense form.
constexpr int HB = 256;   // a workgroup small enough to find room beside the samplers
__global__ __launch_bounds__(HB) void k_alloc_bisect_hist(AllocArgs a, const uint32_t *hist, uint32_t top,
                                                          double target)
{
    __shared__ double red[HB];
    __shared__ unsigned long long kcount;
    const int tid = threadIdx.x;
    if (tid == 0) kcount = 0;
    __syncthreads();
    unsigned long long k = 0;
    for (uint32_t c = 1 + tid; c <= top; c += HB) k += hist[c];
    atomicAdd(&kcount, k);
    __syncthreads();
    const unsigned long long K = kcount;
    double lo = 0.0, hi = 0.0;
    if (K > 0) {
        hi = log((double)K / target);
        if (hi < 0.0) hi = 0.0;
    }
    for (int it = 0; it < 200 && K > 0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double sum = 0.0;
        for (uint32_t c = 1 + tid; c <= top; c += HB) {
            const uint32_t h = hist[c];
            if (h) sum = sum + (double)h * exp(-mid / ((double)c / a.tau0));
        }
        red[tid] = sum;
        __syncthreads();
        for (int o = HB / 2; o > 0; o >>= 1) {
            if (tid < o) red[tid] = red[tid] + red[tid + o];
            __syncthreads();
        }
        const double tot = red[0];
        __syncthreads();
        if (tot <= target) hi = mid; else lo = mid;
    }
    if (tid == 0) {
        a.lo_hi[0] = lo;
        a.lo_hi[1] = hi;
        a.lo_hi[2] = 1.0;
    }
}

__device__ __forceinline__ double alloc_L(const AllocArgs &a, double p, double C)
{
    const double floor_d = a.beta * a.delta / (4.0 * (double)a.n);
    double dv = floor_d;
    if (p > 0.0) dv = (1.0 - a.beta) * exp(-C / p) + floor_d;
    return -log(dv);
}

__global__ void k_alloc_delta(AllocArgs a, double C)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
        const double L = alloc_L(a, prior_of(a, v), C);
        a.LL[v] = L;
        if (a.LU != a.LL) a.LU[v] = L;
    }
}

// Calibration priors take the tau0 + 1 values c / tau0: L is computed once
// per count value (the same expression as for a dense prior) ...
__global__ void k_alloc_ltab(AllocArgs a, double C, uint32_t top, double *ltab)
{
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c <= top; c += gridDim.x * blockDim.x)
        ltab[c] = alloc_L(a, (double)c / a.tau0, C);
}

// ... and every vertex takes its count's value: a pass of 4 bytes read and
// 8 written per vertex instead of an exponential and a logarithm in FP64
// each, on the few CUs the samplers beside the calibration leave free.
__global__ void k_alloc_delta_counts(AllocArgs a, double C, uint32_t top, const double *ltab)
{
    constexpr int R = 8;   // vertices a thread per round, their loads in flight together
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < a.n; v0 += R * stride) {
        uint32_t c[R];
#pragma unroll
        for (int j = 0; j < R; ++j) c[j] = v0 + j * stride < a.n ? a.counts[v0 + j * stride] : 0u;
        double L[R];
#pragma unroll
        for (int j = 0; j < R; ++j) L[j] = c[j] <= top ? ltab[c[j]] : alloc_L(a, (double)c[j] / a.tau0, C);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t v = v0 + j * stride;
            if (v >= a.n) continue;
            a.LL[v] = L[j];
            if (a.LU != a.LL) a.LU[v] = L[j];
        }
    }
}

// ---- BFS sweeps for the vertex-diameter bracket (omega, Sec. III-A phase 1)

__global__ void k_argmax_degree(DevGraph g, unsigned long long *best)
{
    unsigned long long b = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const unsigned long long deg = (unsigned long long)(g.rp[v + 1] - g.rp[v]);
        // ties go to the smallest caller id
        const unsigned long long key = (deg << 32) | (0xFFFFFFFFull - (unsigned long long)g.orig[v]);
        b = key > b ? key : b;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(b, o);
        b = y > b ? y : b;
    }
    __shared__ unsigned long long s_b;   // one global atomic per workgroup
    if (threadIdx.x == 0) s_b = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicMax(&s_b, b);
    __syncthreads();
    if (threadIdx.x == 0 && s_b) atomicMax(best, s_b);
}

// Source of the next sweep, as an internal id in *src: the caller-smallest
// vertex of maximum degree (from k_argmax_degree's packed key) for the
// first sweep, else the caller-smallest vertex at the previous sweep's
// last depth (*far, a caller id, reset here for the sweep to come).  Also
// sets the frontier state for a frontier holding the source alone.
__global__ void k_bfs_source(DevGraph g, const unsigned long long *key, int32_t *far, int32_t *src,
                             int32_t *sizes)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int32_t caller = key ? (int32_t)(0xFFFFFFFFull - (*key & 0xFFFFFFFFull)) : *far;
    const int32_t v = g.newid[caller];
    *far = 0x7fffffff;
    *src = v;
    const int64_t d0 = g.rp[v + 1] - g.rp[v];
    for (int i = 0; i < 12; ++i) sizes[i] = 0;
    sizes[0] = 1;                                  // current frontier size
    sizes[5] = (int32_t)(uint32_t)(d0 & 0xffffffff);
    sizes[6] = (int32_t)(d0 >> 32);                // its degree sum
    sizes[10] = 1;                                 // listed
}

__global__ void k_bfs_init(int32_t n, int32_t *dist, const int32_t *src, int32_t *fr)
{
    const int32_t s0 = *src;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        dist[v] = (v == s0) ? 0 : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) fr[0] = s0;
}

// Smallest caller id among the vertices at the sweep's last depth (sz[3],
// which is also recorded as the sweep's eccentricity in *ecc).
__global__ void k_min_at_depth(int32_t n, const int32_t *dist, const int32_t *orig, const int32_t *sz,
                               int32_t *out, int32_t *ecc)
{
    const int32_t depth = sz[3];
    if (blockIdx.x == 0 && threadIdx.x == 0) *ecc = depth;
    int32_t b = 0x7fffffff;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (dist[v] == depth && orig[v] < b) b = orig[v];
    if (b != 0x7fffffff) atomicMin(out, b);
}

#define CK(expr)                                \
    do {                                        \
        hipError_t ck_ = (expr);                \
        if (ck_ != hipSuccess) return ck_;      \
    } while (0)

// Direction-optimising BFS for the bracket's sweeps, driven on the device:
// the host enqueues steps without waiting, and every kernel of a step reads
// the frontier's state from sz and does nothing when the step is not its
// case.  The frontier at depth k is listed in buf[k & 1] (when listed) and
// always marked in dist.
//   sz[0] frontier size      sz[1] next size        sz[2] frontier depth
//   sz[3] last nonempty depth sz[4] collect cursor  sz[5..6] frontier degree sum
//   sz[7] heavy rows         sz[8..9] next degree sum  sz[10] listed
//   sz[11] the frontier's bitmap is in bits[k & 1]
constexpr int32_t SMALL_V = 4096;         // single-workgroup levels: frontier size and
constexpr int64_t SMALL_D = 16384;        // degree sum at most these
constexpr int64_t HEAVY = 8192;           // top-down rows longer than this are split
constexpr int64_t PIECE = 4096;           // into pieces of this many entries
constexpr int SMALL_LONG = 2048;          // > SMALL_D / 33 rows longer than 32

__device__ __forceinline__ int64_t sz_get64(const int32_t *sz, int i)
{
    return ((int64_t)sz[i + 1] << 32) | (uint32_t)sz[i];
}

// A level goes bottom-up when its frontier is large in vertices or in
// adjacency entries (then most unreached vertices find a parent in the
// first few entries of their own rows).
struct BfsLim {
    int32_t big_v;   // frontier vertices
    int64_t big_e;   // frontier adjacency entries
};
__device__ __forceinline__ bool bfs_bottom_up(const int32_t *sz, BfsLim L)
{
    return sz[0] >= L.big_v || sz_get64(sz, 5) >= L.big_e;
}

// Small frontiers, many levels in one launch: one workgroup, a thread per
// frontier vertex for rows of up to 32 entries, a wave per longer row.
__global__ __launch_bounds__(1024) void k_bfs_small(DevGraph g, int32_t *dist, int32_t *buf0, int32_t *buf1,
                                                    int32_t *sz)
{
    __shared__ int32_t s_next, s_nlong;
    __shared__ unsigned long long s_deg;
    __shared__ int32_t s_long[SMALL_LONG];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    int32_t fsize = sz[0], depth = sz[2], last = sz[3];
    int64_t fdeg = sz_get64(sz, 5);
    if (fsize == 0 || sz[10] == 0 || fsize > SMALL_V || fdeg > SMALL_D) return;
    while (fsize > 0 && fsize <= SMALL_V && fdeg <= SMALL_D) {
        const int32_t *cur = (depth & 1) ? buf1 : buf0;
        int32_t *nxt = (depth & 1) ? buf0 : buf1;
        if (tid == 0) {
            s_next = 0;
            s_nlong = 0;
            s_deg = 0;
        }
        __syncthreads();
        unsigned long long dsum = 0;
        for (int32_t i = tid; i < fsize; i += blockDim.x) {
            const int32_t u = cur[i];
            const int64_t b = g.rp[u], e1 = g.rp[u + 1];
            if (e1 - b > 32) {
                const int32_t slot = atomicAdd(&s_nlong, 1);
                if (slot < SMALL_LONG) {
                    s_long[slot] = u;
                    continue;
                }
            }
            for (int64_t e = b; e < e1; ++e) {
                const int32_t w = g.ci[e];
                if (atomicCAS(&dist[w], -1, depth + 1) == -1) {
                    nxt[atomicAdd(&s_next, 1)] = w;
                    dsum += (unsigned long long)g.deg[w];
                }
            }
        }
        __syncthreads();
        const int32_t nl = min(s_nlong, SMALL_LONG);
        for (int32_t j = wid; j < nl; j += nw) {
            const int32_t u = s_long[j];
            for (int64_t e = g.rp[u] + lane; e < g.rp[u + 1]; e += 64) {
                const int32_t w = g.ci[e];
                if (atomicCAS(&dist[w], -1, depth + 1) == -1) {
                    nxt[atomicAdd(&s_next, 1)] = w;
                    dsum += (unsigned long long)g.deg[w];
                }
            }
        }
        if (dsum) atomicAdd(&s_deg, dsum);
        __syncthreads();
        fsize = s_next;
        fdeg = (int64_t)s_deg;
        depth += 1;
        if (fsize > 0) last = depth;
        __syncthreads();
    }
    if (tid == 0) {
        sz[0] = fsize;
        sz[1] = 0;
        sz[2] = depth;
        sz[3] = last;
        sz[5] = (int32_t)(uint32_t)(fdeg & 0xffffffff);
        sz[6] = (int32_t)(fdeg >> 32);
        sz[10] = 1;
        sz[11] = 0;
    }
}

// Position for a lane's append to a shared list: one atomic per wave (every
// lane of the wave must call; -1 for lanes that append nothing).
__device__ __forceinline__ int32_t wave_append(int32_t *ctr, bool pred)
{
    const uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(ctr, (int32_t)__popcll(m));
    base = __shfl(base, leader);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    return pred ? base + (int32_t)below : -1;
}

// Adds each thread's (count, degree sum) into sz[1] and sz[8..9] with one
// atomic pair per workgroup (every thread of the workgroup must call).
__device__ __forceinline__ void block_add_level(int32_t *sz, int cnt, unsigned long long dsum)
{
    __shared__ int s_cnt;
    __shared__ unsigned long long s_dsum;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_dsum = 0;
    }
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o);
        dsum += __shfl_xor(dsum, o);
    }
    if ((threadIdx.x & 63) == 0) {
        if (cnt) atomicAdd(&s_cnt, cnt);
        if (dsum) atomicAdd(&s_dsum, dsum);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_cnt) atomicAdd(&sz[1], s_cnt);
        if (s_dsum) atomicAdd((unsigned long long *)&sz[8], s_dsum);
    }
}

// List the frontier from dist when the previous level was bottom-up.
__global__ __launch_bounds__(1024) void k_bfs_collect(int32_t n, const int32_t *dist, int32_t *buf0, int32_t *buf1, int32_t *sz,
                              BfsLim lim)
{
    const int32_t fsize = sz[0], depth = sz[2];
    if (fsize == 0 || sz[10] != 0 || bfs_bottom_up(sz, lim)) return;
    int32_t *cur = (depth & 1) ? buf1 : buf0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // one global atomic per workgroup and sweep of the grid: waves take
    // their offsets in LDS, thread 0 reserves the workgroup's range (every
    // thread runs the same trip count)
    __shared__ int32_t s_wcnt[16], s_base;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t span = ((int64_t)n + step - 1) / step * step;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < span; v += step) {
        const bool hit = v < n && dist[v] == depth;
        const uint64_t m = __ballot(hit);
        if (lane == 0) s_wcnt[wid] = __popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t tot = 0;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
                const int32_t c = s_wcnt[i];
                s_wcnt[i] = tot;
                tot += c;
            }
            s_base = tot ? atomicAdd(&sz[4], tot) : 0;
        }
        __syncthreads();
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (hit) cur[s_base + s_wcnt[wid] + (int)below] = (int32_t)v;
        __syncthreads();
    }
}

// One top-down level: a wave per frontier vertex; rows longer than HEAVY
// are listed for k_bfs_heavy.
__global__ void k_bfs_td(DevGraph g, int32_t *dist, int32_t *buf0, int32_t *buf1, int32_t *heavy, int32_t *sz,
                         BfsLim lim)
{
    const int32_t fsize = sz[0], depth = sz[2];
    if (fsize == 0 || bfs_bottom_up(sz, lim)) return;
    const int32_t *cur = (depth & 1) ? buf1 : buf0;
    int32_t *nxt = (depth & 1) ? buf0 : buf1;
    const int lane = threadIdx.x & 63;
    const int32_t wpb = blockDim.x >> 6;
    unsigned long long dsum = 0;
    for (int32_t i = blockIdx.x * wpb + (threadIdx.x >> 6); i < fsize; i += gridDim.x * wpb) {
        const int32_t u = cur[i];
        const int64_t b = g.rp[u], e1 = g.rp[u + 1];
        if (e1 - b > HEAVY) {
            if (lane == 0) heavy[atomicAdd(&sz[7], 1)] = u;
            continue;
        }
        for (int64_t e0 = b; e0 < e1; e0 += 64) {   // wave-uniform trip count
            const int64_t e = e0 + lane;
            int32_t w = 0;
            bool claimed = false;
            if (e < e1) {
                w = g.ci[e];
                claimed = atomicCAS(&dist[w], -1, depth + 1) == -1;
            }
            const int32_t pos = wave_append(&sz[1], claimed);
            if (claimed) {
                nxt[pos] = w;
                dsum += (unsigned long long)g.deg[w];
            }
        }
    }
    block_add_level(sz, 0, dsum);
}

// The heavy rows of a top-down level, cut into pieces of PIECE entries that
// are dealt round-robin to the workgroups.  Rows are taken 256 at a time:
// every workgroup stages the same 256 rows with the prefix of their piece
// counts and then handles pieces blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ __launch_bounds__(256) void k_bfs_heavy(DevGraph g, int32_t *dist, const int32_t *heavy,
                                                   int32_t *buf0, int32_t *buf1, int32_t *sz, BfsLim lim)
{
    __shared__ int64_t s_beg[256], s_end[256], s_pre[257];
    __shared__ int64_t s_wsum[4];
    const int32_t fsize = sz[0], depth = sz[2], nh = sz[7];
    if (fsize == 0 || bfs_bottom_up(sz, lim) || nh == 0) return;
    int32_t *nxt = (depth & 1) ? buf0 : buf1;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    unsigned long long dsum = 0;
    for (int32_t h0 = 0; h0 < nh; h0 += 256) {
        int64_t b = 0, e1 = 0, pc = 0;
        if (h0 + tid < nh) {
            const int32_t u = heavy[h0 + tid];
            b = g.rp[u];
            e1 = g.rp[u + 1];
            pc = (e1 - b + PIECE - 1) / PIECE;
        }
        s_beg[tid] = b;
        s_end[tid] = e1;
        // inclusive scan of the piece counts
        int64_t x = pc;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wsum[wid] = x;
        __syncthreads();
        int64_t before = 0;
        for (int i = 0; i < wid; ++i) before += s_wsum[i];
        s_pre[tid + 1] = before + x;
        if (tid == 0) s_pre[0] = 0;
        __syncthreads();
        const int64_t total = s_pre[256];
        for (int64_t gp = blockIdx.x; gp < total; gp += gridDim.x) {
            int lo_i = 0, hi_i = 255;       // row r with s_pre[r] <= gp < s_pre[r + 1]
            while (lo_i < hi_i) {
                const int mid = (lo_i + hi_i + 1) >> 1;
                if (s_pre[mid] <= gp) lo_i = mid; else hi_i = mid - 1;
            }
            const int64_t pb = s_beg[lo_i] + (gp - s_pre[lo_i]) * PIECE;
            const int64_t pe = min(pb + PIECE, s_end[lo_i]);
            for (int64_t e0 = pb; e0 < pe; e0 += 256) {   // uniform trip count
                const int64_t e = e0 + tid;
                int32_t w = 0;
                bool claimed = false;
                if (e < pe) {
                    w = g.ci[e];
                    claimed = atomicCAS(&dist[w], -1, depth + 1) == -1;
                }
                const int32_t pos = wave_append(&sz[1], claimed);
                if (claimed) {
                    nxt[pos] = w;
                    dsum += (unsigned long long)g.deg[w];
                }
            }
        }
        __syncthreads();
    }
    block_add_level(sz, 0, dsum);
}

// Frontier bitmap of the current depth from dist (before a bottom-up level
// that follows a top-down one).  A wave covers 64 consecutive vertices and
// stores their bits as one word.
__global__ void k_bfs_mark(int32_t n, const int32_t *dist, uint64_t *bits0, uint64_t *bits1, int32_t *sz,
                           BfsLim lim)
{
    const int32_t fsize = sz[0], depth = sz[2];
    if (fsize == 0 || !bfs_bottom_up(sz, lim) || sz[11] != 0) return;
    uint64_t *cur = (depth & 1) ? bits1 : bits0;
    const int32_t nw = (n + 63) >> 6;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < 64ll * nw;
         v += (int64_t)gridDim.x * blockDim.x) {
        const bool in = v < n && dist[v] == depth;
        const uint64_t m = __ballot(in);
        if ((threadIdx.x & 63) == 0) cur[v >> 6] = m;
    }
}

// One bottom-up level: every unreached vertex looks for a neighbour in the
// frontier bitmap and stops at the first one; the new vertices' bits form
// the next bitmap.
__global__ void k_bfs_bu(DevGraph g, int32_t *dist, uint64_t *bits0, uint64_t *bits1, int32_t *sz, BfsLim lim)
{
    const int32_t fsize = sz[0], depth = sz[2];
    if (fsize == 0 || !bfs_bottom_up(sz, lim)) return;
    const uint64_t *cur = (depth & 1) ? bits1 : bits0;
    uint64_t *nxt = (depth & 1) ? bits0 : bits1;
    const int32_t nw = (g.n + 63) >> 6;
    int cnt = 0;
    unsigned long long dsum = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < 64ll * nw;
         v += (int64_t)gridDim.x * blockDim.x) {
        bool found = false;
        if (v < g.n && dist[v] == -1) {
            const int64_t b = g.rp[v], e1 = g.rp[v + 1];
            // eight probes in flight, then the first hit among them
            constexpr int B = 8;
            for (int64_t e0 = b; e0 < e1 && !found; e0 += B) {
                int32_t u[B];
#pragma unroll
                for (int j = 0; j < B; ++j) u[j] = (e0 + j < e1) ? g.ci[e0 + j] : -1;
                uint64_t wd[B];
#pragma unroll
                for (int j = 0; j < B; ++j) wd[j] = u[j] >= 0 ? cur[u[j] >> 6] : 0ull;
#pragma unroll
                for (int j = 0; j < B; ++j)
                    if (u[j] >= 0 && ((wd[j] >> (u[j] & 63)) & 1ull)) found = true;
            }
            if (found) {
                dist[v] = depth + 1;
                cnt += 1;
                dsum += (unsigned long long)(e1 - b);
            }
        }
        const uint64_t m = __ballot(found);
        if ((threadIdx.x & 63) == 0) nxt[v >> 6] = m;
    }
    block_add_level(sz, cnt, dsum);
}

// Close a level: the next frontier becomes the current one.
__global__ void k_bfs_advance(int32_t *sz, BfsLim lim)
{
    const int32_t fsize = sz[0];
    if (fsize == 0) return;
    const int32_t nsize = sz[1];
    sz[10] = bfs_bottom_up(sz, lim) ? 0 : 1;   // top-down listed the next frontier
    sz[11] = bfs_bottom_up(sz, lim) ? 1 : 0;   // bottom-up left its bitmap
    sz[0] = nsize;
    sz[1] = 0;
    sz[2] += 1;
    if (nsize > 0) sz[3] = sz[2];
    sz[4] = 0;
    sz[5] = sz[8];
    sz[6] = sz[9];
    sz[7] = 0;
    sz[8] = 0;
    sz[9] = 0;
}

// ---- exact vertex diameter (bound refinement on top of the sweeps above)

// Eccentricity bounds after a BFS from x (distances d, eccentricity e):
// every vertex v has max(d(v), e - d(v)) <= ecc(v) <= e + d(v).  Keeps the
// tightest bounds seen, and reduces over the vertices whose upper bound
// still exceeds lb (the diameter's lower bound): the largest upper bound
// (with the caller-smallest such vertex) and the smallest lower bound (with
// its caller-smallest vertex), packed into 64-bit keys.
__global__ void k_ecc_bounds(int32_t n, const int32_t *dist, int32_t e, int32_t *L, int32_t *U,
                             const int32_t *orig, int32_t lb, unsigned long long *keys)
{
    unsigned long long ku = 0, kl = ~0ull;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t d = dist[v];
        int32_t l = L[v], u = U[v];
        const int32_t lo = d > e - d ? d : e - d;
        l = lo > l ? lo : l;
        u = e + d < u ? e + d : u;
        L[v] = l;
        U[v] = u;
        if (u > lb) {
            const unsigned long long o = (unsigned long long)(uint32_t)orig[v];
            const unsigned long long a = ((unsigned long long)(uint32_t)u << 32) | (0xFFFFFFFFull - o);
            const unsigned long long b = ((unsigned long long)(uint32_t)l << 32) | o;
            ku = a > ku ? a : ku;
            kl = b < kl ? b : kl;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long x = __shfl_xor(ku, o), y = __shfl_xor(kl, o);
        ku = x > ku ? x : ku;
        kl = y < kl ? y : kl;
    }
    if ((threadIdx.x & 63) == 0) {
        if (ku) atomicMax(&keys[0], ku);
        if (kl != ~0ull) atomicMin(&keys[1], kl);
    }
}

__global__ void k_ecc_init(int32_t n, int32_t *L, int32_t *U)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        L[v] = 0;
        U[v] = 0x7fffffff;
    }
}

int grid_for(int64_t n, int block, int cap = 8192)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_merge_stop_impl(const DevGraph &g, uint32_t *c, uint32_t *sf0, uint32_t *sf1,
                                  const double *LL, const double *LU, double omega, double eps,
                                  unsigned long long cap, unsigned long long E, EpochState *es,
                                  unsigned long long *work_ctr, void *hist, int32_t hist_cap,
                                  HostStatus *hs, hipStream_t st, unsigned long long *pool_epoch, int pools,
                                  unsigned long long *defer_ctr, const uint32_t *lcnt, const double *ltab)
{
    // At most 256 workgroups: the merge runs while sampler workgroups hold
    // the CUs, and each of its workgroups waits for a slot that one of them
    // gives up; fewer, longer workgroups finish the merge sooner there.
    hipLaunchKernelGGL(k_merge_stop, dim3(grid_for(g.n, MB, 256)), dim3(MB), 0, st, g.n, c, sf0, sf1,
                       LL, LU, omega, eps, cap, E, es, work_ctr, (EpochHist *)hist, hist_cap, hs, pool_epoch,
                       pools, defer_ctr, lcnt, ltab);
    return hipGetLastError();
}

size_t epoch_hist_bytes() { return sizeof(EpochHist); }

hipError_t launch_fg(int32_t n, const uint32_t *c, double tau, const double *LL, const double *LU,
                     double omega, double *f, double *g, hipStream_t st)
{
    hipLaunchKernelGGL(k_fg, dim3(grid_for(n, 256)), dim3(256), 0, st, n, c, tau, LL, LU, omega, f, g);
    return hipGetLastError();
}

hipError_t launch_btilde(int32_t n, const uint32_t *c, double tau, double *b, hipStream_t st)
{
    hipLaunchKernelGGL(k_btilde, dim3(grid_for(n, 256)), dim3(256), 0, st, n, c, tau, b);
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, uint64_t stream, uint64_t first, uint32_t count,
                         uint32_t nwords, uint64_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_philox, dim3((count + 255) / 256), dim3(256), 0, st, seed, stream, first, count,
                       nwords, out);
    return hipGetLastError();
}

hipError_t run_alloc(const AllocArgs &a, hipStream_t st, double *C_host)
{
    hipError_t e;
    const double target = 0.25 * a.delta * (1.0 - 1e-9);
    if (a.counts) {
        // calibration counts: the bisection in one launch over the histogram
        // of the counts that the calibration's sampler kept
        if (!a.hist) return hipErrorInvalidValue;
        const uint32_t top = (uint32_t)std::max(1.0, a.tau0);
        hipLaunchKernelGGL(k_alloc_bisect_hist, dim3(1), dim3(HB), 0, st, a, a.hist, top, target);
        double fin[3];
        CK(hipMemcpyAsync(fin, a.lo_hi, sizeof(fin), hipMemcpyDeviceToHost, st));
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        const double C = fin[1];
        if (a.ltab) {
            hipLaunchKernelGGL(k_alloc_ltab, dim3(grid_for((int64_t)top + 1, 256, 64)), dim3(256), 0, st, a, C, top,
                               a.ltab);
            if (!a.lazy)
                hipLaunchKernelGGL(k_alloc_delta_counts, dim3(grid_for(a.n, 256, 256)), dim3(256), 0, st, a, C, top,
                                   a.ltab);
        } else {
            hipLaunchKernelGGL(k_alloc_delta, dim3(grid_for(a.n, 256, 256)), dim3(256), 0, st, a, C);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        *C_host = C;
        return hipSuccess;
    }
    // dense prior: the histogram bracket, then Newton's method on ln S
    // (k_alloc_newton), a launch per step, the state read back after 5
    // steps and then every 3
    // (LL, written only once C is known, holds the compacted priors until then)
    const int32_t chunk = 8192;
    const int32_t nseg = (a.n + chunk - 1) / chunk;
    uint32_t *ph = reinterpret_cast<uint32_t *>(a.partials + 2 * (size_t)nseg + 2);
    int32_t *seg_cnt = reinterpret_cast<int32_t *>(ph + PHB + 1);
    CK(launch_zero_words(ph, PHB, st));
    hipLaunchKernelGGL(k_prior_hist, dim3(grid_for(a.n, 256, 2048)), dim3(256), 0, st, a, ph);
    hipLaunchKernelGGL(k_prior_bracket, dim3(1), dim3(AB), 0, st, a, (const uint32_t *)ph, target);
    hipLaunchKernelGGL(k_prior_compact, dim3(nseg), dim3(AB), 0, st, a, chunk, a.LL, seg_cnt);
    const int32_t spb = (nseg + 255) / 256, nb = (nseg + spb - 1) / spb;
    NewtonState fin{};
    for (int it = 0; it < 400 && !fin.done; ++it) {
        hipLaunchKernelGGL(k_alloc_newton, dim3(nb), dim3(AB), 0, st, a, (const double *)a.LL,
                           (const int32_t *)seg_cnt, nseg, chunk, spb, target);
        if (it == 4 || (it > 4 && (it - 4) % 3 == 0)) {
            CK(hipMemcpyAsync(&fin, a.lo_hi, sizeof(fin), hipMemcpyDeviceToHost, st));
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        }
    }
    if (!fin.done) return hipErrorUnknown;
    const double C = fin.C;
    hipLaunchKernelGGL(k_alloc_delta, dim3(grid_for(a.n, 256)), dim3(256), 0, st, a, C);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    *C_host = C;
    return hipSuccess;
}

// S and M per workgroup, the prior histogram (PHB 4-byte bins, one spare),
// the retained priors per 8192-vertex segment
size_t alloc_partials(int32_t n)
{
    const size_t nseg = (size_t)((n + 8191) / 8192);
    return 2 * nseg + 2 + (PHB + 1) / 2 + (nseg + 1) / 2 + 1;
}

hipError_t run_alloc_L(const AllocArgs &a, double C, hipStream_t st)
{
    const uint32_t top = (uint32_t)std::max(1.0, a.tau0);
    hipLaunchKernelGGL(k_alloc_delta_counts, dim3(grid_for(a.n, 256)), dim3(256), 0, st, a, C, top, a.ltab);
    return hipGetLastError();
}

namespace {
// Budget check of an allocation: per workgroup, the sum of delta_L + delta_U
// over its vertices (Kahan per thread, then a pairwise tree), and a flag for
// any L that is not finite and positive.
constexpr int CB = 256;
__global__ __launch_bounds__(CB) void k_alloc_check(int32_t n, const double *LL, const double *LU,
                                                    double *partial, int32_t *bad)
{
    __shared__ double sh[CB];
    double sum = 0.0, comp = 0.0;
    int flag = 0;
    for (int32_t v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        const double a = LL[v], b = LU[v];
        if (!(a > 0.0) || !(b > 0.0) || !isfinite(a) || !isfinite(b)) flag = 1;
        const double x = exp(-a) + exp(-b);
        const double y = x - comp;
        const double t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    if (flag) atomicOr(bad, 1);
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int o = CB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}
}  // namespace

hipError_t alloc_budget(int32_t n, const double *LL, const double *LU, hipStream_t st, double *sum_out,
                        bool *finite_out)
{
    hipError_t e;
    const int nb = grid_for(n, CB, 1024);
    double *part = nullptr;
    int32_t *bad = nullptr;
    if ((e = hipMallocAsync((void **)&part, sizeof(double) * nb, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&bad, sizeof(int32_t), st)) != hipSuccess) return e;
    CK(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_alloc_check, dim3(nb), dim3(CB), 0, st, n, LL, LU, part, bad);
    std::vector<double> hp(nb);
    int32_t hb = 0;
    CK(hipMemcpyAsync(hp.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    CK(hipFreeAsync(part, st));
    CK(hipFreeAsync(bad, st));
    double sum = 0.0, comp = 0.0;
    for (int i = 0; i < nb; ++i) {
        const double y = hp[i] - comp;
        const double t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    *sum_out = sum;
    *finite_out = hb == 0;
    return hipSuccess;
}

// Buffers of the BFS sweeps.
struct BfsBufs {
    int32_t *dist0 = nullptr, *dist1 = nullptr, *fa = nullptr, *fb = nullptr, *heavy = nullptr, *sizes = nullptr;
    int32_t *pick = nullptr;   // {source (internal id), next source (caller id), ecc x 6}
    uint64_t *bits0 = nullptr, *bits1 = nullptr;
    unsigned long long *best = nullptr;
    BfsLim lim;
    int64_t sweeps = 0;
};

static hipError_t bfs_alloc(const DevGraph &g, hipStream_t st, BfsBufs &b, bool two_dists)
{
    hipError_t e;
    const int32_t n = g.n;
    const size_t nwords = ((size_t)n + 63) / 64;
    if ((e = hipMallocAsync((void **)&b.dist0, sizeof(int32_t) * n, st)) != hipSuccess) return e;
    if (two_dists && (e = hipMallocAsync((void **)&b.dist1, sizeof(int32_t) * n, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.fa, sizeof(int32_t) * n, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.fb, sizeof(int32_t) * (size_t)n, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.heavy, sizeof(int32_t) * (size_t)n, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.bits0, sizeof(uint64_t) * nwords, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.bits1, sizeof(uint64_t) * nwords, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.sizes, sizeof(int32_t) * 12, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.best, sizeof(unsigned long long), st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&b.pick, sizeof(int32_t) * 8, st)) != hipSuccess) return e;
    b.lim.big_v = std::max<int32_t>(n / 16, 1 << 14);
    b.lim.big_e = std::max<int64_t>(g.nnz / 16, (int64_t)1 << 20);
    return hipSuccess;
}

static hipError_t bfs_free(BfsBufs &b, hipStream_t st)
{
    void *ps[] = {b.dist0, b.dist1, b.fa, b.fb, b.heavy, b.bits0, b.bits1, b.sizes, b.best, b.pick};
    for (void *p : ps)
        if (p) CK(hipFreeAsync(p, st));
    return hipSuccess;
}

// One sweep into `dist`: from the vertex of the packed key (the largest
// degree) when `key` is set, else from the caller id in pick[1].  Leaves
// the caller-smallest vertex at the last depth in pick[1] and the
// eccentricity in pick[2 + slot] and *ecc.  `hint`: a lower bound on the
// eccentricity, used to size the first batch of steps.
static hipError_t bfs_sweep(const DevGraph &g, hipStream_t st, BfsBufs &b, int32_t *dist,
                            const unsigned long long *key, int slot, int32_t hint, int32_t *ecc)
{
    const int32_t n = g.n;
    hipLaunchKernelGGL(k_bfs_source, dim3(1), dim3(1), 0, st, g, key, b.pick + 1, b.pick, b.sizes);
    hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(n, 256)), dim3(256), 0, st, n, dist, b.pick, b.fa);
    // Batches of steps enqueued without waiting (a step may run many small
    // levels); the host only looks at the frontier size between batches.
    // A step past the last level does nothing but still costs its launches.
    int32_t hs[4] = {1, 0, 0, 0};
    int32_t batch = key ? 8 : std::min<int32_t>(std::max<int32_t>(hint + 2, 2), 16);
    for (int64_t steps = 0; steps <= (int64_t)n + 1; steps += batch, batch = key ? 4 : 2) {
        for (int k = 0; k < batch; ++k) {
            hipLaunchKernelGGL(k_bfs_small, dim3(1), dim3(1024), 0, st, g, dist, b.fa, b.fb, b.sizes);
            hipLaunchKernelGGL(k_bfs_collect, dim3(grid_for(n, 1024, 1024)), dim3(1024), 0, st, n, dist, b.fa,
                               b.fb, b.sizes, b.lim);
            hipLaunchKernelGGL(k_bfs_td, dim3(2048), dim3(256), 0, st, g, dist, b.fa, b.fb, b.heavy, b.sizes, b.lim);
            hipLaunchKernelGGL(k_bfs_heavy, dim3(1024), dim3(256), 0, st, g, dist, b.heavy, b.fa, b.fb, b.sizes,
                               b.lim);
            hipLaunchKernelGGL(k_bfs_mark, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, n, dist, b.bits0,
                               b.bits1, b.sizes, b.lim);
            hipLaunchKernelGGL(k_bfs_bu, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, g, dist, b.bits0,
                               b.bits1, b.sizes, b.lim);
            hipLaunchKernelGGL(k_bfs_advance, dim3(1), dim3(1), 0, st, b.sizes, b.lim);
        }
        CK(hipMemcpyAsync(hs, b.sizes, sizeof(hs), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        if (hs[0] == 0) break;
    }
    if (hs[0] != 0) return hipErrorUnknown;   // more levels than vertices: cannot happen
    hipLaunchKernelGGL(k_min_at_depth, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, n, dist, g.orig, b.sizes,
                       b.pick + 1, b.pick + 2 + slot);
    *ecc = hs[3];
    b.sweeps += 1;
    return hipGetLastError();
}

// A sampler's BFS arrays, kept from one bracket to the next: freeing them
// after each run released their pages (1.2 ms a run on R-MAT 26, in the
// runtime's free).
struct BfsCache {
    BfsBufs b;
    bool ready = false;
};

BfsCache *bfs_cache_create() { return new BfsCache(); }

void bfs_cache_free(BfsCache *c, hipStream_t st)
{
    if (!c) return;
    if (c->ready) {
        (void)bfs_free(c->b, st);
        (void)hipStreamSynchronize(st);
    }
    delete c;
}

hipError_t device_vd_bracket(const DevGraph &g, hipStream_t st, int64_t *vd_lo, int64_t *vd_hi, BfsCache *cache)
{
    hipError_t e;
    const int32_t n = g.n;
    BfsBufs local;
    if (cache && !cache->ready) {
        if ((e = bfs_alloc(g, st, cache->b, false)) != hipSuccess) return e;
        cache->ready = true;
    }
    BfsBufs &b = cache ? cache->b : local;
    if (!cache && (e = bfs_alloc(g, st, b, false)) != hipSuccess) return e;
    CK(hipMemsetAsync(b.best, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_argmax_degree, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, g, b.best);
    // Three sweeps: from the vertex of largest degree r, from its farthest
    // vertex a, from a's farthest b; each source is picked on the device.
    int32_t er = 0, ea = 0, eb = 0;
    if ((e = bfs_sweep(g, st, b, b.dist0, b.best, 0, 0, &er)) != hipSuccess) return e;
    if ((e = bfs_sweep(g, st, b, b.dist0, nullptr, 1, er, &ea)) != hipSuccess) return e;
    if ((e = bfs_sweep(g, st, b, b.dist0, nullptr, 2, er, &eb)) != hipSuccess) return e;
    const int32_t lb = ea > eb ? ea : eb;
    int32_t mn = er < ea ? er : ea;
    mn = eb < mn ? eb : mn;
    *vd_lo = (int64_t)lb + 1;
    *vd_hi = 2 * (int64_t)mn + 1;
    if (!cache) CK(bfs_free(b, st));
    CK(hipStreamSynchronize(st));
    return hipGetLastError();
}

static double omega_of_vd(int64_t vd, double eps, double delta)
{
    double lg = 0.0;
    if (vd - 2 >= 1) {
        int64_t x = vd - 2, fl = 0;
        while (x > 1) { x >>= 1; ++fl; }
        lg = (double)fl;
    }
    return 0.5 / (eps * eps) * (lg + 1.0 + log(2.0 / delta));
}

// Exact vertex diameter by bound refinement on eccentricities, the
// BFS-based family of exact diameter algorithms the paper's diameter phase
// uses (Borassi et al.; the refinement is Takes and Kosters'): every BFS
// from x gives max(d, e - d) <= ecc(v) <= e + d for every vertex v, the
// largest eccentricity found is a lower bound lb of the diameter and the
// largest upper bound among the vertices is an upper bound.  The first
// three sources are the bracket's sweeps; then the sources alternate
// between the vertex of smallest lower bound (a central vertex, whose BFS
// tightens many upper bounds) and the vertex of largest upper bound, among
// the vertices whose upper bound still exceeds lb (ties: the smallest
// caller id).  With omega_only the search stops as soon as both ends of
// the bracket give the same omega (eps, delta).  Stops with a bracket after
// max_bfs BFS runs (graphs with many vertices of near-diametral
// eccentricity, as random hyperbolic graphs, need very many).
hipError_t device_exact_vd(const DevGraph &g, hipStream_t st, bool omega_only, double eps, double delta,
                           int64_t max_bfs, int64_t *vd_lo, int64_t *vd_hi, int32_t *witness, int64_t *bfs_runs)
{
    hipError_t e;
    const int32_t n = g.n;
    BfsBufs b;
    if ((e = bfs_alloc(g, st, b, true)) != hipSuccess) return e;
    int32_t *Lb = b.dist1, *Ub = nullptr;
    unsigned long long *keys = nullptr;
    if ((e = hipMallocAsync((void **)&Ub, sizeof(int32_t) * (size_t)n, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&keys, 2 * sizeof(unsigned long long), st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ecc_init, dim3(grid_for(n, 256)), dim3(256), 0, st, n, Lb, Ub);
    CK(hipMemsetAsync(b.best, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_argmax_degree, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, g, b.best);
    int64_t lo = 0, hi = INT64_MAX;
    int32_t wit = 0, hint = 0, r_int = 0;
    int32_t hp[8];
    auto settled = [&]() {
        return lo >= hi || (omega_only && omega_of_vd(lo + 1, eps, delta) == omega_of_vd(hi + 1, eps, delta));
    };
    for (int64_t it = 0; it < max_bfs; ++it) {
        // source: the largest degree, then the two sweeps, then the bounds
        int32_t src_caller = -1;
        if (it >= 3) {
            unsigned long long hk[2];
            CK(hipMemcpyAsync(hk, keys, sizeof(hk), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
            if (it % 2 == 1) src_caller = (int32_t)(hk[1] & 0xFFFFFFFFull);           // smallest lower bound
            else src_caller = (int32_t)(0xFFFFFFFFull - (hk[0] & 0xFFFFFFFFull));    // largest upper bound
            CK(hipMemcpyAsync(b.pick + 1, &src_caller, sizeof(src_caller), hipMemcpyHostToDevice, st));
        } else if (it > 0) {
            CK(hipMemcpyAsync(hp, b.pick, sizeof(hp), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
            src_caller = hp[1];   // the previous sweep's farthest vertex
        }
        int32_t ecc = 0;
        if ((e = bfs_sweep(g, st, b, b.dist0, it == 0 ? b.best : nullptr, it < 3 ? (int)it : 3, hint, &ecc)) !=
            hipSuccess)
            return e;
        if (it == 0) {
            CK(hipMemcpyAsync(hp, b.pick, sizeof(hp), hipMemcpyDeviceToHost, st));
            CK(hipStreamSynchronize(st));
            hint = ecc;
            r_int = hp[0];
        }
        if (ecc > lo) {
            lo = ecc;
            wit = src_caller;   // -1: the first source, resolved below
        }
        const unsigned long long init[2] = {0ull, ~0ull};
        CK(hipMemcpyAsync(keys, init, sizeof(init), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_ecc_bounds, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, n, b.dist0, ecc, Lb, Ub,
                           g.orig, (int32_t)lo, keys);
        unsigned long long hk[2];
        CK(hipMemcpyAsync(hk, keys, sizeof(hk), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        hi = hk[0] ? std::max<int64_t>(lo, (int64_t)(hk[0] >> 32)) : lo;
        if (settled()) break;
    }
    if (wit < 0) {   // the vertex of largest degree: the first sweep's source
        CK(hipMemcpyAsync(&wit, g.orig + r_int, 4, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
    }
    *vd_lo = lo + 1;
    *vd_hi = hi + 1;
    if (witness) *witness = wit;
    if (bfs_runs) *bfs_runs = b.sweeps;
    CK(hipFreeAsync(Ub, st));
    CK(hipFreeAsync(keys, st));
    CK(bfs_free(b, st));
    CK(hipStreamSynchronize(st));
    return hipGetLastError();
}

}  // namespace kad
