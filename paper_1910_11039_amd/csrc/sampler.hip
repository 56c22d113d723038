// KADABRA sampler kernel for gfx950: one sample per workgroup at a time,
// persistent workgroups pulling sample indices from a device counter.
//
// One sample (Sec. III-A): draw an ordered pair s != t, run a bidirectional
// BFS that counts shortest paths, choose one shortest s-t path uniformly,
// add one to the counter of each interior vertex.
//
// Search rules (readings; the paper only names a bidirectional BFS):
//  * grow the side whose newest layer has the smaller degree sum (ties: s);
//    each step adds the whole next layer as a set;
//  * the search meets when the new layer of side X contains vertices already
//    reached by side Y; those form the meet set M, all in Y's newest layer;
//  * sigma of a layer is the sum of sigma over its predecessors; it is taken
//    for every layer that gets expanded (while expanding it) and for M;
//  * integer mode: uint64 sums with exact overflow detection; on overflow
//    the whole sample is redone in FP mode; FP mode: FP64 sums in ascending
//    CSR position, each layer rescaled by 2^-400 when its maximum exceeds
//    2^400;
//  * the meet vertex is chosen in ascending id with weight sigma_X * sigma_Y,
//    predecessors in CSR order with weight sigma, walking to s first, then
//    to t; each pick is the first candidate whose inclusive prefix sum
//    exceeds the draw scaled to the total (one draw per pick).
//
// Data layout (HBM): per slot, Rec[n] (16 B: stamp, state, sigma), a
// frontier queue int32[n] (side s grows from the front, side t from the
// back; the two sides never share a vertex outside M) and a meet list
// int32[n].  Records carry the slot's sample stamp, so nothing is cleared
// between samples.
//
// Expansion (integer mode) is edge-parallel and load-balanced: a chunk of
// up to BS frontier vertices is staged in LDS with the exclusive scan of
// their degrees, every lane takes four adjacency entries at a time, finds
// their owners by binary search in LDS, and sigma contributions go to
// per-owner LDS accumulators.  New frontier entries are compacted with a
// wave ballot and mbcnt prefix, one LDS atomic per wave.  A step likely to
// meet is first scanned without claiming (the new layer of a step that
// meets is never used), and an LDS bit filter of the vertices the sample
// has reached lets that scan skip most entries without reading their
// records.  FP mode is vertex-parallel so that every sum runs in CSR order
// in one lane.
#include "kad_internal.h"
#include "philox.h"

namespace kad {
namespace {

constexpr int MCAP = 1024;                 // meet sets up to this size are ranked in LDS
constexpr int LMAX = 30;                   // layers whose queue offsets are kept in LDS
constexpr int MEDGE = 1024;                // meet edges of one frontier chunk folded in LDS

// Bit filter of the vertices a sample has reached: bit (v mod its size) is
// set whenever v is claimed.  A clear bit proves v unreached, so a probe
// scan skips that entry without reading its record.  Sized so that the
// workgroups meant to share a CU fit its LDS: 64 KiB at 1024 threads (one
// per CU), 32 KiB at 512 (two), 8 KiB at 256 (three).
template <int BS>
struct Filter {
    static constexpr int WORDS = (BS >= 1024) ? 16384 : (BS == 512 ? 8192 : (BS == 256 ? 2048 : 1024));
    static constexpr uint32_t MASK = (uint32_t)WORDS * 32u - 1u;
};
constexpr double BIG = 0x1p400;
constexpr double SHRINK = 0x1p-400;
constexpr uint32_t X_SHIFT = 31;

__device__ __forceinline__ uint64_t ld_key(Rec *r)
{
    return __hip_atomic_load(reinterpret_cast<uint64_t *>(r), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool cas_key(Rec *r, uint64_t expect, uint64_t desired)
{
    return __hip_atomic_compare_exchange_strong(reinterpret_cast<uint64_t *>(r), &expect, desired,
                                                __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t or_state(Rec *r, uint32_t bits)
{
    return __hip_atomic_fetch_or(&r->state, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_key(Rec *r, uint64_t v)
{
    __hip_atomic_store(reinterpret_cast<uint64_t *>(r), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t ld_sig(Rec *r)
{
    return __hip_atomic_load(&r->sig, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_sig(Rec *r, uint64_t v)
{
    __hip_atomic_store(&r->sig, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ double as_f64(uint64_t b) { return __builtin_bit_cast(double, b); }
__device__ __forceinline__ uint64_t as_u64(double d) { return __builtin_bit_cast(uint64_t, d); }
__device__ __forceinline__ double unit53(uint64_t u) { return (double)(u >> 11) * 0x1p-53; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int BS>
__device__ __forceinline__ bool filt_test(const uint32_t *f, int32_t v)
{
    const uint32_t b = (uint32_t)v & Filter<BS>::MASK;
    return (f[b >> 5] >> (b & 31)) & 1u;
}
template <int BS>
__device__ __forceinline__ void filt_set(uint32_t *f, int32_t v)
{
    const uint32_t b = (uint32_t)v & Filter<BS>::MASK;
    atomicOr(&f[b >> 5], 1u << (b & 31));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    return v;
}

template <int BS>
struct Smem {
    struct {
        int32_t u[BS];
        int64_t rs[BS];
        int64_t off[BS];
        unsigned long long acc[BS];
        unsigned long long acc2[BS];
    } e;
    struct {
        int32_t id[MCAP];
        unsigned long long w[MCAP];    // sigma_X accumulators, then the meet weights
        unsigned long long w2[MCAP];   // sigma_Y accumulators
    } m;
    int64_t wsum[BS / 64];
    unsigned long long nextdeg;
    unsigned long long sigst;
    unsigned long long fmax_bits;
    unsigned long long sid;
    int64_t sdeg[2], psdeg[2];
    int32_t lo[2], hi[2], dep[2], plo[2], phi[2];
    int32_t loff[2][LMAX + 2];   // layer j of a side = queue positions [loff[j], loff[j+1])
    int32_t me_a[MEDGE];         // meet edges of the current chunk: owner index in the chunk,
    int32_t me_w[MEDGE];         // and the meet vertex
    uint32_t filt[Filter<BS>::WORDS];
    int32_t tail, mcount, ovf, err, w, wmin, mpath, nme, fold_bad, pathc, vsfull, quit;
    const int32_t *stopp;   // the run's stop flag (null: none); kept here, not in registers
    uint32_t stamp;
    int32_t s, t;
};

// Exclusive block scan of int64 values (all threads must call).
template <int BS>
__device__ int64_t block_excl_scan(Smem<BS> &sm, int64_t v, int64_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sm.wsum[wid] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) {
        int64_t s = sm.wsum[i];
        pre += (i < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Sum of one uint64 per thread over the workgroup (all threads call; all get it).
template <int BS>
__device__ uint64_t block_sum_u64(Smem<BS> &sm, uint64_t v)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum_u64(v);
    if (lane == 0) sm.wsum[wid] = (int64_t)v;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) tot += (uint64_t)sm.wsum[i];
    __syncthreads();
    return tot;
}

struct Ctx {
    DevGraph g;
    Rec *R;                     // dense: one record per vertex; sparse: the slot's table
    int32_t *Q;
    int32_t *MB;
    unsigned long long *gacc;   // the slot's meet accumulators: sigma_X, then sigma_Y
    int32_t macc_cap;           // meet positions each of the two holds
    uint32_t cur;
    int fp;
    int32_t qn;                 // capacity of the queue and the meet list (dense: n)
    uint32_t cur16;             // sparse: the stamp as stored in the table
    uint32_t hshift;            // sparse: 64 - log2(table size)
    uint32_t mask;              // sparse: table size - 1
    int32_t claim_limit;        // sparse: vertices a sample may claim (table load <= 0.75)
    int *err;                   // the launch's error word
};

__device__ __forceinline__ int64_t qpos(int32_t n, int side, int64_t p)
{
    return side ? (int64_t)n - 1 - p : p;
}

// ---- visited state.  Dense: record v of the slot's array (key = stamp << 32
// | state).  Sparse: an open-addressing table per slot with linear probing,
// whose buckets have the record layout but a key word packed as
//   stamp (16 bits) | side | meet | depth (15 bits) | vertex (31 bits);
// a bucket whose stamp is not the sample's is free, so runs of the
// sample's buckets end at a free one and a sample never clears its table
// (only when the 16-bit stamp wraps).  The functions below return keys in
// the dense layout (stamp << 32 | state, 0 for a vertex not reached) and a
// record index ri (dense: the vertex; sparse: its bucket), so the search
// code is the same for both.  A sample claims at most claim_limit vertices
// (the table stays at most 3/4 full, so every probe run ends); a sample
// that would claim more, or reach a depth of 2^15, is handed to the dense
// fallback.
constexpr uint32_t SP_DEPTH_MAX = (1u << 15) - 1;

__device__ __forceinline__ uint64_t sp_pack(uint32_t cur16, uint32_t state, int32_t v)
{
    return ((uint64_t)cur16 << 48) | ((uint64_t)(state >> 30) << 46) | ((uint64_t)(state & 0x7fffu) << 31) |
           (uint64_t)(uint32_t)v;
}
__device__ __forceinline__ uint32_t sp_state(uint64_t k)
{
    return (((uint32_t)(k >> 46) & 3u) << 30) | (uint32_t)((k >> 31) & 0x7fffu);
}
__device__ __forceinline__ bool sp_live(const Ctx &c, uint64_t k) { return (uint32_t)(k >> 48) == c.cur16; }
__device__ __forceinline__ int32_t sp_vid(uint64_t k) { return (int32_t)(k & 0x7fffffffu); }
__device__ __forceinline__ uint32_t sp_home(const Ctx &c, int32_t v)
{
    return (uint32_t)(((uint64_t)(uint32_t)v * 0x9E3779B97F4A7C15ull) >> c.hshift);
}

// Key of v (dense layout) and its record index, continuing a probe run from
// bucket b whose key k0 has already been loaded (sparse).
template <bool SP>
__device__ __forceinline__ uint64_t vs_resolve(const Ctx &c, int32_t v, uint32_t b, uint64_t k0, int64_t &ri)
{
    uint64_t k = k0;
    for (;;) {
        if (!sp_live(c, k)) { ri = -1; return 0ull; }
        if (sp_vid(k) == v) { ri = b; return ((uint64_t)c.cur << 32) | sp_state(k); }
        b = (b + 1) & c.mask;
        k = ld_key(c.R + b);
    }
}

template <bool SP>
__device__ __forceinline__ uint64_t vs_key(const Ctx &c, int32_t v, int64_t &ri)
{
    if (!SP) {
        ri = v;
        return ld_key(c.R + v);
    }
    const uint32_t b = sp_home(c, v);
    return vs_resolve<SP>(c, v, b, ld_key(c.R + b), ri);
}

// Record index of a vertex the sample has reached (error 5, and bucket 0,
// if the table does not hold it: never, short of a defect).
template <bool SP>
__device__ __forceinline__ int64_t vs_index(const Ctx &c, int32_t v)
{
    int64_t ri;
    (void)vs_key<SP>(c, v, ri);
    if (SP && ri < 0) {
        *c.err = 5;
        ri = 0;
    }
    return ri;
}

// Claims v with key `desired` (dense layout) unless the sample has reached
// it; `seen` is the key the caller loaded (dense: the compare value).
template <bool SP>
__device__ __forceinline__ bool vs_claim(const Ctx &c, int32_t v, uint64_t seen, uint64_t desired, int64_t &ri)
{
    if (!SP) {
        ri = v;
        return cas_key(c.R + v, seen, desired);
    }
    const uint64_t nk = sp_pack(c.cur16, (uint32_t)desired, v);
    uint32_t b = sp_home(c, v);
    uint64_t k = ld_key(c.R + b);
    for (;;) {
        if (sp_live(c, k)) {
            if (sp_vid(k) == v) { ri = b; return false; }
            b = (b + 1) & c.mask;
            k = ld_key(c.R + b);
            continue;
        }
        uint64_t expect = k;
        if (__hip_atomic_compare_exchange_strong(reinterpret_cast<uint64_t *>(c.R + b), &expect, nk,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP)) {
            ri = b;
            return true;
        }
        k = expect;   // the bucket was taken meanwhile: look at it again
    }
}

// Sets the meet bit; returns the previous state (dense layout).
template <bool SP>
__device__ __forceinline__ uint32_t vs_or_meet(const Ctx &c, int64_t ri)
{
    if (!SP) return or_state(c.R + ri, MEET_BIT);
    const uint64_t old = __hip_atomic_fetch_or(reinterpret_cast<uint64_t *>(c.R + ri), 1ull << 46,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return sp_state(old);
}

// A root of the search (s or t) with key `key` (dense layout).
template <bool SP>
__device__ __forceinline__ int64_t vs_root(const Ctx &c, int32_t v, uint64_t key)
{
    if (!SP) {
        st_key(c.R + v, key);
        return v;
    }
    int64_t ri;
    (void)vs_claim<SP>(c, v, 0ull, key, ri);
    return ri;
}

// Vertices the sample has claimed so far (both queues), read while other
// waves of the workgroup keep appending to X's queue.
template <int BS>
__device__ __forceinline__ int32_t claimed_now(Smem<BS> &sm, int X)
{
    return __hip_atomic_load(&sm.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) + sm.hi[1 - X];
}

// Thread-local statistics, flushed once per workgroup.
struct LocalStats {
    unsigned long long pred, visited;
};

// One expansion of side X from its layer k (frontier = queue positions
// [lo, hi)).  Discovered vertices are appended from position hi on; meet
// vertices go to the meet list.  Computes sigma for layer k (k >= 1).
// With `probe` set nothing is claimed: the scan finds the meet set, the
// meet edges and sigma of layer k, which is all a step that meets needs
// (its new layer is never used); a probe that finds no meet is followed
// by the claiming scan.
template <int BS, bool SP>
__device__ void expand_int(Smem<BS> &sm, const Ctx &c, int X, int32_t k, int32_t lo, int32_t hi,
                           LocalStats &ls, bool probe)
{
    // Each lane takes U adjacency entries per iteration (64 apart, so every
    // load stays coalesced across the wave) and issues their loads
    // together: U column reads, then U record probes, then the U updates.
    constexpr int U = 4;
    const int tid = threadIdx.x, lane = tid & 63;
    const int32_t n = c.qn;   // queue and meet-list capacity
    const uint32_t xbit = (uint32_t)X << X_SHIFT;
    const uint64_t newkey = ((uint64_t)c.cur << 32) | xbit | (uint32_t)(k + 1);
    unsigned long long nd = 0;
    // sigma_X of the meet vertices, should this expansion meet: every meet
    // edge (u, w) adds sigma(u) to w's slot once u's sigma is complete.
    // Slots: LDS below MCAP, the slot's global accumulators below MACC.
    // Meet edges beyond the LDS list of a chunk spill, two words each, to
    // the back of the meet buffer, whose front holds at most the size of
    // Y's newest layer (the meet set lies in it).
    const int64_t spill_cap = max<int64_t>(0, ((int64_t)n - (int64_t)(sm.hi[1 - X] - sm.lo[1 - X]) - 2) / 2);
    for (int32_t i = tid; i < MCAP; i += BS) sm.m.w[i] = 0;
    if (tid == 0) {
        sm.nme = 0;
        sm.fold_bad = 0;
    }
    for (int32_t base = lo; base < hi; base += BS) {
        if (SP && sm.quit) break;   // set in a previous chunk's scan (read after its barrier)
        const int cnt = min(BS, hi - base);
        int32_t u = -1;
        int64_t rs = 0, d = 0, riu = -1;
        if (tid < cnt) {
            u = c.Q[qpos(n, X, base + tid)];
            rs = c.g.rp[u];
            d = c.g.rp[u + 1] - rs;
            if (k >= 1) riu = vs_index<SP>(c, u);
        }
        sm.e.u[tid] = u;
        sm.e.rs[tid] = rs;
        sm.e.acc[tid] = 0;
        int64_t total;
        const int64_t off = block_excl_scan<BS>(sm, d, total);
        sm.e.off[tid] = off;
        __syncthreads();
        // The owners and column reads of the next batch are issued before
        // the current batch's records are probed, so their latencies overlap.
        auto fetch = [&](int64_t eb, int *a, int32_t *w, uint32_t &act) {
            act = 0;
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t e = eb + 64 * j + lane;
                a[j] = 0;
                w[j] = 0;
                if (e < total) {
                    act |= 1u << j;
                    int lo_i = 0, hi_i = cnt - 1;
                    while (lo_i < hi_i) {
                        const int mid = (lo_i + hi_i + 1) >> 1;
                        if (sm.e.off[mid] <= e) lo_i = mid; else hi_i = mid - 1;
                    }
                    a[j] = lo_i;
                    w[j] = c.g.ci[sm.e.rs[lo_i] + (e - sm.e.off[lo_i])];
                }
            }
        };
        int a[U];
        int32_t w[U];
        uint32_t act;
        fetch((int64_t)(tid >> 6) * 64 * U, a, w, act);
        for (int64_t e0 = (int64_t)(tid >> 6) * 64 * U; e0 < total; e0 += (int64_t)BS * U) {
            // A scan of a hub's row can last milliseconds: every 16 rounds
            // (16 BS U entries a workgroup) a wave looks at the stop flag,
            // and once the run has stopped the sample is abandoned (its
            // epoch is past the stop and never merged).
            if (SP && ((e0 / ((int64_t)BS * U)) & 15) == 15) {
                const int32_t *sp = sm.stopp;
                if (sp && __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    sm.quit = 1;
                    break;
                }
            }
            int an[U];
            int32_t wn[U];
            uint32_t actn = 0;
            if (e0 + (int64_t)BS * U < total) fetch(e0 + (int64_t)BS * U, an, wn, actn);
            uint64_t kk[U];
            uint32_t pred = 0, meet = 0, claim = 0;
            if (probe) {
#pragma unroll
                for (int j = 0; j < U; ++j)
                    if ((act >> j & 1) && !filt_test<BS>(sm.filt, w[j])) act &= ~(1u << j);
            }
            int64_t ri[U];
            if (!SP) {
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    ri[j] = w[j];
                    kk[j] = (act >> j & 1) ? ld_key(c.R + w[j]) : 0ull;
                }
            } else {
                // the home buckets' loads together, then the rest of each run
                uint32_t hb[U];
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    hb[j] = sp_home(c, w[j]);
                    kk[j] = (act >> j & 1) ? ld_key(c.R + hb[j]) : 0ull;
                }
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    ri[j] = -1;
                    if (act >> j & 1) kk[j] = vs_resolve<SP>(c, w[j], hb[j], kk[j], ri[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (!(act >> j & 1)) continue;
                const uint32_t st = (uint32_t)kk[j];
                if ((uint32_t)(kk[j] >> 32) == c.cur) {
                    if ((st & SIDE_BIT) == xbit) {
                        if (k >= 1 && (st & DEPTH_MASK) == (uint32_t)(k - 1)) pred |= 1u << j;
                    } else {
                        meet |= 1u << j;
                    }
                } else if (!probe) {
                    claim |= 1u << j;
                }
            }
            uint64_t sv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) sv[j] = (pred >> j & 1) ? ld_sig(c.R + ri[j]) : 0ull;
            uint32_t disc = 0, newmeet = 0;
            if (SP && claim) {
                // the table stays at most 3/4 full: a sample that would claim
                // more vertices (or go deeper than the key holds) is handed
                // to the dense fallback
                if (claimed_now(sm, X) + BS * U > c.claim_limit || (uint32_t)(k + 1) > SP_DEPTH_MAX) {
                    sm.vsfull = 1;
                    claim = 0;
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (claim >> j & 1) {
                    const bool won = vs_claim<SP>(c, w[j], kk[j], newkey, ri[j]);
                    disc |= (uint32_t)won << j;
                    if (won) filt_set<BS>(sm.filt, w[j]);
                }
                if (meet >> j & 1) newmeet |= (uint32_t)!(vs_or_meet<SP>(c, ri[j]) & MEET_BIT) << j;
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (pred >> j & 1) {
                    const unsigned long long old = atomicAdd(&sm.e.acc[a[j]], (unsigned long long)sv[j]);
                    if (old + sv[j] < old) sm.ovf = 1;
                    ls.pred += 1;
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const bool dj = disc >> j & 1;
                const uint64_t dm = __ballot(dj);
                if (dm) {
                    const int leader = __ffsll((unsigned long long)dm) - 1;
                    int pos = 0;
                    if (lane == leader) pos = atomicAdd(&sm.tail, __popcll(dm));
                    pos = __shfl(pos, leader);
                    if (dj) c.Q[qpos(n, X, pos + (int)mbcnt(dm))] = w[j];
                }
                if (meet >> j & 1) {
                    const int32_t slot = atomicAdd(&sm.nme, 1);
                    if (slot < MEDGE) {   // the meet vertex by its record index
                        sm.me_a[slot] = a[j];
                        sm.me_w[slot] = (int32_t)ri[j];
                    } else if ((int64_t)(slot - MEDGE) < spill_cap) {
                        const int64_t q = (int64_t)n - 2 - 2 * (int64_t)(slot - MEDGE);
                        c.MB[q + 1] = (int32_t)ri[j];
                        c.MB[q] = a[j];
                    }
                }
                const bool mj = newmeet >> j & 1;
                const uint64_t mm = __ballot(mj);
                if (mm) {
                    const int leader = __ffsll((unsigned long long)mm) - 1;
                    int pos = 0;
                    if (lane == leader) pos = atomicAdd(&sm.mcount, __popcll(mm));
                    pos = __shfl(pos, leader);
                    if (mj) {
                        const int mp = pos + (int)mbcnt(mm);
                        c.MB[mp] = w[j];
                        st_sig(c.R + ri[j], (uint64_t)mp);   // meet vertices are never expanded:
                                                            // their sigma field holds the list position
                        if (mp >= MCAP && mp < c.macc_cap) c.gacc[mp] = 0;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) nd += (disc >> j & 1) ? (unsigned long long)c.g.deg[w[j]] : 0ull;
            ls.visited += __popc(disc);
#pragma unroll
            for (int j = 0; j < U; ++j) {
                a[j] = an[j];
                w[j] = wn[j];
            }
            act = actn;
        }
        __syncthreads();
        if (k >= 1 && tid < cnt) st_sig(c.R + riu, sm.e.acc[tid]);
        const int32_t nme = sm.nme;
        if (nme > 0) {
            // the chunk's sigmas are complete; meet positions were written
            // by the lanes that set the meet bits, before the barrier
            if ((int64_t)nme - MEDGE > spill_cap && tid == 0) sm.fold_bad = 1;
            const int32_t nfold = (int32_t)min<int64_t>(nme, (int64_t)MEDGE + spill_cap);
            for (int32_t i = tid; i < nfold; i += BS) {
                int32_t ai, wi;
                if (i < MEDGE) {
                    ai = sm.me_a[i];
                    wi = sm.me_w[i];
                } else {
                    const int64_t q = (int64_t)n - 2 - 2 * (int64_t)(i - MEDGE);
                    wi = c.MB[q + 1];
                    ai = c.MB[q];
                }
                const uint64_t su = (k >= 1) ? (uint64_t)sm.e.acc[ai] : 1ull;
                const uint64_t mp = ld_sig(c.R + wi);
                unsigned long long *slotp = nullptr;
                if (mp < (uint64_t)MCAP) slotp = &sm.m.w[mp];
                else if (mp < (uint64_t)c.macc_cap) slotp = c.gacc + mp;
                if (slotp) {
                    const unsigned long long old = atomicAdd(slotp, (unsigned long long)su);
                    if (old + su < old) sm.ovf = 1;
                } else {
                    sm.fold_bad = 1;
                }
            }
        }
        __syncthreads();
        if (tid == 0) sm.nme = 0;
    }
    if (nd) atomicAdd(&sm.nextdeg, nd);
}

template <int BS, bool SP>
__device__ void expand_fp(Smem<BS> &sm, const Ctx &c, int X, int32_t k, int32_t lo, int32_t hi,
                          LocalStats &ls)
{
    // One lane per frontier vertex (so its sum runs in CSR order); the
    // row is read V entries at a time with all loads of a batch in flight.
    constexpr int V = 8;
    const int tid = threadIdx.x;
    const int32_t n = c.qn;   // queue and meet-list capacity
    const uint32_t xbit = (uint32_t)X << X_SHIFT;
    const uint64_t newkey = ((uint64_t)c.cur << 32) | xbit | (uint32_t)(k + 1);
    unsigned long long nd = 0;
    double mx = 0.0;
    for (int32_t p = lo + tid; p < hi; p += BS) {
        const int32_t u = c.Q[qpos(n, X, p)];
        double acc = 0.0;
        const int64_t beg = c.g.rp[u], end = c.g.rp[u + 1];
        for (int64_t e0 = beg; e0 < end; e0 += V) {
            const int m = (int)min<int64_t>(V, end - e0);
            int32_t w[V];
            uint64_t kk[V];
#pragma unroll
            for (int j = 0; j < V; ++j) w[j] = j < m ? c.g.cci[e0 + j] : 0;
            int64_t ri[V];
#pragma unroll
            for (int j = 0; j < V; ++j) {
                ri[j] = -1;
                kk[j] = j < m ? vs_key<SP>(c, w[j], ri[j]) : 0ull;
            }
            uint32_t pred = 0;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                if (j >= m) continue;
                if ((uint32_t)(kk[j] >> 32) == c.cur) {
                    const uint32_t st = (uint32_t)kk[j];
                    if ((st & SIDE_BIT) == xbit) {
                        if (k >= 1 && (st & DEPTH_MASK) == (uint32_t)(k - 1)) pred |= 1u << j;
                    } else {
                        const uint32_t old = vs_or_meet<SP>(c, ri[j]);
                        if (!(old & MEET_BIT)) c.MB[atomicAdd(&sm.mcount, 1)] = w[j];
                    }
                } else if (SP && (claimed_now(sm, X) + BS * V > c.claim_limit || (uint32_t)(k + 1) > SP_DEPTH_MAX)) {
                    sm.vsfull = 1;   // handed to the dense fallback
                } else if (vs_claim<SP>(c, w[j], kk[j], newkey, ri[j])) {
                    c.Q[qpos(n, X, atomicAdd(&sm.tail, 1))] = w[j];
                    nd += (unsigned long long)c.g.deg[w[j]];
                    ls.visited += 1;
                }
            }
            double sv[V];
#pragma unroll
            for (int j = 0; j < V; ++j) sv[j] = (pred >> j & 1) ? as_f64(ld_sig(c.R + ri[j])) : 0.0;
#pragma unroll
            for (int j = 0; j < V; ++j)
                if (pred >> j & 1) {       // CSR order within and across batches
                    acc = acc + sv[j];
                    ls.pred += 1;
                }
        }
        if (k >= 1) {
            st_sig(c.R + vs_index<SP>(c, u), as_u64(acc));
            mx = acc > mx ? acc : mx;
        }
    }
    if (nd) atomicAdd(&sm.nextdeg, nd);
    if (mx > 0.0) atomicMax(&sm.fmax_bits, (unsigned long long)as_u64(mx));
}

// sigma_X(w) * sigma_Y(w) for every meet vertex, stored in w's record.
template <int BS, bool SP>
__device__ void meet_weights_int(Smem<BS> &sm, const Ctx &c, int X, int32_t kX, int32_t kY, int32_t m)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t xbit = (uint32_t)X << X_SHIFT, ybit = (uint32_t)(1 - X) << X_SHIFT;
    for (int32_t base = 0; base < m; base += BS) {
        const int cnt = min(BS, m - base);
        int32_t w = -1;
        int64_t rs = 0, d = 0;
        if (tid < cnt) {
            w = c.MB[base + tid];
            rs = c.g.rp[w];
            d = c.g.rp[w + 1] - rs;
        }
        sm.e.u[tid] = w;
        sm.e.rs[tid] = rs;
        sm.e.acc[tid] = 0;
        sm.e.acc2[tid] = 0;
        int64_t total;
        const int64_t off = block_excl_scan<BS>(sm, d, total);
        sm.e.off[tid] = off;
        __syncthreads();
        for (int64_t e0 = tid & ~63; e0 < total; e0 += BS) {
            const int64_t e = e0 + lane;
            if (e < total) {
                int a = 0, b = cnt - 1;
                while (a < b) {
                    int mid = (a + b + 1) >> 1;
                    if (sm.e.off[mid] <= e) a = mid; else b = mid - 1;
                }
                const int32_t x = c.g.ci[sm.e.rs[a] + (e - sm.e.off[a])];
                int64_t rx;
                const uint64_t kk = vs_key<SP>(c, x, rx);
                Rec *r = c.R + rx;
                if ((uint32_t)(kk >> 32) == c.cur) {
                    const uint32_t st = (uint32_t)kk;
                    const uint32_t dep = st & DEPTH_MASK;
                    unsigned long long *acc = nullptr;
                    if ((st & SIDE_BIT) == xbit && dep == (uint32_t)kX) acc = &sm.e.acc[a];
                    else if ((st & SIDE_BIT) == ybit && kY >= 1 && dep == (uint32_t)(kY - 1)) acc = &sm.e.acc2[a];
                    if (acc) {
                        const uint64_t v = ld_sig(r);
                        const unsigned long long old = atomicAdd(acc, (unsigned long long)v);
                        if (old + v < old) sm.ovf = 1;
                    }
                }
            }
        }
        (void)lane;
        __syncthreads();
        if (tid < cnt) {
            const uint64_t ax = sm.e.acc[tid];
            const uint64_t ay = (kY == 0) ? 1ull : (uint64_t)sm.e.acc2[tid];
            if (__umul64hi(ax, ay) != 0) sm.ovf = 1;
            const uint64_t a = ax * ay;
            st_sig(c.R + vs_index<SP>(c, w), a);
            const unsigned long long old = atomicAdd(&sm.sigst, (unsigned long long)a);
            if (old + a < old) sm.ovf = 1;
        }
        __syncthreads();
    }
}

// Adds sigma(u) to acc[position of w] for every edge (u, w) with u in the
// queue positions [lo, hi) of `side` and w a meet vertex.
template <int BS, bool SP>
__device__ void push_to_meet(Smem<BS> &sm, const Ctx &c, int side, int32_t lo, int32_t hi,
                             unsigned long long *acc)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int32_t n = c.qn;
    for (int32_t base = lo; base < hi; base += BS) {
        const int cnt = min(BS, hi - base);
        int64_t rs = 0, d = 0;
        uint64_t su = 0;
        if (tid < cnt) {
            const int32_t u = c.Q[qpos(n, side, base + tid)];
            rs = c.g.rp[u];
            d = c.g.rp[u + 1] - rs;
            su = ld_sig(c.R + vs_index<SP>(c, u));
        }
        sm.e.rs[tid] = rs;
        sm.e.acc[tid] = su;
        int64_t total;
        const int64_t off = block_excl_scan<BS>(sm, d, total);
        sm.e.off[tid] = off;
        __syncthreads();
        for (int64_t e0 = tid & ~63; e0 < total; e0 += BS) {
            const int64_t e = e0 + lane;
            if (e < total) {
                int a = 0, b = cnt - 1;
                while (a < b) {
                    int mid = (a + b + 1) >> 1;
                    if (sm.e.off[mid] <= e) a = mid; else b = mid - 1;
                }
                int64_t rx;
                const uint64_t kk = vs_key<SP>(c, c.g.ci[sm.e.rs[a] + (e - sm.e.off[a])], rx);
                Rec *r = c.R + rx;
                if ((uint32_t)(kk >> 32) == c.cur && ((uint32_t)kk & MEET_BIT)) {
                    const uint64_t v = sm.e.acc[a];
                    const unsigned long long old = atomicAdd(acc + ld_sig(r), (unsigned long long)v);
                    if (old + v < old) sm.ovf = 1;
                }
            }
        }
        __syncthreads();
    }
}

// For every meet vertex w (list position i): accX[i] += sigma of w's
// neighbours in layer kX of X, accY[i] += sigma of w's neighbours in layer
// kY - 1 of Y (either accumulator may be null: that side is skipped).
template <int BS, bool SP>
__device__ void pull_to_meet(Smem<BS> &sm, const Ctx &c, int X, int32_t kX, int32_t kY, int32_t m,
                             unsigned long long *accX, unsigned long long *accY)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t xstate = ((uint32_t)X << X_SHIFT) | (uint32_t)kX;
    const uint32_t ystate = ((uint32_t)(1 - X) << X_SHIFT) | (uint32_t)(kY - 1);
    for (int32_t base = 0; base < m; base += BS) {
        const int cnt = min(BS, m - base);
        int64_t rs = 0, d = 0;
        if (tid < cnt) {
            const int32_t w = c.MB[base + tid];
            rs = c.g.rp[w];
            d = c.g.rp[w + 1] - rs;
        }
        sm.e.rs[tid] = rs;
        int64_t total;
        const int64_t off = block_excl_scan<BS>(sm, d, total);
        sm.e.off[tid] = off;
        __syncthreads();
        for (int64_t e0 = tid & ~63; e0 < total; e0 += BS) {
            const int64_t e = e0 + lane;
            if (e < total) {
                int a = 0, b = cnt - 1;
                while (a < b) {
                    int mid = (a + b + 1) >> 1;
                    if (sm.e.off[mid] <= e) a = mid; else b = mid - 1;
                }
                int64_t rx;
                const uint64_t kk = vs_key<SP>(c, c.g.ci[sm.e.rs[a] + (e - sm.e.off[a])], rx);
                Rec *r = c.R + rx;
                if ((uint32_t)(kk >> 32) == c.cur) {
                    const uint32_t st = (uint32_t)kk & ~MEET_BIT;
                    unsigned long long *acc = nullptr;
                    if (accX && st == xstate) acc = accX + base + a;
                    else if (accY && kY >= 1 && st == ystate) acc = accY + base + a;
                    if (acc) {
                        const uint64_t v = ld_sig(r);
                        const unsigned long long old = atomicAdd(acc, (unsigned long long)v);
                        if (old + v < old) sm.ovf = 1;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Integer-mode meet weights a_w = sigma_X(w) * sigma_Y(w).  Each side's sum
// is taken over whichever edge set is smaller: the edges of the layer the
// predecessors live in (pushed to the meet vertices) or the edges of the
// meet vertices themselves (pulled).  Integer sums do not depend on the
// order, so both give the same value.  Weights end in sm.m.w (m <= MCAP),
// in the slot's global buffer (m <= MACC) or, beyond that, in the meet
// vertices' sigma fields; sm.mpath says which.
template <int BS, bool SP>
__device__ void meet_int(Smem<BS> &sm, const Ctx &c, int X, int32_t kX, int32_t kY, int32_t m,
                         unsigned long long *gacc, int32_t macc_cap)
{
    const int tid = threadIdx.x;
    const int path = (m <= MCAP) ? 0 : (m <= macc_cap ? 1 : 2);
    if (path == 2) {
        meet_weights_int<BS, SP>(sm, c, X, kX, kY, m);
        if (tid == 0) sm.mpath = 2;
        __syncthreads();
        return;
    }
    unsigned long long *accX = path == 0 ? sm.m.w : gacc;
    unsigned long long *accY = path == 0 ? sm.m.w2 : gacc + macc_cap;
    // the expansion folded sigma_X of every meet vertex (positions below
    // MCAP in sm.m.w, the rest in the slot buffer) unless the meet edges
    // overflowed the spill space (then it is recomputed here)
    const bool foldX = path <= 1 && !sm.fold_bad;
    uint64_t dsum = 0;
    for (int32_t i = tid; i < m; i += BS) {
        const int32_t w = c.MB[i];
        dsum += (uint64_t)(c.g.rp[w + 1] - c.g.rp[w]);
        if (!foldX) accX[i] = 0;
        else if (path == 1 && i < MCAP) accX[i] = sm.m.w[i];
        accY[i] = 0;
        if (path == 0) sm.m.id[i] = c.g.orig[w];
    }
    const uint64_t dM = block_sum_u64<BS>(sm, dsum);
    const int Y = 1 - X;
    const bool pushX = !foldX && (uint64_t)sm.sdeg[X] <= dM;
    const bool pullX = !foldX && !pushX;
    const bool pushY = kY >= 1 && (uint64_t)sm.psdeg[Y] <= dM;
    const bool pullY = kY >= 1 && !pushY;
    if (pushX) push_to_meet<BS, SP>(sm, c, X, sm.lo[X], sm.hi[X], accX);
    if (pushY) push_to_meet<BS, SP>(sm, c, Y, sm.plo[Y], sm.phi[Y], accY);
    if (pullX || pullY)
        pull_to_meet<BS, SP>(sm, c, X, kX, kY, m, pullX ? accX : nullptr, pullY ? accY : nullptr);
    __syncthreads();
    for (int32_t i = tid; i < m; i += BS) {
        const uint64_t ax = accX[i];
        const uint64_t ay = (kY == 0) ? 1ull : (uint64_t)accY[i];
        if (__umul64hi(ax, ay) != 0) sm.ovf = 1;
        const uint64_t a = ax * ay;
        accX[i] = a;
        const unsigned long long old = atomicAdd(&sm.sigst, (unsigned long long)a);
        if (old + a < old) sm.ovf = 1;
    }
    if (tid == 0) sm.mpath = path;
    __syncthreads();
}

template <int BS, bool SP>
__device__ void meet_weights_fp(Smem<BS> &sm, const Ctx &c, int X, int32_t kX, int32_t kY, int32_t m)
{
    const uint32_t xstate = ((uint32_t)X << X_SHIFT) | (uint32_t)kX;
    const uint32_t ystate = ((uint32_t)(1 - X) << X_SHIFT) | (uint32_t)(kY - 1);
    for (int32_t i = threadIdx.x; i < m; i += BS) {
        const int32_t w = c.MB[i];
        double ax = 0.0, ay = 0.0;
        for (int64_t e = c.g.rp[w]; e < c.g.rp[w + 1]; ++e) {
            const int32_t x = c.g.cci[e];
            int64_t rx;
            const uint64_t kk = vs_key<SP>(c, x, rx);
            Rec *r = c.R + rx;
            if ((uint32_t)(kk >> 32) != c.cur) continue;
            const uint32_t st = (uint32_t)kk & ~MEET_BIT;
            if (st == xstate) ax = ax + as_f64(ld_sig(r));
            else if (kY >= 1 && st == ystate) ay = ay + as_f64(ld_sig(r));
        }
        if (kY == 0) ay = 1.0;
        st_sig(c.R + vs_index<SP>(c, w), as_u64(ax * ay));
    }
    (void)sm;
}

// Smallest caller id of the meet list above `last` (all threads call;
// uniform result).
template <int BS>
__device__ int32_t next_min(Smem<BS> &sm, const Ctx &c, int32_t m, int32_t last)
{
    if (threadIdx.x == 0) sm.wmin = 0x7fffffff;
    __syncthreads();
    int32_t best = 0x7fffffff;
    for (int32_t i = threadIdx.x; i < m; i += BS) {
        const int32_t id = c.g.orig[c.MB[i]];
        if (id > last && id < best) best = id;
    }
    if (best != 0x7fffffff) atomicMin(&sm.wmin, best);
    __syncthreads();
    const int32_t r = sm.wmin;
    __syncthreads();
    return r;
}

// Chooses the meet vertex; result in sm.w (all threads call).
template <int BS, bool SP>
__device__ void choose_meet(Smem<BS> &sm, const Ctx &c, int32_t m, uint64_t u2,
                            const unsigned long long *gacc)
{
    constexpr int PER = MCAP / BS;
    const int tid = threadIdx.x;
    if (m <= MCAP) {
        if (c.fp) {   // integer mode filled ids and weights in LDS already
            for (int32_t i = tid; i < m; i += BS) {
                const int32_t w = c.MB[i];
                sm.m.id[i] = c.g.orig[w];
                sm.m.w[i] = ld_sig(c.R + vs_index<SP>(c, w));
            }
        }
        __syncthreads();
        int32_t myid[PER];
        uint64_t myw[PER];
        int32_t myrank[PER];
        uint64_t mypre[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int32_t i = tid + j * BS;
            myid[j] = -1;
            myw[j] = 0;
            myrank[j] = 0;
            mypre[j] = 0;
            if (i < m) {
                myid[j] = sm.m.id[i];
                myw[j] = sm.m.w[i];
            }
        }
        // rank (and, in integer mode, exclusive prefix) in ascending caller id
        for (int32_t jj = 0; jj < m; ++jj) {
            const int32_t idj = sm.m.id[jj];
            const uint64_t wj = sm.m.w[jj];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                if (myid[j] >= 0 && idj < myid[j]) {
                    myrank[j] += 1;
                    mypre[j] += wj;
                }
            }
        }
        if (!c.fp) {
            const uint64_t r = __umul64hi(u2, (uint64_t)sm.sigst);
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (myid[j] >= 0 && mypre[j] <= r && r - mypre[j] < myw[j]) sm.w = c.g.newid[myid[j]];
            __syncthreads();
            return;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (myid[j] >= 0) {
                sm.m.id[myrank[j]] = myid[j];
                sm.m.w[myrank[j]] = myw[j];
            }
        }
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int32_t i = 0; i < m; ++i) tot = tot + as_f64(sm.m.w[i]);
            const double r = unit53(u2) * tot;
            double pre = 0.0;
            int32_t pick = -1;
            for (int32_t i = 0; i < m; ++i) {
                const double a = as_f64(sm.m.w[i]);
                pre = pre + a;
                if (a != 0.0) pick = sm.m.id[i];
                if (pre > r) { pick = sm.m.id[i]; break; }
            }
            sm.w = pick >= 0 ? c.g.newid[pick] : pick;
        }
        __syncthreads();
        return;
    }
    // Large meet sets, integer mode: the chosen vertex is the smallest
    // caller id x at which the weight of the meet vertices with caller id
    // <= x exceeds r; binary search over the id range, one block-wide sum
    // per step.
    if (!c.fp) {
        const uint64_t r = __umul64hi(u2, (uint64_t)sm.sigst);
        const bool global_w = sm.mpath == 1;    // weights in the slot buffer, else in sigma fields
        int32_t lo = 0, hi = c.g.n - 1;
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            uint64_t part = 0;
            for (int32_t i = tid; i < m; i += BS) {
                const int32_t w = c.MB[i];
                if (c.g.orig[w] <= mid) part += global_w ? (uint64_t)gacc[i] : ld_sig(c.R + vs_index<SP>(c, w));
            }
            const uint64_t tot = block_sum_u64<BS>(sm, part);
            if (tot > r) hi = mid; else lo = mid + 1;
        }
        if (tid == 0) sm.w = c.g.newid[lo];
        __syncthreads();
        return;
    }
    // FP mode, large meet set: sort (caller id, list position) keys in the
    // slot's meet accumulators (idle in FP mode) with a block-wide bitonic
    // sort, gather the weights in that order behind them, then one wave sums
    // them left to right (the rounding order the definition fixes) and finds
    // the pick in a second ordered pass.
    int32_t mp = 1;
    while (mp < m) mp <<= 1;
    if (mp <= c.macc_cap) {
        // keys in [0, mp), weights in [mp, mp + m): within 2 * macc_cap
        uint64_t *key = reinterpret_cast<uint64_t *>(c.gacc);
        double *wsorted = reinterpret_cast<double *>(c.gacc) + mp;
        for (int32_t i = tid; i < mp; i += BS)
            key[i] = i < m ? (((uint64_t)(uint32_t)c.g.orig[c.MB[i]] << 32) | (uint32_t)i) : ~0ull;
        __syncthreads();
        for (int32_t k = 2; k <= mp; k <<= 1) {
            for (int32_t j = k >> 1; j > 0; j >>= 1) {
                for (int32_t i = tid; i < mp; i += BS) {
                    const int32_t l = i ^ j;
                    if (l > i) {
                        const uint64_t a = key[i], b = key[l];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            key[i] = b;
                            key[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int32_t i = tid; i < m; i += BS)
            wsorted[i] = as_f64(ld_sig(c.R + vs_index<SP>(c, c.MB[(uint32_t)key[i]])));
        __syncthreads();
        if (tid < 64) {
            const int lane = tid;
            double tot = 0.0;
            for (int32_t b0 = 0; b0 < m; b0 += 64) {
                const double x = b0 + lane < m ? wsorted[b0 + lane] : 0.0;
                const int cnt = min(64, m - b0);
                for (int j = 0; j < cnt; ++j) tot = tot + __shfl(x, j);
            }
            const double r = unit53(u2) * tot;
            double pre = 0.0;
            int32_t pick = -1;
            bool done = false;
            for (int32_t b0 = 0; b0 < m && !done; b0 += 64) {
                const double x = b0 + lane < m ? wsorted[b0 + lane] : 0.0;
                const int32_t idk = b0 + lane < m ? (int32_t)(key[b0 + lane] >> 32) : -1;
                const int cnt = min(64, m - b0);
                for (int j = 0; j < cnt; ++j) {
                    const double a = __shfl(x, j);
                    const int32_t id = __shfl(idk, j);
                    pre = pre + a;
                    if (a != 0.0) pick = id;
                    if (pre > r) { pick = id; done = true; break; }
                }
            }
            if (lane == 0) sm.w = pick >= 0 ? c.g.newid[pick] : pick;
        }
        __syncthreads();
        return;
    }
    // beyond the accumulators: visit the list in ascending id by repeated
    // minimum search; first pass sums the weights, second finds the pick.
    double tot = 0.0;
    for (int32_t step = 0, last = -1; step < m; ++step) {
        const int32_t id = next_min<BS>(sm, c, m, last);
        tot = tot + as_f64(ld_sig(c.R + vs_index<SP>(c, c.g.newid[id])));
        last = id;
    }
    const double r = unit53(u2) * tot;
    double pre = 0.0;
    int32_t pick = -1;
    for (int32_t step = 0, last = -1; step < m; ++step) {
        const int32_t id = next_min<BS>(sm, c, m, last);
        const double a = as_f64(ld_sig(c.R + vs_index<SP>(c, c.g.newid[id])));
        pre = pre + a;
        if (a != 0.0) pick = id;
        if (pre > r) { pick = id; break; }
        last = id;
    }
    if (tid == 0) sm.w = pick >= 0 ? c.g.newid[pick] : pick;
    __syncthreads();
}

// One predecessor pick walking back on `side` from v at depth l (>= 2).
template <bool SP>
__device__ int32_t pick_pred(const Ctx &c, int side, int32_t v, int32_t l, uint64_t u, int lane)
{
    const uint32_t want = ((uint32_t)side << X_SHIFT) | (uint32_t)(l - 1);
    const int64_t beg = c.g.rp[v], end = c.g.rp[v + 1];
    if (end - beg <= 64) {
        // a row that fits one wave: read once, total and pick from registers
        const int64_t e = beg + lane;
        int32_t x = -1;
        uint64_t bits = 0;
        bool cand = false;
        if (e < end) {
            x = c.g.cci[e];
            int64_t rx;
            const uint64_t kk = vs_key<SP>(c, x, rx);
            Rec *r = c.R + rx;
            if ((uint32_t)(kk >> 32) == c.cur && ((uint32_t)kk & ~MEET_BIT) == want) {
                cand = true;
                bits = ld_sig(r);
            }
        }
        if (!c.fp) {
            const uint64_t wt = cand ? bits : 0ull;
            const uint64_t tot = wave_sum_u64(wt);
            const uint64_t r = __umul64hi(u, tot);
            const uint64_t incl = wave_incl_scan_u64(wt, lane);
            const uint64_t hit = __ballot(wt != 0 && incl > r);
            return hit ? __shfl(x, __ffsll((unsigned long long)hit) - 1) : -1;
        }
        const double wt = cand ? as_f64(bits) : 0.0;
        const uint64_t mask = __ballot(cand);
        double tot = 0.0;
        for (uint64_t mm = mask; mm; mm &= mm - 1) tot = tot + __shfl(wt, __ffsll((unsigned long long)mm) - 1);
        const double r = unit53(u) * tot;
        double pre = 0.0;
        int32_t last_nz = -1;
        for (uint64_t mm = mask; mm; mm &= mm - 1) {
            const int j = __ffsll((unsigned long long)mm) - 1;
            const double a = __shfl(wt, j);
            const int32_t xj = __shfl(x, j);
            pre = pre + a;
            if (a != 0.0) last_nz = xj;
            if (pre > r) return xj;
        }
        return last_nz;
    }
    if (!c.fp) {
        uint64_t tot = 0;
        for (int64_t c0 = beg; c0 < end; c0 += 64) {
            const int64_t e = c0 + lane;
            uint64_t wt = 0;
            if (e < end) {
                int64_t rx;
                const uint64_t kk = vs_key<SP>(c, c.g.cci[e], rx);
                Rec *r = c.R + rx;
                if ((uint32_t)(kk >> 32) == c.cur && ((uint32_t)kk & ~MEET_BIT) == want) wt = ld_sig(r);
            }
            tot += wave_sum_u64(wt);
        }
        const uint64_t r = __umul64hi(u, tot);
        uint64_t pre = 0;
        for (int64_t c0 = beg; c0 < end; c0 += 64) {
            const int64_t e = c0 + lane;
            uint64_t wt = 0;
            int32_t x = -1;
            if (e < end) {
                x = c.g.cci[e];
                int64_t rx;
                const uint64_t kk = vs_key<SP>(c, x, rx);
                Rec *rc = c.R + rx;
                if ((uint32_t)(kk >> 32) == c.cur && ((uint32_t)kk & ~MEET_BIT) == want) wt = ld_sig(rc);
            }
            const uint64_t incl = wave_incl_scan_u64(wt, lane);
            const uint64_t hit = __ballot(wt != 0 && pre + incl > r);
            if (hit) return __shfl(x, __ffsll((unsigned long long)hit) - 1);
            pre += __shfl(incl, 63);
        }
        return -1;
    }
    double tot = 0.0;
    for (int64_t c0 = beg; c0 < end; c0 += 64) {
        const int64_t e = c0 + lane;
        double wt = 0.0;
        bool cand = false;
        if (e < end) {
            int64_t rx;
            const uint64_t kk = vs_key<SP>(c, c.g.cci[e], rx);
            Rec *r = c.R + rx;
            if ((uint32_t)(kk >> 32) == c.cur && ((uint32_t)kk & ~MEET_BIT) == want) {
                cand = true;
                wt = as_f64(ld_sig(r));
            }
        }
        uint64_t mask = __ballot(cand);
        while (mask) {
            const int j = __ffsll((unsigned long long)mask) - 1;
            tot = tot + __shfl(wt, j);
            mask &= mask - 1;
        }
    }
    const double r = unit53(u) * tot;
    double pre = 0.0;
    int32_t last_nz = -1;
    for (int64_t c0 = beg; c0 < end; c0 += 64) {
        const int64_t e = c0 + lane;
        double wt = 0.0;
        bool cand = false;
        int32_t x = -1;
        if (e < end) {
            x = c.g.cci[e];
            int64_t rx;
            const uint64_t kk = vs_key<SP>(c, x, rx);
            Rec *rc = c.R + rx;
            if ((uint32_t)(kk >> 32) == c.cur && ((uint32_t)kk & ~MEET_BIT) == want) {
                cand = true;
                wt = as_f64(ld_sig(rc));
            }
        }
        uint64_t mask = __ballot(cand);
        while (mask) {
            const int j = __ffsll((unsigned long long)mask) - 1;
            const double a = __shfl(wt, j);
            const int32_t xj = __shfl(x, j);
            pre = pre + a;
            if (a != 0.0) last_nz = xj;
            if (pre > r) return xj;
            mask &= mask - 1;
        }
    }
    return last_nz;
}

__device__ __forceinline__ bool row_contains(const DevGraph &g, int32_t row, int32_t target)
{
    int64_t lo = g.rp[row], hi = g.rp[row + 1];
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (g.ci[mid] < target) lo = mid + 1; else hi = mid;
    }
    return lo < end && g.ci[lo] == target;
}

// Integer-mode predecessor pick at a high-degree vertex v: the candidates
// are the vertices of layer l - 1 of `side` (queue positions [lo, hi))
// adjacent to v, found by binary search in the shorter of the two rows;
// the pick is the same as scanning v's row (ascending id = CSR order).
// One wave; candidates go to its part [base, base + cap) of the (idle)
// expansion LDS area.  Returns -2 when there are more candidates than fit
// (the caller scans v's row).
template <int BS, bool SP>
__device__ int32_t pick_pred_layer(Smem<BS> &sm, const Ctx &c, int side, int32_t v, int32_t lo,
                                   int32_t hi, uint64_t u, int lane, int32_t base, int32_t cap)
{
    const int32_t n = c.qn;
    const int64_t dv = c.g.rp[v + 1] - c.g.rp[v];
    uint64_t tot = 0;
    int32_t ncand = 0;
    for (int32_t p0 = lo; p0 < hi; p0 += 64) {
        const int32_t p = p0 + lane;
        bool cand = false;
        int32_t x = -1;
        uint64_t wt = 0;
        if (p < hi) {
            x = c.Q[qpos(n, side, p)];
            const int64_t dx = c.g.rp[x + 1] - c.g.rp[x];
            cand = dx <= dv ? row_contains(c.g, x, v) : row_contains(c.g, v, x);
            if (cand) wt = ld_sig(c.R + vs_index<SP>(c, x));
        }
        const uint64_t cm = __ballot(cand);
        const int32_t k = __popcll(cm);
        if (ncand + k > cap) return -2;
        if (cand) {
            const int32_t slot = base + ncand + (int32_t)mbcnt(cm);
            sm.e.u[slot] = c.g.orig[x];    // ranked by caller id (= CSR order)
            sm.e.acc[slot] = wt;
        }
        ncand += k;
        tot += wave_sum_u64(wt);
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const uint64_t r = __umul64hi(u, tot);
    int32_t pick = -1;
    for (int32_t i0 = 0; i0 < ncand; i0 += 64) {
        const int32_t i = i0 + lane;
        bool hit = false;
        int32_t id = -1;
        if (i < ncand) {
            id = sm.e.u[base + i];
            const uint64_t wi = sm.e.acc[base + i];
            uint64_t pre = 0;
            for (int32_t j = 0; j < ncand; ++j)
                if (sm.e.u[base + j] < id) pre += sm.e.acc[base + j];
            hit = pre <= r && r - pre < wi;
        }
        const uint64_t hm = __ballot(hit);
        if (hm) { pick = __shfl(id, __ffsll((unsigned long long)hm) - 1); break; }
    }
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return pick >= 0 ? c.g.newid[pick] : pick;
}

// One count for an interior vertex (at its caller id when the launch maps
// counters to the caller's numbering).  With a histogram (the calibration),
// its bins follow the counter: the value moves from bin c to bin c + 1
// (a vertex is counted at most once per sample, so c < samples <= top).
__device__ __forceinline__ void count_vertex(const SampleLaunch &a, uint32_t *sf, int32_t v)
{
    const uint32_t old = atomicAdd(sf + (a.count_map ? a.count_map[v] : v), 1u);
    if (a.hist) {
        if (old >= 1) atomicSub(a.hist + min(old, a.hist_top), 1u);
        atomicAdd(a.hist + min(old + 1, a.hist_top), 1u);
    }
}

// The second bound is the minimum of waves per SIMD.  The 256-thread
// shape is held to three (three workgroups per CU): the high-diameter
// graphs depend on that many samples in flight; the 512-thread shape to
// four (two workgroups per CU).
template <int BS, bool SP>
__global__ __launch_bounds__(BS, (BS == 256 ? 3 : (BS == 512 ? 4 : 1))) void k_sample(SampleLaunch a)
{
    __shared__ Smem<BS> sm;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (a.stop_flag && __hip_atomic_load(a.stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    uint64_t first = a.first, count = a.count;
    uint32_t *sf = a.sf[0];
    // a replayed graph reads the run's seed from the device (its launch
    // arguments were fixed when it was captured)
    const uint64_t seed = a.dev_seed ? *a.dev_seed : a.seed;
    if (a.dev_epoch) {
        const unsigned long long k = *a.dev_epoch;
        first = k * a.E;
        count = first < a.cap ? (a.cap - first < a.E ? a.cap - first : a.E) : 0;
    }
    const int32_t n = a.g.n;
    const size_t slot = blockIdx.x;
    Ctx c;
    c.g = a.g;
    // dense: a record per vertex, queue and meet list of n; sparse: a table
    // of 2^vcap_log2 buckets, queue and meet list of as many entries
    const int32_t qn = SP ? (int32_t)(1u << a.vcap_log2) : n;
    c.qn = qn;
    c.R = a.recs + slot * (size_t)qn;
    c.Q = a.queues + slot * (size_t)qn;
    c.MB = a.mbufs + slot * (size_t)qn;
    c.mask = SP ? (uint32_t)qn - 1u : 0u;
    c.hshift = SP ? 64u - a.vcap_log2 : 0u;
    c.claim_limit = a.claim_limit;
    c.err = &a.stats->error;
    unsigned long long *gacc = a.macc + slot * 2 * (size_t)a.macc_cap;
    c.gacc = gacc;
    c.macc_cap = a.macc_cap;
    LocalStats ls{0, 0};
    unsigned long long st_edges = 0, st_exp = 0, st_path = 0, st_fp = 0, st_samples = 0, st_all = 0;

    for (;;) {
        if (tid == 0) {
            // a later epoch that became speculative (the run stopped) quits early
            const bool stop = a.stop_flag &&
                              __hip_atomic_load(a.stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.defer_in) {   // the dense fallback: the samples a sparse launch handed over
                const unsigned long long q = stop ? ~0ull : atomicAdd(a.work_ctr, 1ull);
                const unsigned long long nd =
                    __hip_atomic_load(a.defer_in_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sm.sid = (q < nd && q < (unsigned long long)a.defer_cap) ? (unsigned long long)a.defer_in[q] : count;
            } else {
                sm.sid = stop ? count : atomicAdd(a.work_ctr, 1ull);
            }
        }
        __syncthreads();
        const unsigned long long sid = sm.sid;
        if (sid >= count) break;
        const uint64_t idx = first + sid;
        const uint64_t t_begin = wall_clock64();
        int fp = a.sigma_fp;
        int attempts = 0;
        if (tid == 0) {
            SampleDraws dr;
            dr.init(seed, a.stream, idx);
            const uint64_t u0 = dr.get(0), u1 = dr.get(1);
            const int32_t s = (int32_t)__umul64hi(u0, (uint64_t)n);
            int32_t t = (int32_t)__umul64hi(u1, (uint64_t)(n - 1));
            if (t >= s) t += 1;
            sm.s = a.g.newid[s];   // the pair is drawn in caller ids
            sm.t = a.g.newid[t];
        }
        uint64_t t_exp = 0, t_mw = 0, t_ch = 0, t_walk = 0, t_mark = 0;
        int X = 0;
        int32_t kX = 0, kY = 0, m = 0;
        unsigned long long edges = 0;
        int steps = 0;
        bool failed = false, deferred = false, quit = false;
        const unsigned long long vis0 = ls.visited, pred0 = ls.pred, exp0 = st_exp;
        for (;;) {  // attempt (integer mode, then FP mode if it overflowed)
            attempts += 1;
            for (int i = tid; i < Filter<BS>::WORDS; i += BS) sm.filt[i] = 0;
            __syncthreads();
            if (tid == 0) {
                const uint32_t cur = a.stamps[slot] + 1;
                a.stamps[slot] = cur;
                sm.stamp = cur;
            }
            __syncthreads();
            c.cur = sm.stamp;
            c.cur16 = ((c.cur - 1u) % 65535u) + 1u;
            if (SP && c.cur16 == 1u && c.cur > 1u) {
                // the 16-bit stamp wrapped: every bucket is made free again
                for (int32_t i = tid; i < qn; i += BS) st_key(c.R + i, 0ull);
                __syncthreads();
            }
            if (tid == 0) {
                const uint32_t cur = c.cur;
                const int32_t s = sm.s, t = sm.t;
                st_sig(c.R + vs_root<SP>(c, s, ((uint64_t)cur << 32) | 0u), fp ? as_u64(1.0) : 1ull);
                st_sig(c.R + vs_root<SP>(c, t, ((uint64_t)cur << 32) | SIDE_BIT), fp ? as_u64(1.0) : 1ull);
                c.Q[0] = s;
                c.Q[qn - 1] = t;
                filt_set<BS>(sm.filt, s);
                filt_set<BS>(sm.filt, t);
                sm.lo[0] = sm.lo[1] = 0;
                sm.hi[0] = sm.hi[1] = 1;
                sm.plo[0] = sm.plo[1] = 0;
                sm.phi[0] = sm.phi[1] = 0;
                sm.loff[0][0] = sm.loff[1][0] = 0;
                sm.loff[0][1] = sm.loff[1][1] = 1;
                sm.psdeg[0] = sm.psdeg[1] = 0;
                sm.dep[0] = sm.dep[1] = 0;
                sm.sdeg[0] = a.g.rp[s + 1] - a.g.rp[s];
                sm.sdeg[1] = a.g.rp[t + 1] - a.g.rp[t];
                sm.ovf = 0;
                sm.err = 0;
                sm.sigst = 0;
                sm.tail = 1;          // set-up of the first step (both sides hold one vertex)
                sm.mcount = 0;
                sm.nextdeg = 0;
                sm.fmax_bits = 0;
                sm.vsfull = 0;
                sm.quit = 0;
                sm.stopp = a.stop_flag;
            }
            __syncthreads();
            c.fp = fp;
            edges = 0;
            steps = 0;
            for (;;) {
                X = (sm.sdeg[0] <= sm.sdeg[1]) ? 0 : 1;
                const int32_t k = sm.dep[X], lo = sm.lo[X], hi = sm.hi[X];
                edges += (unsigned long long)sm.sdeg[X];
                st_exp += (unsigned long long)(hi - lo);
                steps += 1;
                // tail, mcount, nextdeg and fmax_bits were set for this step
                // by the previous step's bookkeeping (or the attempt's set-up)
                t_mark = wall_clock64();
                // A step whose two frontiers are likely to meet (the product
                // of their degree sums reaches the number of adjacency
                // entries) is scanned without claiming first.
                const bool probe = !fp && (double)sm.sdeg[X] * (double)sm.sdeg[1 - X] >= (double)c.g.nnz;
                if (!fp) expand_int<BS, SP>(sm, c, X, k, lo, hi, ls, probe);
                else expand_fp<BS, SP>(sm, c, X, k, lo, hi, ls);
                __syncthreads();
                if (SP && sm.quit) {   // cut short by the stop: its meets and σ are partial
                    quit = true;
                    break;
                }
                if (probe && !sm.ovf && sm.mcount == 0) {
                    __syncthreads();
                    const unsigned long long pred_before = ls.pred;   // the rescan meets the
                    expand_int<BS, SP>(sm, c, X, k, lo, hi, ls, false);  // same predecessor edges
                    ls.pred = pred_before;
                    __syncthreads();
                    st_all += (unsigned long long)sm.sdeg[X];
                }
                t_exp += wall_clock64() - t_mark;
                if (SP && sm.vsfull) { deferred = true; break; }
                if (fp && k >= 1 && as_f64(sm.fmax_bits) > BIG) {
                    for (int32_t p = lo + tid; p < hi; p += BS) {
                        Rec *r = c.R + vs_index<SP>(c, c.Q[qpos(qn, X, p)]);
                        st_sig(r, as_u64(as_f64(ld_sig(r)) * SHRINK));
                    }
                    __syncthreads();
                }
                if (!fp && sm.ovf) break;
                if (sm.mcount > 0) break;
                if (sm.tail == hi && !(SP && sm.quit)) { failed = true; break; }
                __syncthreads();
                if (tid == 0) {
                    sm.plo[X] = lo;
                    sm.phi[X] = hi;
                    sm.psdeg[X] = sm.sdeg[X];
                    sm.lo[X] = hi;
                    sm.hi[X] = sm.tail;
                    sm.dep[X] = k + 1;
                    sm.sdeg[X] = (int64_t)sm.nextdeg;
                    if (k + 2 <= LMAX + 1) sm.loff[X][k + 2] = sm.tail;
                    // set up the next step
                    const int nx = (sm.sdeg[0] <= sm.sdeg[1]) ? 0 : 1;
                    sm.tail = sm.hi[nx];
                    sm.mcount = 0;
                    sm.nextdeg = 0;
                    sm.fmax_bits = 0;
                    // the run stopped while this (speculative) sample was
                    // searching: its counts would never be merged
                    sm.quit = a.stop_flag ? __hip_atomic_load(a.stop_flag, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT)
                                          : 0;
                }
                __syncthreads();
                if (sm.quit) {
                    quit = true;
                    break;
                }
            }
            st_all += edges;
            if (failed || deferred || quit) break;
            if (!fp && sm.ovf) { __syncthreads(); fp = 1; continue; }
            kX = sm.dep[X];
            kY = sm.dep[1 - X];
            m = sm.mcount;
            __syncthreads();
            t_mark = wall_clock64();
            if (!fp) meet_int<BS, SP>(sm, c, X, kX, kY, m, gacc, a.macc_cap);
            else meet_weights_fp<BS, SP>(sm, c, X, kX, kY, m);
            __syncthreads();
            t_mw += wall_clock64() - t_mark;
            if (!fp && sm.ovf) { __syncthreads(); fp = 1; continue; }
            break;
        }
        if (failed) {
            if (tid == 0) a.stats->error = 1;
            __syncthreads();
            continue;
        }
        if (quit) {   // abandoned: the sample loop sees the stop and ends
            ls.visited = vis0;
            ls.pred = pred0;
            st_exp = exp0;
            __syncthreads();
            continue;
        }
        if (deferred) {   // to the dense fallback launch that follows this one, which
            ls.visited = vis0;   // counts the sample's statistics
            ls.pred = pred0;
            st_exp = exp0;
            if (tid == 0) {
                const unsigned long long q = atomicAdd(a.defer_count, 1ull);
                if (q < (unsigned long long)a.defer_cap) a.defer_list[q] = (uint32_t)sid;
                else a.stats->error = 4;
                atomicAdd(&a.stats->deferred, 1ull);
            }
            __syncthreads();
            continue;
        }
        // meet vertex
        if (tid == 0) sm.w = -1;
        __syncthreads();
        t_mark = wall_clock64();
        {
            SampleDraws dr;
            dr.init(seed, a.stream, idx);
            const uint64_t u2 = dr.get(2);
            choose_meet<BS, SP>(sm, c, m, u2, gacc);
        }
        t_ch = wall_clock64() - t_mark;
        t_mark = wall_clock64();
        // walk back and count: the two sides are independent (their draw
        // indices are fixed by the depths), so wave 0 walks to s and wave 1
        // to t at the same time (one wave does both when BS is 64)
        const int32_t d = kX + 1 + kY;
        if (sm.w < 0) {   // no meet vertex chosen: report instead of walking
            if (tid == 0) a.stats->error = 3;
            __syncthreads();
            continue;
        }
        if (tid == 0) sm.pathc = 0;
        __syncthreads();
        constexpr int WALKERS = BS >= 128 ? 2 : 1;
        if (wid < WALKERS) {
            const int32_t s = sm.s, t = sm.t, w = sm.w;
            int32_t dep[2];
            dep[X] = kX + 1;
            dep[1 - X] = kY;
            int32_t *prow = nullptr;
            if (a.paths) {
                if (d + 1 <= a.max_len) prow = a.paths + (size_t)sid * (size_t)a.max_len;
                else if (lane == 0) a.stats->error = 2;
            }
            unsigned long long cnt = 0;
            if (wid == 0) {
                if (prow && lane == 0) {
                    prow[0] = a.g.orig[s];
                    prow[d] = a.g.orig[t];
                    prow[dep[0]] = a.g.orig[w];
                }
                if (w != s && w != t) {
                    if (lane == 0) count_vertex(a, sf, w);
                    cnt += 1;
                }
            }
            SampleDraws dr;
            dr.init(seed, a.stream, idx);
            const int32_t cap = (int32_t)(sizeof(sm.e.u) / sizeof(sm.e.u[0])) / WALKERS;
            for (int side = (WALKERS == 2 ? wid : 0); side < (WALKERS == 2 ? wid + 1 : 2); ++side) {
                // draws 3, 4, ... go to the s side first, then to the t side
                uint64_t j = 3 + (side == 1 ? (uint64_t)(dep[0] >= 2 ? dep[0] - 1 : 0) : 0);
                int32_t v = w;
                for (int32_t l = dep[side]; l >= 2; --l) {
                    const uint64_t u = dr.get(j++);
                    int32_t p = -2;
                    if (!fp && l - 1 <= LMAX) {
                        const int32_t llo = sm.loff[side][l - 1], lhi = sm.loff[side][l];
                        const int64_t dv = a.g.rp[v + 1] - a.g.rp[v];
                        if (2 * (int64_t)(lhi - llo) < dv)
                            p = pick_pred_layer<BS, SP>(sm, c, side, v, llo, lhi, u, lane, wid * cap, cap);
                    }
                    if (p == -2) p = pick_pred<SP>(c, side, v, l, u, lane);
                    if (p < 0) {   // no predecessor found: report, stop this walk
                        if (lane == 0) a.stats->error = 3;
                        break;
                    }
                    if (lane == 0) {
                        count_vertex(a, sf, p);
                        if (prow) prow[side == 0 ? (l - 1) : (d - (l - 1))] = a.g.orig[p];
                    }
                    cnt += 1;
                    v = p;
                }
            }
            if (lane == 0 && cnt) atomicAdd(&sm.pathc, (int32_t)cnt);
        }
        __syncthreads();
        if (tid == 0) {
            st_path += (unsigned long long)sm.pathc;
            if (a.info) {
                int64_t *inf = a.info + (size_t)sid * KAD_INFO_WIDTH;
                inf[0] = a.g.orig[sm.s];
                inf[1] = a.g.orig[sm.t];
                inf[2] = d;
                inf[3] = a.g.orig[sm.w];
                inf[4] = fp;
                inf[5] = m;
                inf[6] = steps;
                inf[7] = (int64_t)edges;
                t_walk = wall_clock64() - t_mark;
                inf[8] = (int64_t)(wall_clock64() - t_begin);   // ticks of the constant wall clock
                inf[9] = attempts;
                inf[10] = (int64_t)t_exp;
                inf[11] = (int64_t)t_mw;
                inf[12] = (int64_t)t_ch;
                inf[13] = (int64_t)t_walk;
            }
        }
        st_edges += edges;
        st_fp += fp ? 1 : 0;
        st_samples += 1;
        __syncthreads();
    }
    // flush statistics
    unsigned long long pred = ls.pred, vis = ls.visited;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        pred += __shfl_xor(pred, o);
        vis += __shfl_xor(vis, o);
    }
    if (lane == 0) {
        if (pred) atomicAdd(&a.stats->pred_edges, pred);
        if (vis) atomicAdd(&a.stats->visited, vis);
    }
    if (tid == 0) {
        atomicAdd(&a.stats->edges, st_edges);
        atomicAdd(&a.stats->expanded, st_exp);
        atomicAdd(&a.stats->path_vertices, st_path);
        atomicAdd(&a.stats->fp_samples, st_fp);
        atomicAdd(&a.stats->samples, st_samples);
        atomicAdd(&a.stats->edges_all, st_all);
    }
}

}  // namespace

int sampler_max_block() { return 1024; }

int sampler_blocks_per_cu(int block, bool sparse)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define KAD_OCC(B)                                                                                          \
    case B:                                                                                                 \
        e = sparse ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<B, true>, B, 0)           \
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample<B, false>, B, 0);         \
        break;
    switch (block) {
        KAD_OCC(64)
        KAD_OCC(128)
        KAD_OCC(256)
        KAD_OCC(512)
        KAD_OCC(1024)
    default: break;
    }
#undef KAD_OCC
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_sampler(const SampleLaunch &a, int slots, int block, hipStream_t st)
{
#define KAD_LAUNCH(B)                                                                                       \
    case B:                                                                                                 \
        if (a.sparse) hipLaunchKernelGGL((k_sample<B, true>), dim3(slots), dim3(B), 0, st, a);             \
        else hipLaunchKernelGGL((k_sample<B, false>), dim3(slots), dim3(B), 0, st, a);                     \
        break;
    switch (block) {
        KAD_LAUNCH(64)
        KAD_LAUNCH(128)
        KAD_LAUNCH(256)
        KAD_LAUNCH(512)
        KAD_LAUNCH(1024)
    default: return hipErrorInvalidValue;
    }
#undef KAD_LAUNCH
    return hipGetLastError();
}

}  // namespace kad
