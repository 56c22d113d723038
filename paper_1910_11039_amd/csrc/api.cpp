// Host driver behind the C-ABI (include/kadabra.h): contexts, graph upload,
// sampler state, the epoch loop and the phases of a run (Sec. III-A:
// diameter -> omega, calibration of delta_L/delta_U, adaptive sampling).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "kad_internal.h"

using namespace kad;

namespace {

thread_local std::string g_err;

kad_status fail(kad_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(KAD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Device scratch of kad_count_samples_noalloc: a file-scope array, one copy
// per GPU, held until the process ends.  Its device address is taken once
// per device (kad_create) with hipGetSymbolAddress; host code uses only that
// address, never the array's name.
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)KAD_NOALLOC_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[MAX_DEVICES];
}  // namespace
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Called with `device` current.
static kad_status scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(KAD_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return KAD_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(KAD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (unsigned char *)p;
    return KAD_OK;
}

struct kad_ctx {
    int device;
    hipStream_t stream;
    bool own_stream;
    int cu_count;
    // Streams of slot pools 1..3 (pool 0 runs on `stream`), shared by every
    // sampler of the context and created right after `stream`: HIP deals its
    // hardware queues (four by default) to streams in creation order, and
    // streams created per sampler could leave two pools on one queue, where
    // they run one after the other.  side[2] also carries the learned
    // prior's network beside the bracket's BFS.
    hipStream_t side[3];
};

struct kad_graph {
    kad_ctx *ctx;
    int device;
    int32_t n;
    int64_t nnz;
    int64_t *d_rp;       // internal (hub-first) numbering
    int32_t *d_ci;
    int32_t *d_orig;     // internal id -> caller id
    int32_t *d_newid;    // caller id -> internal id
    int32_t *d_cci;      // rows in the caller's order
    uint32_t *d_deg;
    int32_t nruns;                      // runs of equal degree (descending)
    int32_t *d_run_start;               // nruns + 1 entries
    uint32_t *d_run_deg;                // nruns entries
    std::vector<int32_t> h_run_start;
    DevGraph dev() const { return DevGraph{n, nnz, d_rp, d_ci, d_orig, d_newid, d_cci, d_deg}; }
    DegreeRuns runs() const { return DegreeRuns{nruns, d_run_start, d_run_deg, h_run_start.data()}; }
};

struct kad_sampler {
    kad_ctx *ctx;
    int device;
    const kad_graph *g;
    kad_opts o;
    double omega;
    int64_t vd_lo, vd_hi;
    unsigned long long cap;
    uint32_t E;
    int slots, block, inflight;
    // P slot pools, state frames and streams: epoch k uses pool, frame and
    // stream k mod P, so that later epochs sample while epoch k finishes
    // its tail
    int P;
    int cal_pool;   // pool index of the calibration's slots: P when memory holds a pool of its own, else 0
    hipStream_t sts[4];          // sts[0] is the context's stream
    hipEvent_t ev_merge[4];
    hipEvent_t ev_cal = nullptr;   // the allocation done on the calibration's stream
    std::vector<hipEvent_t> ev_ring;   // one per epoch in flight: its merge is done
    HostStatus *h_status, *d_status;   // pinned verdict mirror
    unsigned long long next_epoch;     // epochs enqueued since the reset
    // device state
    uint32_t *c, *sf[4], *cprime, *scratch_counts;
    double *LL, *LU, *lo_hi, *partials, *prior;
    double *LU_own;   // LU's buffer: LU points at LL when the allocation makes delta_L = delta_U
    Rec *recs;
    int32_t *queues, *mbufs;
    unsigned long long *macc;
    int32_t macc_cap;
    uint32_t *stamps;
    unsigned long long *work_ctr;
    unsigned long long *pool_epoch;   // replayed graphs: the next epoch of each pool, then the seed
    SampleStats *stats;
    SampleStats *cal_stats;   // the calibration's samples (they may run beside adaptive epochs)
    uint32_t *cal_hist = nullptr;   // histogram of the calibration counts, kept by its sampler
    double *cal_ltab = nullptr;     // L of each count value 0..tau0
    uint32_t cal_hist_top = 0;      // its last bin: tau0
    EpochState *es;
    void *hist;
    int32_t hist_cap;
    EpochState *h_es;   // pinned mirror
    // phases
    bool delta_ready, ran_alloc;
    uint64_t tau0;
    double C;
    std::vector<float> mlp_params, mlp_norm;
    bool have_mlp;
    // the learned prior's network output, computed on `aux` while the
    // bracket's BFS runs (it does not depend on omega)
    hipStream_t aux;
    hipEvent_t ev_aux;
    float *yhat;
    bool yhat_pending;
    // the network's inputs, kept for every run: features (n x 3), weights
    // and standardisation vector, the feature pass's workspace
    float *feat_buf = nullptr, *mlp_dev = nullptr;
    void *feat_ws = nullptr;
    kad_result res;
    double t_kernel_ms;
    uint32_t launches;
    hipGraphExec_t gexec;
    bool have_graph;
    bool tune_block;
    double tune_rate[3];     // samples/s of the trial per candidate block size
    // visited state: dense (a record per vertex in every slot) or hashed
    // (a table of 2^vlog2 buckets per slot; a sample that would fill more
    // than 3/4 of it is finished by a second launch on `fb` dense slots of
    // the pool, from the pool's defer list)
    bool sparse = false;
    uint32_t vlog2 = 0;
    size_t slot_n = 0;            // entries per slot in recs, queues and mbufs
    int32_t claim_limit = 0;
    int fb = 0;
    Rec *fb_recs = nullptr;
    int32_t *fb_queues = nullptr, *fb_mbufs = nullptr;
    unsigned long long *fb_macc = nullptr;
    uint32_t *fb_stamps = nullptr;
    uint32_t *defer = nullptr;    // KAD_DEFER_LISTS lists of defer_cap sample indices
    uint32_t defer_cap = 0;
    BfsCache *bfs_cache = nullptr;   // the bracket's BFS arrays, kept between runs
    ~kad_sampler()
    {
        if (bfs_cache) bfs_cache_free(bfs_cache, ctx ? ctx->stream : nullptr);
    }
    // plain allocation: the merges read L by calibration count (cprime,
    // cal_ltab), and the L arrays are filled only when fetched
    bool L_lazy = false;
    mutable bool L_pending = false;
    AllocArgs lazy_args{};
    double lazy_C = 0.0;
};

namespace {
// Sample counters in work_ctr: [0, 4) the pools' epochs, [4] the
// non-adaptive launches, then per defer list i a (deferred, fallback taken)
// pair at [8 + 2i]: lists 0..3 belong to the pools, list 4 to the
// non-adaptive launches.
constexpr int KAD_DEFER_LISTS = 5;
constexpr size_t KAD_WORK_CTRS = 8 + 2 * KAD_DEFER_LISTS;
constexpr uint32_t KAD_DEFER_CAP = 1u << 16;   // samples a hashed launch may defer: its count at most
// Dense fallback slots per pool: one.  The fallback launch sits between an
// epoch's sampler and its merge and usually has nothing to do, but each of
// its workgroups must still find a CU among those the other pools' samplers
// hold (the XCDs take a launch's workgroups in turn, so eight workgroups
// wait for a free CU in eight XCDs); a single workgroup waits least.
constexpr int KAD_FB_SLOTS = 1;
}  // namespace

extern "C" const char *kad_last_error(void) { return g_err.c_str(); }

extern "C" kad_status kad_create(int device, void *hip_stream, kad_ctx **out)
{
    if (!out) return fail(KAD_EINVAL, "out is null");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(KAD_EINVAL, "no such device");
    HIPCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos)
        return fail(KAD_EDEVICE, std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
    {
        const kad_status sr = scratch_init(device);
        if (sr != KAD_OK) return sr;
    }
    {
        // The stream-ordered allocations of a run (the bracket's BFS
        // arrays, about 0.6 GB on R-MAT 26, and smaller workspaces) stay in
        // the device's pool between runs instead of being unmapped at each
        // synchronisation and mapped again (1.2 ms a run on R-MAT 26).
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    kad_ctx *c = new kad_ctx();
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        hipError_t e = hipStreamCreate(&c->stream);
        if (e != hipSuccess) { delete c; return fail(KAD_EDEVICE, hipGetErrorString(e)); }
        c->own_stream = true;
    }
    for (int i = 0; i < 3; ++i) {
        hipError_t e = hipStreamCreate(&c->side[i]);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipStreamDestroy(c->side[j]);
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(KAD_EDEVICE, hipGetErrorString(e));
        }
    }
    *out = c;
    return KAD_OK;
}

extern "C" void kad_destroy(kad_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (int i = 0; i < 3; ++i) {
        (void)hipStreamSynchronize(ctx->side[i]);
        (void)hipStreamDestroy(ctx->side[i]);
    }
    if (ctx->own_stream) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
}

static kad_status validate_graph(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *ci)
{
    if (rp[0] != 0 || rp[n] != nnz) return fail(KAD_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] = nnz");
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) return fail(KAD_EINVAL, "row_ptr not monotone");
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t u = ci[e];
            if (u < 0 || u >= n) return fail(KAD_EINVAL, "column index out of range");
            if (u == v) return fail(KAD_EINVAL, "self loop");
            if (e > rp[v] && ci[e - 1] >= u) return fail(KAD_EINVAL, "row not strictly ascending");
            if (!std::binary_search(ci + rp[u], ci + rp[u + 1], v))
                return fail(KAD_EINVAL, "graph not symmetric");
        }
    }
    std::vector<int32_t> queue;
    std::vector<char> seen(n, 0);
    queue.reserve(n);
    queue.push_back(0);
    seen[0] = 1;
    for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t u = queue[h];
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e)
            if (!seen[ci[e]]) { seen[ci[e]] = 1; queue.push_back(ci[e]); }
    }
    if ((int32_t)queue.size() != n) return fail(KAD_ENOTCONNECTED, "graph is not connected");
    return KAD_OK;
}

extern "C" kad_status kad_graph_upload(kad_ctx *ctx, int32_t n, int64_t nnz, const int64_t *h_row_ptr,
                                       const int32_t *h_col_idx, uint32_t flags, kad_graph **out)
{
    if (!ctx || !out || !h_row_ptr || (nnz > 0 && !h_col_idx)) return fail(KAD_EINVAL, "null argument");
    if (n < 2) return fail(KAD_EINVAL, "need at least two vertices");
    if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(KAD_EOVERFLOW, "nnz must be below 2^31");
    if (h_row_ptr[n] != nnz) return fail(KAD_EINVAL, "row_ptr[n] != nnz");
    if (flags & KAD_GRAPH_VALIDATE) {
        kad_status st = validate_graph(n, nnz, h_row_ptr, h_col_idx);
        if (st != KAD_OK) return st;
    }
    HIPCHK(hipSetDevice(ctx->device));
    // hub-first numbering: a stable counting sort by descending degree
    std::vector<int32_t> orig(n), newid(n), run_start;
    std::vector<uint32_t> run_deg;
    std::vector<int64_t> rp2((size_t)n + 1);
    {
        int64_t maxdeg = 0;
        for (int32_t v = 0; v < n; ++v) maxdeg = std::max<int64_t>(maxdeg, h_row_ptr[v + 1] - h_row_ptr[v]);
        std::vector<int64_t> pos((size_t)maxdeg + 2, 0);
        for (int32_t v = 0; v < n; ++v) pos[(size_t)(maxdeg - (h_row_ptr[v + 1] - h_row_ptr[v])) + 1]++;
        for (size_t d = 1; d < pos.size(); ++d) pos[d] += pos[d - 1];
        for (int32_t v = 0; v < n; ++v) {
            const int32_t i = (int32_t)pos[(size_t)(maxdeg - (h_row_ptr[v + 1] - h_row_ptr[v]))]++;
            orig[i] = v;
            newid[v] = i;
        }
        rp2[0] = 0;
        for (int32_t i = 0; i < n; ++i) rp2[i + 1] = rp2[i] + (h_row_ptr[orig[i] + 1] - h_row_ptr[orig[i]]);
        // runs of equal degree: pos[j] now ends the vertices of degree maxdeg - j
        for (size_t j = 0; j + 1 < pos.size(); ++j) {
            const int64_t b = j == 0 ? 0 : pos[j - 1];
            if (pos[j] > b) {
                run_start.push_back((int32_t)b);
                run_deg.push_back((uint32_t)(maxdeg - (int64_t)j));
            }
        }
        run_start.push_back(n);
    }
    kad_graph *g = new kad_graph();
    g->ctx = ctx;
    g->device = ctx->device;
    g->n = n;
    g->nnz = nnz;
    int64_t *t_rp = nullptr;
    int32_t *t_ci = nullptr;
    const size_t ci_bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1);
    if (hipMalloc((void **)&g->d_rp, sizeof(int64_t) * ((size_t)n + 1)) != hipSuccess ||
        hipMalloc((void **)&g->d_ci, ci_bytes) != hipSuccess ||
        hipMalloc((void **)&g->d_orig, sizeof(int32_t) * (size_t)n) != hipSuccess ||
        hipMalloc((void **)&g->d_newid, sizeof(int32_t) * (size_t)n) != hipSuccess ||
        hipMalloc((void **)&g->d_cci, ci_bytes) != hipSuccess ||
        hipMalloc((void **)&g->d_deg, sizeof(uint32_t) * (size_t)n) != hipSuccess ||
        hipMalloc((void **)&g->d_run_start, sizeof(int32_t) * run_start.size()) != hipSuccess ||
        hipMalloc((void **)&g->d_run_deg, sizeof(uint32_t) * run_deg.size()) != hipSuccess ||
        hipMalloc((void **)&t_rp, sizeof(int64_t) * ((size_t)n + 1)) != hipSuccess ||
        hipMalloc((void **)&t_ci, ci_bytes) != hipSuccess) {
        (void)hipFree(g->d_rp);
        (void)hipFree(g->d_ci);
        (void)hipFree(g->d_orig);
        (void)hipFree(g->d_newid);
        (void)hipFree(g->d_cci);
        (void)hipFree(g->d_deg);
        (void)hipFree(g->d_run_start);
        (void)hipFree(g->d_run_deg);
        (void)hipFree(t_rp);
        (void)hipFree(t_ci);
        delete g;
        return fail(KAD_ENOMEM, "graph allocation failed");
    }
    hipStream_t st = ctx->stream;
    HIPCHK(hipMemcpyAsync(t_rp, h_row_ptr, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, st));
    if (nnz > 0) HIPCHK(hipMemcpyAsync(t_ci, h_col_idx, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->d_rp, rp2.data(), sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->d_orig, orig.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->d_newid, newid.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->d_run_start, run_start.data(), sizeof(int32_t) * run_start.size(),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(g->d_run_deg, run_deg.data(), sizeof(uint32_t) * run_deg.size(), hipMemcpyHostToDevice,
                          st));
    g->nruns = (int32_t)run_deg.size();
    g->h_run_start = std::move(run_start);
    HIPCHK(launch_relabel_rows(n, t_rp, t_ci, g->d_orig, g->d_newid, g->d_rp, g->d_cci, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(t_rp));
    HIPCHK(hipFree(t_ci));
    if (nnz > 0) HIPCHK(sort_rows(n, nnz, g->d_rp, g->d_cci, g->d_ci, st));
    HIPCHK(launch_degrees(n, g->d_rp, g->d_deg, st));
    HIPCHK(hipStreamSynchronize(st));
    *out = g;
    return KAD_OK;
}

extern "C" void kad_graph_free(kad_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    (void)hipFree(g->d_rp);
    (void)hipFree(g->d_ci);
    (void)hipFree(g->d_orig);
    (void)hipFree(g->d_newid);
    (void)hipFree(g->d_cci);
    (void)hipFree(g->d_deg);
    (void)hipFree(g->d_run_start);
    (void)hipFree(g->d_run_deg);
    delete g;
}

extern "C" double kad_omega(int64_t vd_lo, int64_t vd_hi, double eps, double delta)
{
    auto om = [&](int64_t vd) {
        double lg = 0.0;
        if (vd - 2 >= 1) {
            int64_t x = vd - 2, fl = 0;
            while (x > 1) { x >>= 1; ++fl; }
            lg = (double)fl;
        }
        return 0.5 / (eps * eps) * (lg + 1.0 + log(2.0 / delta));
    };
    const double lo = om(vd_lo), hi = om(vd_hi);
    return lo == hi ? lo : hi;
}

extern "C" kad_status kad_exact_vd(kad_ctx *ctx, const kad_graph *g, int64_t *h_vd, int32_t *h_witness,
                                   int64_t *h_bfs)
{
    if (!ctx || !g || !h_vd) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    int64_t lo = 0, hi = 0;
    HIPCHK(device_exact_vd(g->dev(), ctx->stream, false, 0.0, 0.0, 2000, &lo, &hi, h_witness, h_bfs));
    if (lo != hi) return fail(KAD_EOVERFLOW, "the exact diameter search did not settle within its BFS budget");
    *h_vd = lo;
    return KAD_OK;
}

// Phase 1 (Sec. III-A): the vertex-diameter bracket behind omega, from the
// three sweeps, or refined on the device until omega is settled.
static hipError_t omega_bracket(const kad_sampler *s, int64_t *lo, int64_t *hi);

extern "C" kad_status kad_vd_bracket(kad_ctx *ctx, const kad_graph *g, int64_t *vd_lo, int64_t *vd_hi)
{
    if (!ctx || !g || !vd_lo || !vd_hi) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(device_vd_bracket(g->dev(), ctx->stream, vd_lo, vd_hi));
    return KAD_OK;
}

static kad_status enqueue_network(kad_sampler *s, hipStream_t st);

static hipError_t omega_bracket(const kad_sampler *s, int64_t *lo, int64_t *hi)
{
    if (s->o.exact_diameter)
        return device_exact_vd(s->g->dev(), s->ctx->stream, true, s->o.epsilon, s->o.delta, 64, lo, hi, nullptr,
                               nullptr);
    return device_vd_bracket(s->g->dev(), s->ctx->stream, lo, hi, s->bfs_cache);
}

static void free_sampler(kad_sampler *s)
{
    if (s->have_graph) (void)hipGraphExecDestroy(s->gexec);
    for (hipEvent_t e : s->ev_ring) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ev_merge) if (e) (void)hipEventDestroy(e);
    // the streams are the context's: wait for this sampler's work on them
    for (int i = 0; i < 4; ++i) if (s->sts[i]) (void)hipStreamSynchronize(s->sts[i]);
    if (s->aux) (void)hipStreamSynchronize(s->aux);
    if (s->ev_aux) (void)hipEventDestroy(s->ev_aux);
    if (s->ev_cal) (void)hipEventDestroy(s->ev_cal);
    if (s->cal_hist) (void)hipFree(s->cal_hist);
    if (s->cal_ltab) (void)hipFree(s->cal_ltab);
    if (s->yhat) (void)hipFree(s->yhat);
    if (s->feat_buf) (void)hipFree(s->feat_buf);
    if (s->mlp_dev) (void)hipFree(s->mlp_dev);
    if (s->feat_ws) (void)hipFree(s->feat_ws);
    if (s->h_status) (void)hipHostFree(s->h_status);
    void *ptrs[] = {s->c, s->sf[0], s->sf[1], s->sf[2], s->sf[3], s->cprime, s->scratch_counts, s->LL, s->LU_own, s->lo_hi, s->macc,
                    s->partials, s->prior, s->recs, s->queues, s->mbufs, s->stamps, s->work_ctr, s->pool_epoch,
                    s->stats, s->cal_stats, s->es, s->hist, s->fb_recs, s->fb_queues, s->fb_mbufs, s->fb_macc,
                    s->fb_stamps, s->defer};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->h_es) (void)hipHostFree(s->h_es);
    delete s;
}

extern "C" void kad_sampler_free(kad_sampler *s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    free_sampler(s);
}

static kad_status reset_epochs(kad_sampler *s)
{
    hipStream_t st = s->ctx->stream;
    EpochState init;
    memset(&init, 0, sizeof(init));
    init.all_ok = 1;
    const double inf = INFINITY;
    memcpy(&init.min_margin_bits, &inf, sizeof(double));
    init.range[0] = 0;
    init.range[1] = std::min<unsigned long long>(s->E, s->cap);
    init.range[2] = 0;
    HIPCHK(hipMemcpyAsync(s->es, &init, sizeof(init), hipMemcpyHostToDevice, st));
    // n-sized clears by a kernel: the runtime's fill ran at a tenth of the
    // HBM bandwidth on these sizes
    HIPCHK(launch_zero_words(s->c, (size_t)s->g->n, st));
    for (int i = 0; i < s->P; ++i) HIPCHK(launch_zero_words(s->sf[i], (size_t)s->g->n, st));
    HIPCHK(hipMemsetAsync(s->work_ctr, 0, KAD_WORK_CTRS * sizeof(unsigned long long), st));
    {
        // pool p starts at epoch p; the run's seed for replayed graphs
        const unsigned long long pe[5] = {0, 1, 2, 3, (unsigned long long)s->o.seed};
        HIPCHK(hipMemcpyAsync(s->pool_epoch, pe, sizeof(pe), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemsetAsync(s->stats, 0, sizeof(SampleStats), st));
    HIPCHK(hipStreamSynchronize(st));
    if (s->h_status) memset(s->h_status, 0, sizeof(HostStatus));
    s->next_epoch = 0;
    return KAD_OK;
}

static kad_status count_into(kad_sampler *s, uint64_t stream, uint64_t first, uint64_t count,
                             uint32_t *target, int32_t *paths, int64_t *info, int32_t max_len,
                             SampleStats *stats = nullptr, hipStream_t on = nullptr,
                             uint32_t *hist = nullptr, uint32_t hist_top = 0);

// Autotuner (workgroup shape and samples per epoch).  Workgroup size:
// each candidate (256, 512, 1024 threads, each with one full wave of
// slots) samples the same trial -- four rounds of the widest wave -- on
// the tuning stream (counts discarded), timed with HIP events; when
// samples are short, each then samples sixteen rounds of its own wave.  Fewer,
// wider workgroups trade parallelism inside a sample for a smaller combined
// visited-state footprint, and the balance depends on the graph.  With
// short samples the widest shape within 5% of the fastest wins; with long
// ones the fastest, but 1024 is kept within 5% of it.  Epoch size: see
// the end of autotune().
static int cands_block(int i)
{
    static const int c[3] = {256, 512, 1024};
    return c[i];
}

static kad_status autotune(kad_sampler *s)
{
    hipStream_t st = s->ctx->stream;
    if (s->tune_block) {
        const int cands[3] = {cands_block(0), cands_block(1), cands_block(2)};
        double best = -1.0;
        int best_b = 256, best_slots = s->slots;
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const int all_slots = s->slots;
        const uint64_t N = 4ull * (uint64_t)all_slots;
        // pass 0: the same trial for every shape; pass 1, only when samples
        // are short: sixteen rounds of each shape's own wave, the share of
        // an epoch that the epoch-size rule below gives it, so that a shape
        // with more slots is not judged on a trial dominated by its tail
        bool short_samples = false;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                int fastest = 0;
                for (int i = 1; i < 3; ++i)
                    if (s->tune_rate[i] > s->tune_rate[fastest]) fastest = i;
                const int sl = std::min(all_slots, s->ctx->cu_count * sampler_blocks_per_cu(cands[fastest], s->sparse));
                if ((double)sl / s->tune_rate[fastest] > 0.010) break;
                short_samples = true;
                best = -1.0;
            }
            for (int i = 0; i < 3; ++i) {
                const int b = cands[i];
                const int sl = std::min(all_slots, s->ctx->cu_count * sampler_blocks_per_cu(b, s->sparse));
                const uint64_t trial = pass == 0 ? N : 16ull * (uint64_t)sl;
                s->block = b;
                s->slots = sl;
                HIPCHK(hipMemsetAsync(s->scratch_counts, 0, 4ull * s->g->n, st));
                HIPCHK(hipEventRecord(e0, st));
                kad_status r = count_into(s, KAD_STREAM_TUNE, 0, trial, s->scratch_counts, nullptr, nullptr, 0);
                if (r != KAD_OK) return r;
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                const double rate = (double)trial / (ms * 1e-3);
                s->tune_rate[i] = rate;
                best = std::max(best, rate);
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // short samples: the widest shape within 5% of the fastest, so that
        // timing noise between near-equal shapes does not flip the choice
        // from run to run; long samples (one trial of few rounds): the
        // fastest, but the 1024-thread shape within 5% of it
        int pick = 0;
        if (short_samples) {
            for (int i = 0; i < 3; ++i)
                if (s->tune_rate[i] >= 0.95 * best) pick = i;
        } else {
            for (int i = 1; i < 3; ++i)
                if (s->tune_rate[i] > s->tune_rate[pick]) pick = i;
            if (s->tune_rate[2] >= 0.95 * best) pick = 2;
        }
        best_b = cands[pick];
        best_slots = std::min(all_slots, s->ctx->cu_count * sampler_blocks_per_cu(cands[pick], s->sparse));
        s->block = best_b;
        s->slots = best_slots;
        HIPCHK(hipMemsetAsync(s->stats, 0, sizeof(SampleStats), st));
    }
    if (s->E == 0) {
        // Long samples (a slot takes over 10 ms per sample at the trial's
        // rate, as on high-diameter graphs) get two rounds of the slot wave
        // per epoch, so the stop is not overshot by much.  Otherwise sixteen
        // rounds, which amortise the merge and the epoch's tail, but at
        // most omega / 16 samples so that the stop epoch's overshoot stays
        // small against the run.
        double rate = 0.0;
        for (int i = 0; i < 3; ++i)
            if (s->tune_block && cands_block(i) == s->block) rate = s->tune_rate[i];
        const bool long_samples = rate > 0.0 && (double)s->slots / rate > 0.010;
        uint64_t E;
        if (long_samples) {
            E = 2ull * (uint64_t)s->slots;
        } else {
            E = 16ull * (uint64_t)s->slots;
            E = std::min<uint64_t>(E, (uint64_t)(s->omega / 16.0));
        }
        E = (E + 255) / 256 * 256;
        s->E = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(E, 256), 16384);
    }
    return KAD_OK;
}

extern "C" kad_status kad_sampler_init(kad_ctx *ctx, const kad_graph *g, const kad_opts *o,
                                       kad_sampler **out)
{
    if (!ctx || !g || !o || !out) return fail(KAD_EINVAL, "null argument");
    if (!(o->epsilon > 0.0 && o->epsilon < 1.0)) return fail(KAD_EINVAL, "epsilon must lie in (0, 1)");
    if (!(o->delta > 0.0 && o->delta < 1.0)) return fail(KAD_EINVAL, "delta must lie in (0, 1)");
    if (o->alloc_mode < 0 || o->alloc_mode > 2) return fail(KAD_EINVAL, "bad alloc_mode");
    if (o->sigma_mode < 0 || o->sigma_mode > 1) return fail(KAD_EINVAL, "bad sigma_mode");
    int block = o->block_size ? o->block_size : 256;
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return fail(KAD_EINVAL, "block_size must be 64, 128, 256, 512 or 1024");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    kad_sampler *s = new kad_sampler();
    s->bfs_cache = bfs_cache_create();
    memset(&s->res, 0, sizeof(s->res));
    s->ctx = ctx;
    s->device = ctx->device;
    s->g = g;
    s->o = *o;
    s->block = block;
    const int32_t n = g->n;

    // Phase 1 (Sec. III-A): omega from the vertex-diameter bracket.
    const double t0 = now_ms();
    if (o->omega_override > 0.0) {
        s->omega = o->omega_override;
        s->vd_lo = s->vd_hi = 0;
    } else {
        hipError_t e = omega_bracket(s, &s->vd_lo, &s->vd_hi);
        if (e != hipSuccess) { delete s; return fail(KAD_EDEVICE, hipGetErrorString(e)); }
        s->omega = kad_omega(s->vd_lo, s->vd_hi, o->epsilon, o->delta);
    }
    s->res.t_omega_ms = now_ms() - t0;
    s->cap = (unsigned long long)ceil(s->omega);

    // Slots: as many concurrent samples as fit the visited-state budget.
    // Persistent workgroups: more slots than can be resident would only
    // start once resident ones exit, so the default is one full wave of
    // them.  With block_size = 0 the pools are sized for the largest wave
    // among the candidate block sizes and the autotuner picks one below.
    if (o->visited_mode < 0 || o->visited_mode > 2) {
        delete s;
        return fail(KAD_EINVAL, "visited_mode must be 0 (auto), 1 (dense) or 2 (hashed)");
    }
    if (o->visited_log2 != 0 && (o->visited_log2 < 10 || o->visited_log2 > 26)) {
        delete s;
        return fail(KAD_EINVAL, "visited_log2 must be 0 (auto) or within [10, 26]");
    }
    const size_t macc_bytes = 16ull * (size_t)std::min<int64_t>(n, 1 << 16);
    const size_t per_dense = (size_t)n * (sizeof(Rec) + 2 * sizeof(int32_t)) + macc_bytes;
    // hashed table: 2^vlog2 buckets, by default the power of two at or above
    // n / 32 within [2^16, 2^22]
    uint32_t vlog2 = (uint32_t)o->visited_log2;
    if (vlog2 == 0) {
        vlog2 = 16;
        while (vlog2 < 22 && ((size_t)1 << vlog2) < (size_t)n / 32) ++vlog2;
    }
    const size_t per_sparse = ((size_t)1 << vlog2) * (sizeof(Rec) + 2 * sizeof(int32_t)) + macc_bytes;
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    size_t budget = o->visited_budget_bytes ? (size_t)o->visited_budget_bytes : free_b / 4 * 3;
    s->tune_block = o->block_size == 0;
    auto full_wave = [&](bool sp) {
        if (!s->tune_block) return ctx->cu_count * sampler_blocks_per_cu(block, sp);
        int w = 0;
        for (int b : {256, 512, 1024}) w = std::max(w, ctx->cu_count * sampler_blocks_per_cu(b, sp));
        return w;
    };
    if (o->pools < 0 || o->pools > 4) {
        delete s;
        return fail(KAD_EINVAL, "pools must be 0 (auto) or 1..4");
    }
    // Auto: hashed when the dense state holds fewer than 1.25 full waves of
    // 1024-thread slots (so that two dense pools would leave CUs idle), the
    // table is at most an eighth of a dense slot, and the graph is
    // small-world (vertex diameter at most 32 by the bracket), so that a
    // search claims a small share of the vertices and deferrals stay rare;
    // otherwise (and when omega was given, with no bracket) dense.  (On the
    // R-MAT and hyperbolic sweep, 2^23..2^26 vertices, hashed won where the
    // dense state held 1-1.1 waves: 15% and 34% at 2^26; where it held two
    // or more, dense was 6-25% faster.)
    s->sparse = o->visited_mode == KAD_VISITED_HASHED;
    if (o->visited_mode == KAD_VISITED_AUTO && o->slots <= 0) {
        const size_t wave1024 = (size_t)ctx->cu_count * (size_t)sampler_blocks_per_cu(1024, false);
        s->sparse = budget / per_dense * 4 < 5 * wave1024 && per_sparse * 8 <= per_dense && s->vd_hi > 0 &&
                    s->vd_hi <= 32;
    }
    // Hashed state without a given shape: 1024-thread workgroups, not the
    // trial's pick.  A trial times one launch; with four overlapped pools
    // the 512-thread shape it favoured ran R-MAT 26 to the stop in 69 ms
    // against 48 ms for 1024 threads.
    if (s->sparse && o->block_size == 0) {
        s->tune_block = false;
        block = 1024;
        s->block = block;
    }
    size_t pools_alloc = 0;
    if (s->sparse) {
        // every pool: a full wave of hashed slots, its dense fallback slots
        // and its defer list; four pools (or the requested number), fewer
        // when the budget does not hold them
        const int want = o->slots > 0 ? o->slots : std::min(full_wave(true), 1 << 16);
        const size_t pool_bytes = (size_t)want * per_sparse + (size_t)KAD_FB_SLOTS * per_dense;
        int P = o->pools > 0 ? o->pools : 4;
        while (o->pools == 0 && P > 1 && (size_t)P * pool_bytes > budget) --P;
        if ((size_t)P * pool_bytes > budget) {
            delete s;
            return fail(KAD_ENOMEM, "the hashed visited state of the requested pools and slots exceeds the budget");
        }
        s->slots = want;
        s->P = P;
        s->cal_pool = ((size_t)(P + 1) * pool_bytes <= budget) ? P : 0;
        s->vlog2 = vlog2;
        s->slot_n = (size_t)1 << vlog2;
        s->claim_limit = (int32_t)(s->slot_n / 4 * 3);
        s->fb = KAD_FB_SLOTS;
        s->defer_cap = KAD_DEFER_CAP;
    } else {
        const size_t per_slot = per_dense;
        int want = 0;
        if (o->slots > 0) want = o->slots;
        else want = full_wave(false);
        const size_t fit = budget / per_slot;
        if (fit < 1) {
            delete s;
            return fail(KAD_ENOMEM, "not even one sample slot fits the visited-state budget");
        }
        // pools: up to 4 while a full wave of slots fits each (epochs overlap
        // across pools); when fewer than two full waves fit, two pools of half
        // the slots (two concurrent epochs still cover every CU and fill each
        // other's tails); a single pool only when even that does not fit
        s->slots = (int)std::max<size_t>(1, std::min<size_t>((size_t)want, std::min<size_t>(fit, 1 << 16)));
        s->P = (int)std::max<size_t>(1, std::min<size_t>(4, fit / (size_t)s->slots));
        if (s->P == 1 && o->slots <= 0 && o->pools != 1 && fit / 2 >= (size_t)std::max(1, ctx->cu_count / 2)) {
            s->slots = (int)std::min<size_t>((size_t)s->slots, fit / 2);
            s->P = 2;
        }
        if (o->pools > 0) {
            if ((size_t)o->pools * (size_t)s->slots > fit) {
                delete s;
                return fail(KAD_ENOMEM, "requested pools exceed the visited-state budget");
            }
            s->P = o->pools;
        }
        if (o->slots > 0 && s->slots < o->slots) {
            delete s;
            return fail(KAD_ENOMEM, "requested slots exceed the visited-state budget");
        }
        // the calibration (and the other non-adaptive launches) get a pool of
        // their own when memory holds one, so that all P first epochs can run
        // beside the calibration
        s->cal_pool = ((size_t)(s->P + 1) * (size_t)s->slots <= fit) ? s->P : 0;
        s->slot_n = (size_t)n;
    }
    pools_alloc = (size_t)s->P + (s->cal_pool ? 1 : 0);
    s->E = o->epoch_size;
    s->inflight = o->epochs_in_flight > 0 ? o->epochs_in_flight : 4;
    s->macc_cap = (int32_t)std::min<int64_t>(n, 1 << 16);   // larger meet sets take the slow path
    // the history is sized for the smallest epoch the autotuner may choose
    s->hist_cap = (int32_t)((s->cap + (s->E ? s->E : 256) - 1) / (s->E ? s->E : 256) + 2);

    auto alloc = [&](void **p, size_t bytes) {
        return hipMalloc(p, std::max<size_t>(bytes, 16)) == hipSuccess;
    };
    const size_t sn = s->slot_n, nslots = pools_alloc * (size_t)s->slots, nfb = pools_alloc * (size_t)s->fb;
    bool ok = alloc((void **)&s->c, 4ull * n) && alloc((void **)&s->sf[0], 4ull * n) &&
              alloc((void **)&s->sf[1], 4ull * n) && alloc((void **)&s->sf[2], 4ull * n) &&
              alloc((void **)&s->sf[3], 4ull * n) && alloc((void **)&s->cprime, 4ull * n) &&
              alloc((void **)&s->scratch_counts, 4ull * n) && alloc((void **)&s->LL, 8ull * n) &&
              alloc((void **)&s->LU_own, 8ull * n) && alloc((void **)&s->lo_hi, 64) &&
              alloc((void **)&s->partials, 8 * alloc_partials(n)) && alloc((void **)&s->prior, 8ull * n) &&
              alloc((void **)&s->recs, sizeof(Rec) * sn * nslots) &&
              alloc((void **)&s->queues, 4ull * sn * nslots) &&
              alloc((void **)&s->mbufs, 4ull * sn * nslots) &&
              alloc((void **)&s->macc, 16ull * (size_t)s->macc_cap * nslots) &&
              alloc((void **)&s->stamps, 4ull * nslots) &&
              alloc((void **)&s->work_ctr, sizeof(unsigned long long) * KAD_WORK_CTRS) &&
              alloc((void **)&s->pool_epoch, 64) &&
              alloc((void **)&s->stats, sizeof(SampleStats)) && alloc((void **)&s->cal_stats, sizeof(SampleStats)) &&
              alloc((void **)&s->es, sizeof(EpochState)) &&
              alloc((void **)&s->hist, epoch_hist_bytes() * s->hist_cap);
    if (ok && s->sparse)
        ok = alloc((void **)&s->fb_recs, sizeof(Rec) * (size_t)n * nfb) &&
             alloc((void **)&s->fb_queues, 4ull * n * nfb) && alloc((void **)&s->fb_mbufs, 4ull * n * nfb) &&
             alloc((void **)&s->fb_macc, 16ull * (size_t)s->macc_cap * nfb) &&
             alloc((void **)&s->fb_stamps, 4ull * nfb) &&
             alloc((void **)&s->defer, 4ull * s->defer_cap * KAD_DEFER_LISTS);
    if (!ok || hipHostMalloc((void **)&s->h_es, sizeof(EpochState), 0) != hipSuccess ||
        hipHostMalloc((void **)&s->h_status, sizeof(HostStatus), hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&s->d_status, s->h_status, 0) != hipSuccess ||
        false) {
        free_sampler(s);
        return fail(KAD_ENOMEM, "sampler allocation failed");
    }
    s->LU = s->LU_own;
    s->sts[0] = st;
    for (int i = 0; i < s->P; ++i) {
        if (i > 0) s->sts[i] = s->ctx->side[i - 1];
        HIPCHK(hipEventCreateWithFlags(&s->ev_merge[i], hipEventDisableTiming));
    }
    s->ev_ring.resize(std::max(s->inflight, s->P) + 1);
    for (auto &e : s->ev_ring) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->ev_cal, hipEventDisableTiming));
    s->aux = s->ctx->side[2];
    HIPCHK(hipEventCreateWithFlags(&s->ev_aux, hipEventDisableTiming));
    // records start unstamped (a key of zero is nobody's): cleared by a kernel
    HIPCHK(launch_zero_words((uint32_t *)s->recs, sizeof(Rec) / 4 * sn * nslots, st));
    HIPCHK(launch_zero_words(s->stamps, nslots, st));
    if (s->sparse) {
        HIPCHK(launch_zero_words((uint32_t *)s->fb_recs, sizeof(Rec) / 4 * (size_t)n * nfb, st));
        HIPCHK(launch_zero_words(s->fb_stamps, nfb, st));
    }
    HIPCHK(launch_zero_words((uint32_t *)s->work_ctr, 2 * KAD_WORK_CTRS, st));
    kad_status rs = autotune(s);
    if (rs != KAD_OK) { free_sampler(s); return rs; }
    rs = reset_epochs(s);
    if (rs != KAD_OK) { free_sampler(s); return rs; }
    HIPCHK(hipStreamSynchronize(st));
    s->res.omega = s->omega;
    s->res.vd_lo = s->vd_lo;
    s->res.vd_hi = s->vd_hi;
    s->res.epoch_size = s->E;
    s->res.slots = s->slots;
    *out = s;
    return KAD_OK;
}

extern "C" kad_status kad_sampler_reset(kad_sampler *s, uint64_t seed)
{
    if (!s) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = s->ctx->stream;
    for (int i = 0; i < s->P; ++i) HIPCHK(hipStreamSynchronize(s->sts[i]));
    s->o.seed = seed;
    const double t0 = now_ms();
    if (s->o.alloc_mode == KAD_ALLOC_LEARNED && s->have_mlp) {
        // the network does not need omega: run it beside the bracket's BFS
        HIPCHK(hipStreamSynchronize(s->aux));
        kad_status r = enqueue_network(s, s->aux);
        if (r != KAD_OK) return r;
        HIPCHK(hipEventRecord(s->ev_aux, s->aux));
        s->yhat_pending = true;
    }
    if (!(s->o.omega_override > 0.0)) {
        HIPCHK(omega_bracket(s, &s->vd_lo, &s->vd_hi));
        const double om = kad_omega(s->vd_lo, s->vd_hi, s->o.epsilon, s->o.delta);
        if (om != s->omega) return fail(KAD_ESTATE, "omega changed for the same graph");
    }
    const double t_omega = now_ms() - t0;
    kad_status r = reset_epochs(s);
    if (r != KAD_OK) return r;
    if (s->o.alloc_mode != KAD_ALLOC_EXPLICIT) s->delta_ready = false;
    memset(&s->res, 0, sizeof(s->res));
    s->res.t_omega_ms = t_omega;
    s->res.omega = s->omega;
    s->res.vd_lo = s->vd_lo;
    s->res.vd_hi = s->vd_hi;
    s->res.epoch_size = s->E;
    s->res.slots = s->slots;
    s->t_kernel_ms = 0.0;
    s->launches = 0;
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

static SampleLaunch base_launch(kad_sampler *s, int pool = 0)
{
    const size_t sn = s->slot_n, sl = (size_t)s->slots * pool;
    SampleLaunch a;
    memset(&a, 0, sizeof(a));
    a.g = s->g->dev();
    a.seed = s->o.seed;
    a.stream = KAD_STREAM_ADS;
    a.sf[0] = s->sf[0];
    a.sf[1] = s->sf[1];
    a.recs = s->recs + sl * sn;
    a.queues = s->queues + sl * sn;
    a.mbufs = s->mbufs + sl * sn;
    a.macc = s->macc + sl * 2 * (size_t)s->macc_cap;
    a.macc_cap = s->macc_cap;
    a.stamps = s->stamps + sl;
    a.work_ctr = s->work_ctr + pool;
    a.stats = s->stats;
    a.sigma_fp = s->o.sigma_mode == KAD_SIGMA_FP;
    return a;
}

// Launches `a` (built by base_launch for `pool`) on `slots` workgroups.
// Hashed state: the hashed launch runs, then the pool's dense fallback
// slots finish the samples it deferred (a launch that exits at once when
// there are none).  The two counters of defer list `list` must be zero:
// with `clear` a kernel clears them first (the epochs' lists are cleared
// by the reset and then by each merge, so that no extra launch waits for
// a CU between an epoch's sampler and the previous merge).  Everything is
// enqueued on `st`, with kernels only, so that the sequence may be
// captured in a graph.
static unsigned long long *defer_counters(kad_sampler *s, int list) { return s->work_ctr + 8 + 2 * list; }

static hipError_t launch_pool(kad_sampler *s, SampleLaunch a, int pool, int list, int slots, hipStream_t st,
                              bool clear)
{
    if (!s->sparse) return launch_sampler(a, slots, s->block, st);
    unsigned long long *dc = defer_counters(s, list);
    hipError_t e = hipSuccess;
    if (clear && (e = launch_zero_words(reinterpret_cast<uint32_t *>(dc), 4, st)) != hipSuccess) return e;
    a.sparse = 1;
    a.vcap_log2 = s->vlog2;
    a.claim_limit = s->claim_limit;
    a.defer_list = s->defer + (size_t)list * s->defer_cap;
    a.defer_count = dc;
    a.defer_cap = s->defer_cap;
    e = launch_sampler(a, slots, s->block, st);
    if (e != hipSuccess) return e;
    const size_t n = (size_t)s->g->n, fl = (size_t)s->fb * pool;
    SampleLaunch f = a;
    f.sparse = 0;
    f.vcap_log2 = 0;
    f.claim_limit = 0;
    f.recs = s->fb_recs + fl * n;
    f.queues = s->fb_queues + fl * n;
    f.mbufs = s->fb_mbufs + fl * n;
    f.macc = s->fb_macc + fl * 2 * (size_t)s->macc_cap;
    f.stamps = s->fb_stamps + fl;
    f.work_ctr = dc + 1;
    f.defer_list = nullptr;
    f.defer_count = nullptr;
    f.defer_in = a.defer_list;
    f.defer_in_count = dc;
    return launch_sampler(f, s->fb, s->block, st);
}

// Non-adaptive samples [first, first+count) of `stream` counted into `target`.
static kad_status count_into(kad_sampler *s, uint64_t stream, uint64_t first, uint64_t count,
                             uint32_t *target, int32_t *paths, int64_t *info, int32_t max_len,
                             SampleStats *stats, hipStream_t on, uint32_t *hist, uint32_t hist_top)
{
    if (count == 0) return KAD_OK;
    hipStream_t st = on ? on : s->ctx->stream;
    // hashed state: launches of at most defer_cap samples, so that every
    // sample a launch defers has a place in the list
    const uint64_t chunk = s->sparse ? (uint64_t)s->defer_cap : count;
    for (uint64_t done = 0; done < count; done += chunk) {
        const uint64_t cnt = std::min<uint64_t>(chunk, count - done);
        SampleLaunch a = base_launch(s, s->cal_pool);
        if (stats) a.stats = stats;
        a.work_ctr = s->work_ctr + 4;   // a counter of its own: pool 0's stays at zero for its epochs
        a.stream = stream;
        a.first = first + done;
        a.count = cnt;
        a.sf[0] = target;
        a.sf[1] = target;
        a.paths = paths ? paths + done * (uint64_t)max_len : nullptr;
        a.info = info ? info + done * (uint64_t)KAD_INFO_WIDTH : nullptr;
        a.max_len = max_len;
        a.hist = hist;
        a.hist_top = hist_top;
        HIPCHK(launch_zero_words(reinterpret_cast<uint32_t *>(a.work_ctr), 2, st));
        const int slots = (int)std::min<uint64_t>(s->slots, cnt);
        HIPCHK(launch_pool(s, a, s->cal_pool, KAD_DEFER_LISTS - 1, slots, st, true));
    }
    return KAD_OK;
}

static kad_status check_stats_error(kad_sampler *s, const SampleStats *src = nullptr, hipStream_t on = nullptr)
{
    SampleStats h;
    hipStream_t st = on ? on : s->ctx->stream;
    HIPCHK(hipMemcpyAsync(&h, src ? src : s->stats, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h.error == 1) return fail(KAD_ENOTCONNECTED, "a sampled pair has no path: graph not connected");
    if (h.error == 2) return fail(KAD_EOVERFLOW, "a path is longer than max_len - 1");
    if (h.error == 3) return fail(KAD_EDEVICE, "internal error: a path choice found no candidate");
    if (h.error == 4) return fail(KAD_EDEVICE, "internal error: a launch deferred more samples than its list holds");
    if (h.error == 5) return fail(KAD_EDEVICE, "internal error: a reached vertex is missing from the hashed state");
    return KAD_OK;
}

extern "C" kad_status kad_set_delta(kad_sampler *s, const double *h_delta_L, const double *h_delta_U)
{
    if (!s || !h_delta_L || !h_delta_U) return fail(KAD_EINVAL, "null argument");
    const int32_t n = s->g->n;
    long double sum = 0.0L;
    for (int32_t v = 0; v < n; ++v) {
        if (!(h_delta_L[v] > 0.0 && h_delta_L[v] < 1.0 && h_delta_U[v] > 0.0 && h_delta_U[v] < 1.0))
            return fail(KAD_EINVAL, "delta values must lie in (0, 1)");
        sum += (long double)h_delta_L[v] + (long double)h_delta_U[v];
    }
    if (!(sum < 0.5L * (long double)s->o.delta))
        return fail(KAD_EINVAL, "sum of delta_L + delta_U must stay below delta / 2");
    s->LU = s->LU_own;   // delta_U may differ from delta_L here
    s->L_lazy = false;
    s->L_pending = false;
    // L = ln(1/delta) is taken once per vertex on the host in FP64 (the
    // C library's log), in the caller's numbering, then mapped in
    std::vector<double> Lh((size_t)n);
    HIPCHK(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    double *t = nullptr;
    HIPCHK(hipMallocAsync((void **)&t, 8ull * n, st));
    for (int side = 0; side < 2; ++side) {
        const double *d = side ? h_delta_U : h_delta_L;
        for (int32_t v = 0; v < n; ++v) Lh[(size_t)v] = -log(d[v]);
        HIPCHK(hipMemcpyAsync(t, Lh.data(), 8ull * n, hipMemcpyHostToDevice, st));
        HIPCHK(launch_from_caller_f64(n, s->g->d_orig, t, side ? s->LU : s->LL, st));
        HIPCHK(hipStreamSynchronize(st));   // Lh is refilled for the other side
    }
    HIPCHK(hipFreeAsync(t, st));
    HIPCHK(hipStreamSynchronize(st));
    s->delta_ready = true;
    return KAD_OK;
}

extern "C" kad_status kad_set_mlp_weights(kad_sampler *s, const float *h_params, const float *h_norm)
{
    if (!s || !h_params || !h_norm) return fail(KAD_EINVAL, "null argument");
    if (s->aux) HIPCHK(hipStreamSynchronize(s->aux));   // a pending output used the old weights
    s->yhat_pending = false;
    s->mlp_params.assign(h_params, h_params + 4481);
    s->mlp_norm.assign(h_norm, h_norm + 6);
    HIPCHK(hipSetDevice(s->device));
    const size_t n = (size_t)s->g->n;
    if (!s->yhat && hipMalloc((void **)&s->yhat, sizeof(float) * n) != hipSuccess) s->yhat = nullptr;
    if (!s->feat_buf && hipMalloc((void **)&s->feat_buf, sizeof(float) * 3 * n) != hipSuccess) s->feat_buf = nullptr;
    if (!s->mlp_dev && hipMalloc((void **)&s->mlp_dev, sizeof(float) * (4544 + 64)) != hipSuccess) s->mlp_dev = nullptr;
    if (!s->feat_ws && hipMalloc(&s->feat_ws, features_workspace_bytes(s->g->dev())) != hipSuccess) s->feat_ws = nullptr;
    if (!s->yhat || !s->feat_buf || !s->mlp_dev || !s->feat_ws)
        return fail(KAD_ENOMEM, "learned-prior buffers");
    // weights at the front, the standardisation vector 256-byte aligned behind
    HIPCHK(hipMemcpy(s->mlp_dev, h_params, sizeof(float) * 4481, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->mlp_dev + 4544, h_norm, sizeof(float) * 6, hipMemcpyHostToDevice));
    s->have_mlp = true;
    return KAD_OK;
}

// Network output of the learned prior, y = MLP(standardised features),
// enqueued on stream `st` into s->yhat.
static kad_status enqueue_network(kad_sampler *s, hipStream_t st)
{
    const int32_t n = s->g->n;
    HIPCHK(launch_features_ws(s->g->dev(), s->g->runs(), s->feat_buf, s->feat_ws, st));
    HIPCHK(launch_mlp_forward(s->mlp_dev, s->feat_buf, s->mlp_dev + 4544, n, s->yhat, st));
    return KAD_OK;
}

// Learned prior: features -> standardise -> MLP -> b_hat = max(0, e^y - 1/omega).
// The network part was started by the reset on the side stream when it
// is pending; otherwise it runs here.
static kad_status learned_prior(kad_sampler *s)
{
    hipStream_t st = s->ctx->stream;
    if (s->yhat_pending) {
        HIPCHK(hipStreamWaitEvent(st, s->ev_aux, 0));
        s->yhat_pending = false;
    } else {
        kad_status r = enqueue_network(s, st);
        if (r != KAD_OK) return r;
    }
    HIPCHK(launch_prior_from_mlp(s->g->n, s->yhat, s->omega, s->prior, st));
    return KAD_OK;
}

// Checks the allocation's budget on the device: every delta in (0, 1) and
// the sum of delta_L + delta_U below delta / 2.
static bool alloc_is_valid(kad_sampler *s)
{
    double sum = 0.0;
    bool finite = false;
    if (alloc_budget(s->g->n, s->LL, s->LU, s->ctx->stream, &sum, &finite) != hipSuccess) return false;
    return finite && sum <= 0.5 * s->o.delta;
}

// `after_calibration` (optional) runs once the calibration's sampler is
// enqueued, before the host waits for the allocation; `cal_stream`
// (optional) carries the calibration and the plain allocation.
static kad_status ensure_delta(kad_sampler *s, const std::function<kad_status()> &after_calibration = {},
                               hipStream_t cal_stream = nullptr)
{
    if (s->delta_ready) return KAD_OK;
    hipStream_t st = s->ctx->stream;
    const int32_t n = s->g->n;
    const double t0 = now_ms();
    AllocArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.delta = s->o.delta;
    a.beta = 1e-3;
    a.lo_hi = s->lo_hi;
    a.partials = s->partials;
    // the computed allocations have delta_L = delta_U: one array serves
    // both bounds, and the merges read it once
    s->LU = s->LL;
    a.LL = s->LL;
    a.LU = s->LU;
    bool learned = false;
    if (s->o.alloc_mode == KAD_ALLOC_EXPLICIT) return fail(KAD_ESTATE, "EXPLICIT mode needs kad_set_delta first");
    if (s->o.alloc_mode == KAD_ALLOC_LEARNED) {
        if (!s->have_mlp) return fail(KAD_ESTATE, "LEARNED mode needs kad_set_mlp_weights first");
        kad_status r = learned_prior(s);
        if (r != KAD_OK) return r;
        a.dense_prior = s->prior;
        s->L_lazy = false;
        s->L_pending = false;
        double C = 0.0;
        HIPCHK(run_alloc(a, st, &C));
        HIPCHK(hipStreamSynchronize(st));
        s->C = C;
        learned = alloc_is_valid(s);   // fallback to the plain allocation otherwise
    }
    if (!learned) {
        // Phase 2 (Sec. III-A): tau0 = ceil(omega / 100) non-adaptive samples on stream 1.
        s->tau0 = (uint64_t)ceil(s->omega / 100.0);
        hipStream_t cst = cal_stream ? cal_stream : st;
        const uint32_t top = (uint32_t)std::max<uint64_t>(1, s->tau0);
        if (s->cal_hist && s->cal_hist_top != top) {
            (void)hipFree(s->cal_hist);
            (void)hipFree(s->cal_ltab);
            s->cal_hist = nullptr;
            s->cal_ltab = nullptr;
        }
        if (!s->cal_hist) {
            if (hipMalloc((void **)&s->cal_hist, sizeof(uint32_t) * ((size_t)top + 1)) != hipSuccess ||
                hipMalloc((void **)&s->cal_ltab, sizeof(double) * ((size_t)top + 1)) != hipSuccess) {
                if (s->cal_hist) (void)hipFree(s->cal_hist);
                s->cal_hist = nullptr;
                s->cal_ltab = nullptr;
                return fail(KAD_ENOMEM, "calibration histogram allocation failed");
            }
            s->cal_hist_top = top;
        }
        HIPCHK(launch_zero_words(s->cprime, (size_t)n, cst));
        HIPCHK(hipMemsetAsync(s->cal_stats, 0, sizeof(SampleStats), cst));
        HIPCHK(hipMemsetAsync(s->cal_hist, 0, sizeof(uint32_t) * ((size_t)top + 1), cst));
        kad_status r = count_into(s, KAD_STREAM_CALIB, 0, s->tau0, s->cprime, nullptr, nullptr, 0, s->cal_stats, cst,
                                  s->cal_hist, top);
        if (r == KAD_OK && after_calibration) r = after_calibration();
        if (r != KAD_OK) return r;
        a.counts = s->cprime;
        a.tau0 = (double)s->tau0;
        a.hist = s->cal_hist;
        a.ltab = s->cal_ltab;
        // plain mode: the merges read L by count value; a learned run that
        // fell back builds the arrays (its merges read them)
        a.lazy = s->o.alloc_mode == KAD_ALLOC_PLAIN ? 1 : 0;
        double C = 0.0;
        HIPCHK(run_alloc(a, cst, &C));
        HIPCHK(hipStreamSynchronize(cst));
        s->C = C;
        s->L_lazy = a.lazy != 0;
        s->L_pending = s->L_lazy;
        s->lazy_args = a;
        s->lazy_C = C;
        r = check_stats_error(s, s->cal_stats, cst);
        if (r != KAD_OK) return r;
    }
    s->res.tau0 = learned ? 0 : s->tau0;
    s->res.t_alloc_ms = now_ms() - t0;
    s->delta_ready = true;
    return KAD_OK;
}

// Enqueue epoch k overlapped with its neighbours: epoch k uses stream,
// slot pool and state frame k mod P; its sampler runs after that stream's
// previous merge (which cleared the frame), and its merge waits for the
// merge of epoch k - 1, so c~ grows and the rule is checked in epoch order
// on exactly samples [0, tau).  A sampler whose epoch turns out to follow
// the stop quits at its next sample; its frame is never merged.
static kad_status enqueue_sampler_k(kad_sampler *s, unsigned long long k, hipEvent_t ev0, hipEvent_t ev1,
                                    int width = 0)
{
    const int p = (int)(k % (unsigned long long)s->P);
    hipStream_t st = s->sts[p];
    const unsigned long long first = k * s->E;
    const unsigned long long count = std::min<unsigned long long>(s->E, s->cap - first);
    SampleLaunch a = base_launch(s, p);
    a.first = first;
    a.count = count;
    a.sf[0] = a.sf[1] = s->sf[p];
    a.stop_flag = &s->es->stopped;
    // the pool's sample counter is zero here: set by the reset, then cleared
    // by the merge of this stream's previous epoch
    if (ev0) HIPCHK(hipEventRecord(ev0, st));
    const int w = width > 0 ? std::min(width, s->slots) : s->slots;
    HIPCHK(launch_pool(s, a, p, p, (int)std::min<unsigned long long>((unsigned long long)w, count), st, false));
    if (ev1) HIPCHK(hipEventRecord(ev1, st));
    return KAD_OK;
}

// The merge of epoch k: after epoch k - 1's merge (in host order too, so
// that the event it waits on is already recorded).
static kad_status enqueue_merge_k(kad_sampler *s, unsigned long long k)
{
    const int p = (int)(k % (unsigned long long)s->P);
    hipStream_t st = s->sts[p];
    if (k > 0) HIPCHK(hipStreamWaitEvent(st, s->ev_merge[(p + s->P - 1) % s->P], 0));
    HIPCHK(launch_merge_stop_impl(s->g->dev(), s->c, s->sf[p], s->sf[p], s->LL, s->LU, s->omega,
                                  s->o.epsilon, s->cap, s->E, s->es, s->work_ctr + p, s->hist, s->hist_cap,
                                  s->d_status, st, nullptr, 0, s->sparse ? defer_counters(s, p) : nullptr,
                                  s->L_lazy ? s->cprime : nullptr, s->L_lazy ? s->cal_ltab : nullptr));
    HIPCHK(hipEventRecord(s->ev_merge[p], st));
    HIPCHK(hipEventRecord(s->ev_ring[k % s->ev_ring.size()], st));
    return KAD_OK;
}

static kad_status enqueue_epoch_k(kad_sampler *s, unsigned long long k, hipEvent_t ev0, hipEvent_t ev1)
{
    kad_status r = enqueue_sampler_k(s, k, ev0, ev1);
    if (r != KAD_OK) return r;
    return enqueue_merge_k(s, k);
}

static kad_status read_state(kad_sampler *s)
{
    HIPCHK(hipMemcpyAsync(s->h_es, s->es, sizeof(EpochState), hipMemcpyDeviceToHost, s->ctx->stream));
    HIPCHK(hipStreamSynchronize(s->ctx->stream));
    return KAD_OK;
}

extern "C" kad_status kad_step_epoch(kad_sampler *s, int *stopped)
{
    if (!s || !stopped) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    kad_status r = ensure_delta(s);
    if (r != KAD_OK) return r;
    r = read_state(s);
    if (r != KAD_OK) return r;
    if (!s->h_es->stopped) {
        r = enqueue_epoch_k(s, s->next_epoch++, nullptr, nullptr);
        if (r != KAD_OK) return r;
        for (int i = 1; i < s->P; ++i) HIPCHK(hipStreamSynchronize(s->sts[i]));
        r = read_state(s);
        if (r != KAD_OK) return r;
        r = check_stats_error(s);
        if (r != KAD_OK) return r;
    }
    *stopped = s->h_es->stopped;
    return KAD_OK;
}

static kad_status fill_result(kad_sampler *s)
{
    SampleStats h;
    HIPCHK(hipMemcpy(&h, s->stats, sizeof(h), hipMemcpyDeviceToHost));
    kad_result &r = s->res;
    r.tau = s->h_es->tau;
    r.epochs = (uint32_t)s->h_es->epoch;
    r.stop_reason = s->h_es->reason;
    r.max_f = s->h_es->max_f;
    r.max_g = s->h_es->max_g;
    r.min_margin = s->h_es->min_margin;
    r.edges_scanned = (int64_t)h.edges;
    r.vertices_expanded = (int64_t)h.expanded;
    r.vertices_visited = (int64_t)h.visited;
    r.pred_edges = (int64_t)h.pred_edges;
    r.path_vertices = (int64_t)h.path_vertices;
    r.fp_samples = (int64_t)h.fp_samples;
    r.samples_run = (int64_t)h.samples;
    r.t_sample_kernel_ms = s->t_kernel_ms;
    r.sample_launches = s->launches;
    r.epoch_size = s->E;
    r.slots = s->slots;
    r.block_size = s->block;
    r.pools = s->P;
    r.visited_mode = s->sparse ? 2 : 1;
    r.visited_log2 = (int32_t)s->vlog2;
    r.deferred = (int64_t)h.deferred;
    return KAD_OK;
}

// The pooled epoch schedule captured as one graph: the epochs of a replay
// are dealt to the pools in turn, each pool's sampler reads its epoch from
// the device (its merge advances it by P), and every merge waits for the
// previous epoch's merge, so c~ grows and the rule is checked in epoch
// order.  A replay covers G epochs (a multiple of P, enough for the run
// unless omega is far away); samplers and merges after the stop return at
// once.  Streams join the capture through events; nothing is cleared with
// a memset node (the merges clear their frames and counters).
static kad_status build_graph(kad_sampler *s)
{
    hipStream_t st = s->ctx->stream;
    const unsigned long long total = (s->cap + s->E - 1) / s->E;
    const int per = (int)std::min<unsigned long long>(std::max<unsigned long long>((unsigned long long)s->P,
                                                                                 std::min<unsigned long long>(total, 16)),
                                                      64);
    const int G = (per + s->P - 1) / s->P * s->P;
    std::vector<hipEvent_t> evs((size_t)G + 2 * (size_t)s->P + 1);
    for (auto &e : evs) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    auto cleanup = [&]() {
        for (auto &e : evs) (void)hipEventDestroy(e);
    };
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    kad_status r = KAD_OK;
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && r == KAD_OK) r = fail(KAD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    size_t ev = 0;
    chk(hipEventRecord(evs[ev], st), "fork");
    for (int p = 1; p < s->P; ++p) chk(hipStreamWaitEvent(s->sts[p], evs[ev], 0), "fork wait");
    ++ev;
    hipEvent_t prev_merge = nullptr;
    for (int j = 0; j < G && r == KAD_OK; ++j) {
        const int p = j % s->P;
        hipStream_t sp = s->sts[p];
        SampleLaunch a = base_launch(s, p);
        a.dev_epoch = s->pool_epoch + p;
        a.dev_seed = reinterpret_cast<const uint64_t *>(s->pool_epoch + 4);
        a.E = s->E;
        a.cap = s->cap;
        a.sf[0] = a.sf[1] = s->sf[p];
        a.stop_flag = &s->es->stopped;
        chk(launch_pool(s, a, p, p, s->slots, sp, false), "sampler");
        if (prev_merge) chk(hipStreamWaitEvent(sp, prev_merge, 0), "merge order");
        chk(launch_merge_stop_impl(s->g->dev(), s->c, s->sf[p], s->sf[p], s->LL, s->LU, s->omega, s->o.epsilon,
                                   s->cap, s->E, s->es, s->work_ctr + p, s->hist, s->hist_cap, s->d_status, sp,
                                   s->pool_epoch + p, s->P, s->sparse ? defer_counters(s, p) : nullptr,
                                   s->L_lazy ? s->cprime : nullptr, s->L_lazy ? s->cal_ltab : nullptr),
            "merge");
        chk(hipEventRecord(evs[ev], sp), "merge event");
        prev_merge = evs[ev++];
    }
    for (int p = 1; p < s->P; ++p) {
        chk(hipEventRecord(evs[ev], s->sts[p]), "join");
        chk(hipStreamWaitEvent(st, evs[ev], 0), "join wait");
        ++ev;
    }
    const hipError_t ce = hipStreamEndCapture(st, &graph);
    if (r != KAD_OK) {
        if (ce == hipSuccess) (void)hipGraphDestroy(graph);
        cleanup();
        return r;
    }
    if (ce != hipSuccess) {
        cleanup();
        return fail(KAD_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    }
    const hipError_t ie = hipGraphInstantiate(&s->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    cleanup();
    if (ie != hipSuccess) return fail(KAD_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    s->have_graph = true;
    return KAD_OK;
}

extern "C" kad_status kad_run_to_stop(kad_sampler *s, kad_result *out)
{
    if (!s) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    const double t_start = now_ms();
    const bool timing = s->o.timing != 0;
    std::vector<hipEvent_t> evs;
    auto timing_events = [&](hipEvent_t *e0, hipEvent_t *e1) -> kad_status {
        *e0 = *e1 = nullptr;
        if (!timing) return KAD_OK;
        HIPCHK(hipEventCreate(e0));
        HIPCHK(hipEventCreate(e1));
        evs.push_back(*e0);
        evs.push_back(*e1);
        return KAD_OK;
    };
    // Adaptive samples do not depend on the delta allocation, only their
    // merges do: when a plain allocation is still to come, the first
    // epochs' samplers start on their pools right after the calibration's
    // sampler and fill its tail; the merges follow the allocation.  The
    // learned allocation is a chain of short launches that would wait for
    // CUs behind those samplers, so it runs first on an idle GPU.
    const unsigned long long total = (s->cap + s->E - 1) / s->E;
    // (a run already advanced epoch by epoch stays on the stream loop)
    const bool graph_path = s->o.use_graphs != 0 && s->next_epoch == 0;
    unsigned long long pre_hi = 0;
    kad_status r = read_state(s);   // the allocation does not touch the epoch state
    if (r != KAD_OK) return r;
    if (!s->delta_ready && s->o.alloc_mode == KAD_ALLOC_PLAIN && !graph_path && s->P > 1 &&
        s->next_epoch == 0 && !s->h_es->stopped)
        pre_hi = std::min<unsigned long long>((unsigned long long)s->P, total);
    // The calibration is enqueued first, so that its workgroups take the
    // CUs before the early samplers fill in behind it.  With slots of its
    // own it runs on the last pool's stream and only that pool's epoch
    // waits for the allocation; otherwise it uses pool 0 and epoch 0 waits.
    const bool own_cal = pre_hi > 0 && s->cal_pool != 0 && s->P > 1;
    const unsigned long long late = own_cal ? (unsigned long long)(s->P - 1) : 0;
    hipStream_t cst = own_cal ? s->sts[s->P - 1] : nullptr;
    // The early epochs share the slots between them and leave 16 free
    // (eight CUs' worth at two workgroups per CU), so that the allocation's
    // launches and the first merges find room instead of waiting for a
    // whole epoch launch to drain.
    const unsigned long long npre = pre_hi - (late < pre_hi ? 1 : 0);
    const int pre_width = npre > 0 ? std::max(1, (int)((s->slots - std::min(16, s->slots / 4)) / (int)npre)) : 0;
    r = ensure_delta(s, [&]() -> kad_status {
        for (unsigned long long k = 0; k < pre_hi; ++k) {
            if (k == late) continue;
            hipEvent_t e0, e1;
            kad_status rr = timing_events(&e0, &e1);
            if (rr == KAD_OK) rr = enqueue_sampler_k(s, k, e0, e1, pre_width);
            if (rr != KAD_OK) return rr;
        }
        return KAD_OK;
    }, cst);
    if (r != KAD_OK) return r;
    if (pre_hi > 0) {
        if (own_cal) {   // the merges see the delta arrays written on that stream
            HIPCHK(hipEventRecord(s->ev_cal, cst));
            HIPCHK(hipStreamWaitEvent(s->sts[0], s->ev_cal, 0));
        }
        if (late < pre_hi) {
            hipEvent_t e0, e1;
            r = timing_events(&e0, &e1);
            if (r == KAD_OK) r = enqueue_sampler_k(s, late, e0, e1);
        }
        for (unsigned long long k = 0; r == KAD_OK && k < pre_hi; ++k) r = enqueue_merge_k(s, k);
        if (r != KAD_OK) return r;
        s->next_epoch = pre_hi;
    }
    const double t_ads0 = now_ms();
    if (graph_path && !s->have_graph) {
        r = build_graph(s);
        if (r != KAD_OK) return r;
    }
    if (graph_path) {
        while (!s->h_es->stopped) {
            HIPCHK(hipGraphLaunch(s->gexec, st));
            r = read_state(s);
            if (r != KAD_OK) return r;
        }
    } else if (!s->h_es->stopped) {
        // Keep `inflight` epochs queued ahead of the newest verdict the host
        // has seen; the verdict of epoch k is polled from pinned memory once
        // its merge has completed.
        unsigned long long known = pre_hi > 0 ? 0 : s->next_epoch;
        for (;;) {
            while (s->next_epoch < total && s->next_epoch < known + (unsigned long long)s->inflight) {
                hipEvent_t e0, e1;
                r = timing_events(&e0, &e1);
                if (r != KAD_OK) return r;
                r = enqueue_epoch_k(s, s->next_epoch++, e0, e1);
                if (r != KAD_OK) return r;
            }
            HIPCHK(hipEventSynchronize(s->ev_ring[known % s->ev_ring.size()]));
            ++known;
            if (__atomic_load_n(&s->h_status->stopped, __ATOMIC_ACQUIRE)) break;
            if (known >= total) break;
        }
        for (int i = 0; i < s->P; ++i) HIPCHK(hipStreamSynchronize(s->sts[i]));
        r = read_state(s);
        if (r != KAD_OK) return r;
    }
    const double t_ads1 = now_ms();
    if (timing) {
        // every launch counts, speculative ones included: the work counters
        // cover their samples too
        for (size_t i = 0; i + 1 < evs.size(); i += 2) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
            s->t_kernel_ms += ms;
            s->launches += 1;
        }
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    }
    r = check_stats_error(s);
    if (r != KAD_OK) return r;
    s->res.t_ads_ms = t_ads1 - t_ads0;
    s->res.t_total_ms = s->res.t_omega_ms + (t_ads1 - t_start);
    r = fill_result(s);
    if (r != KAD_OK) return r;
    if (out) *out = s->res;
    return KAD_OK;
}

// Copies an n-sized per-vertex device array (internal numbering) to the
// host in the caller's numbering.
static kad_status copy_to_caller(const kad_graph *g, const uint32_t *d_in, uint32_t *h_out, hipStream_t st)
{
    uint32_t *t = nullptr;
    HIPCHK(hipMallocAsync((void **)&t, 4ull * g->n, st));
    HIPCHK(launch_to_caller_u32(g->n, g->d_orig, d_in, t, st));
    HIPCHK(hipMemcpyAsync(h_out, t, 4ull * g->n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipFreeAsync(t, st));
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

static kad_status copy_to_caller(const kad_graph *g, const double *d_in, double *h_out, hipStream_t st)
{
    double *t = nullptr;
    HIPCHK(hipMallocAsync((void **)&t, 8ull * g->n, st));
    HIPCHK(launch_to_caller_f64(g->n, g->d_orig, d_in, t, st));
    HIPCHK(hipMemcpyAsync(h_out, t, 8ull * g->n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipFreeAsync(t, st));
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

// The L arrays of a plain allocation, built from the count table when
// first needed (the merges read the table).
static kad_status ensure_L(const kad_sampler *s)
{
    if (!s->L_pending) return KAD_OK;
    HIPCHK(run_alloc_L(s->lazy_args, s->lazy_C, s->ctx->stream));
    HIPCHK(hipStreamSynchronize(s->ctx->stream));
    s->L_pending = false;
    return KAD_OK;
}

extern "C" kad_status kad_fetch_result(const kad_sampler *s, kad_result *out)
{
    if (!s || !out) return fail(KAD_EINVAL, "null argument");
    *out = s->res;
    return KAD_OK;
}

extern "C" kad_status kad_fetch_counts(const kad_sampler *s, uint32_t *h_c, uint64_t *h_tau)
{
    if (!s || !h_c) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    EpochState es;
    kad_status r = copy_to_caller(s->g, s->c, h_c, s->ctx->stream);
    if (r != KAD_OK) return r;
    HIPCHK(hipMemcpyAsync(&es, s->es, sizeof(es), hipMemcpyDeviceToHost, s->ctx->stream));
    HIPCHK(hipStreamSynchronize(s->ctx->stream));
    if (h_tau) *h_tau = es.tau;
    return KAD_OK;
}

static kad_status fetch_tau(const kad_sampler *s, double *tau)
{
    EpochState es;
    HIPCHK(hipMemcpyAsync(&es, s->es, sizeof(es), hipMemcpyDeviceToHost, s->ctx->stream));
    HIPCHK(hipStreamSynchronize(s->ctx->stream));
    if (es.tau == 0) return fail(KAD_ESTATE, "no samples merged yet");
    *tau = (double)es.tau;
    return KAD_OK;
}

extern "C" kad_status kad_fetch_btilde(const kad_sampler *s, double *h_b)
{
    if (!s || !h_b) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    double tau;
    kad_status r = fetch_tau(s, &tau);
    if (r != KAD_OK) return r;
    hipStream_t st = s->ctx->stream;
    double *d = nullptr;
    HIPCHK(hipMallocAsync((void **)&d, 8ull * s->g->n, st));
    HIPCHK(launch_btilde(s->g->n, s->c, tau, d, st));
    r = copy_to_caller(s->g, d, h_b, st);
    HIPCHK(hipFreeAsync(d, st));
    HIPCHK(hipStreamSynchronize(st));
    return r;
}

extern "C" kad_status kad_fetch_fg(const kad_sampler *s, double *h_f, double *h_g)
{
    if (!s || !h_f || !h_g) return fail(KAD_EINVAL, "null argument");
    if (!s->delta_ready) return fail(KAD_ESTATE, "delta allocation not done");
    HIPCHK(hipSetDevice(s->ctx->device));
    double tau;
    kad_status r = fetch_tau(s, &tau);
    if (r != KAD_OK) return r;
    hipStream_t st = s->ctx->stream;
    double *f = nullptr, *g = nullptr;
    r = ensure_L(s);
    if (r != KAD_OK) return r;
    HIPCHK(hipMallocAsync((void **)&f, 8ull * s->g->n, st));
    HIPCHK(hipMallocAsync((void **)&g, 8ull * s->g->n, st));
    HIPCHK(launch_fg(s->g->n, s->c, tau, s->LL, s->LU, s->omega, f, g, st));
    r = copy_to_caller(s->g, f, h_f, st);
    if (r == KAD_OK) r = copy_to_caller(s->g, g, h_g, st);
    HIPCHK(hipFreeAsync(f, st));
    HIPCHK(hipFreeAsync(g, st));
    HIPCHK(hipStreamSynchronize(st));
    return r;
}

extern "C" kad_status kad_fetch_delta(const kad_sampler *s, double *h_lnInvDL, double *h_lnInvDU)
{
    if (!s || !h_lnInvDL || !h_lnInvDU) return fail(KAD_EINVAL, "null argument");
    if (!s->delta_ready) return fail(KAD_ESTATE, "delta allocation not done");
    HIPCHK(hipSetDevice(s->ctx->device));
    kad_status r = ensure_L(s);
    if (r == KAD_OK) r = copy_to_caller(s->g, s->LL, h_lnInvDL, s->ctx->stream);
    if (r == KAD_OK) r = copy_to_caller(s->g, s->LU, h_lnInvDU, s->ctx->stream);
    return r;
}

extern "C" kad_status kad_fetch_history(const kad_sampler *s, uint32_t epochs, double *h_hist)
{
    if (!s || !h_hist) return fail(KAD_EINVAL, "null argument");
    if ((int32_t)epochs > s->hist_cap) return fail(KAD_EINVAL, "more epochs than recorded");
    HIPCHK(hipSetDevice(s->ctx->device));
    const size_t rec = epoch_hist_bytes();
    std::vector<unsigned char> buf(rec * epochs);
    if (epochs) {
        HIPCHK(hipMemcpyAsync(buf.data(), s->hist, rec * epochs, hipMemcpyDeviceToHost, s->ctx->stream));
        HIPCHK(hipStreamSynchronize(s->ctx->stream));
    }
    for (uint32_t i = 0; i < epochs; ++i) {
        double v[3];
        int32_t ok;
        memcpy(v, buf.data() + rec * i, sizeof(v));
        memcpy(&ok, buf.data() + rec * i + sizeof(v), sizeof(ok));
        h_hist[4 * i + 0] = v[0];
        h_hist[4 * i + 1] = v[1];
        h_hist[4 * i + 2] = v[2];
        h_hist[4 * i + 3] = ok ? 1.0 : 0.0;
    }
    return KAD_OK;
}

extern "C" kad_status kad_fetch_calibration(const kad_sampler *s, uint32_t *h_cprime, uint64_t *h_tau0,
                                            double *h_C)
{
    if (!s) return fail(KAD_EINVAL, "null argument");
    if (!s->delta_ready || s->o.alloc_mode == KAD_ALLOC_EXPLICIT)
        return fail(KAD_ESTATE, "no calibration has run");
    HIPCHK(hipSetDevice(s->ctx->device));
    if (h_cprime) {
        kad_status r = copy_to_caller(s->g, s->cprime, h_cprime, s->ctx->stream);
        if (r != KAD_OK) return r;
    }
    if (h_tau0) *h_tau0 = s->res.tau0;
    if (h_C) *h_C = s->C;
    return KAD_OK;
}

extern "C" kad_status kad_count_samples(kad_sampler *s, uint64_t stream, uint64_t first, uint64_t count,
                                        uint32_t *h_c)
{
    if (!s || !h_c) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    const int32_t n = s->g->n;
    HIPCHK(hipMemsetAsync(s->scratch_counts, 0, 4ull * n, st));
    HIPCHK(hipMemsetAsync(s->stats, 0, sizeof(SampleStats), st));
    kad_status r = count_into(s, stream, first, count, s->scratch_counts, nullptr, nullptr, 0);
    if (r != KAD_OK) return r;
    r = check_stats_error(s);
    if (r != KAD_OK) return r;
    std::vector<uint32_t> tmp(n);
    r = copy_to_caller(s->g, s->scratch_counts, tmp.data(), st);
    if (r != KAD_OK) return r;
    for (int32_t v = 0; v < n; ++v) h_c[v] += tmp[v];
    return KAD_OK;
}

// The no-allocation variant of kad_count_samples.  The slots' visited state
// (records, frontier queues, meet lists, meet accumulators, stamps), the
// sample counter and the statistics are carved out of the device scratch;
// everything the launch uses is cleared by a kernel first, since the
// scratch keeps the last call's contents and a record left with a stamp
// the next call reuses would be taken for one of its own.
extern "C" kad_status kad_count_samples_noalloc(kad_ctx *ctx, const kad_graph *g, uint64_t seed,
                                                uint64_t stream, uint64_t first, uint64_t count,
                                                int32_t sigma_mode, uint32_t *d_c)
{
    if (!ctx || !g || !d_c) return fail(KAD_EINVAL, "null argument");
    if (sigma_mode != KAD_SIGMA_AUTO && sigma_mode != KAD_SIGMA_FP) return fail(KAD_EINVAL, "bad sigma_mode");
    if (first + count < first) return fail(KAD_EINVAL, "sample range wraps around");
    if (g->device != ctx->device) return fail(KAD_EINVAL, "graph and context are on different devices");
    if (count == 0) return KAD_OK;
    HIPCHK(hipSetDevice(ctx->device));
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[ctx->device];
    }
    if (!base) return fail(KAD_ESTATE, "device scratch not initialised for this device");
    const size_t n = (size_t)g->n;
    const int block = 256;
    const int32_t macc_cap = (int32_t)std::min<size_t>(n, (size_t)1 << 16);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t fixed = up(sizeof(SampleStats)) + up(sizeof(unsigned long long));
    // per slot: records, queue, meet list, meet accumulators, stamp (each
    // array 256-byte aligned per slot count below)
    const size_t per_slot = n * (sizeof(Rec) + 2 * sizeof(int32_t)) + 16 * (size_t)macc_cap + sizeof(uint32_t);
    size_t slots = NOALLOC_SCRATCH_BYTES > fixed + 5 * 256 ? (NOALLOC_SCRATCH_BYTES - fixed - 5 * 256) / per_slot : 0;
    if (slots < 1)
        return fail(KAD_EOVERFLOW, "graph too large for kad_count_samples_noalloc: one slot needs " +
                                       std::to_string(per_slot) + " bytes, the scratch holds " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES));
    slots = std::min<size_t>(slots, (size_t)ctx->cu_count * (size_t)sampler_blocks_per_cu(block, false));
    slots = std::min<size_t>(slots, count);
    unsigned char *p = base;
    auto take = [&](size_t bytes) { unsigned char *q = p; p += up(bytes); return q; };
    SampleStats *stats = (SampleStats *)take(sizeof(SampleStats));
    unsigned long long *work = (unsigned long long *)take(sizeof(unsigned long long));
    uint32_t *stamps = (uint32_t *)take(4 * slots);
    Rec *recs = (Rec *)take(sizeof(Rec) * n * slots);
    int32_t *queues = (int32_t *)take(4 * n * slots);
    int32_t *mbufs = (int32_t *)take(4 * n * slots);
    unsigned long long *macc = (unsigned long long *)take(16 * (size_t)macc_cap * slots);
    const size_t used = (size_t)(p - base);
    if (used > NOALLOC_SCRATCH_BYTES) return fail(KAD_EOVERFLOW, "scratch layout exceeds the scratch");
    hipStream_t st = ctx->stream;
    HIPCHK(launch_zero_words((uint32_t *)base, used / 4, st));
    SampleLaunch a;
    memset(&a, 0, sizeof(a));
    a.g = g->dev();
    a.seed = seed;
    a.stream = stream;
    a.first = first;
    a.count = count;
    a.sf[0] = a.sf[1] = d_c;
    a.recs = recs;
    a.queues = queues;
    a.mbufs = mbufs;
    a.macc = macc;
    a.macc_cap = macc_cap;
    a.stamps = stamps;
    a.work_ctr = work;
    a.stats = stats;
    a.sigma_fp = sigma_mode == KAD_SIGMA_FP;
    a.count_map = g->d_orig;
    HIPCHK(launch_sampler(a, (int)slots, block, st));
    SampleStats h;
    HIPCHK(hipMemcpyAsync(&h, stats, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h.error == 1) return fail(KAD_ENOTCONNECTED, "a sampled pair has no path: graph not connected");
    if (h.error != 0) return fail(KAD_EDEVICE, "internal error: a path choice found no candidate");
    return KAD_OK;
}

extern "C" kad_status kad_sample_paths(kad_sampler *s, uint64_t stream, uint64_t first, uint32_t count,
                                       int32_t max_len, int32_t *h_paths, int64_t *h_info)
{
    if (!s || !h_paths || !h_info || max_len < 2) return fail(KAD_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    const int32_t n = s->g->n;
    int32_t *dp = nullptr;
    int64_t *di = nullptr;
    HIPCHK(hipMallocAsync((void **)&dp, sizeof(int32_t) * (size_t)count * max_len + 4, st));
    HIPCHK(hipMallocAsync((void **)&di, sizeof(int64_t) * (size_t)count * KAD_INFO_WIDTH + 8, st));
    HIPCHK(hipMemsetAsync(dp, 0xFF, sizeof(int32_t) * (size_t)count * max_len + 4, st));
    HIPCHK(hipMemsetAsync(s->scratch_counts, 0, 4ull * n, st));
    HIPCHK(hipMemsetAsync(s->stats, 0, sizeof(SampleStats), st));
    kad_status r = count_into(s, stream, first, count, s->scratch_counts, dp, di, max_len);
    if (r == KAD_OK) r = check_stats_error(s);
    if (r == KAD_OK) {
        HIPCHK(hipMemcpyAsync(h_paths, dp, sizeof(int32_t) * (size_t)count * max_len, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_info, di, sizeof(int64_t) * (size_t)count * KAD_INFO_WIDTH,
                              hipMemcpyDeviceToHost, st));
    }
    (void)hipFreeAsync(dp, st);
    (void)hipFreeAsync(di, st);
    HIPCHK(hipStreamSynchronize(st));
    if (r == KAD_OK) {
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device));
        for (uint32_t i = 0; i < count; ++i) {
            for (int k : {8, 10, 11, 12, 13}) {
                int64_t &t = h_info[(size_t)i * KAD_INFO_WIDTH + k];
                t = khz > 0 ? (int64_t)((double)t * 1e6 / (double)khz) : -1;   // ticks -> ns
            }
        }
    }
    return r;
}

extern "C" kad_status kad_philox(kad_ctx *ctx, uint64_t seed, uint64_t stream, uint64_t first,
                                 uint32_t count, uint32_t nwords, uint64_t *h_out)
{
    if (!ctx || !h_out || count == 0 || nwords == 0) return fail(KAD_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    uint64_t *d = nullptr;
    const size_t bytes = sizeof(uint64_t) * (size_t)count * nwords;
    HIPCHK(hipMallocAsync((void **)&d, bytes, st));
    HIPCHK(launch_philox(seed, stream, first, count, nwords, d, st));
    HIPCHK(hipMemcpyAsync(h_out, d, bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipFreeAsync(d, st));
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

// ------------------------------------------------------------- learned prior

struct kad_mlp {
    kad_ctx *ctx;
    int device;
    float *params, *grad, *m, *v, *loss;
    float *scratch;
    size_t scratch_cap;
    int step;
};

extern "C" kad_status kad_features(kad_ctx *ctx, const kad_graph *g, float *d_out, float *h_out)
{
    if (!ctx || !g || (!d_out && !h_out)) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const size_t bytes = sizeof(float) * 3 * (size_t)g->n;
    float *t = nullptr, *d = d_out;
    HIPCHK(hipMallocAsync((void **)&t, bytes, st));
    if (!d) HIPCHK(hipMallocAsync((void **)&d, bytes, st));
    HIPCHK(launch_features(g->dev(), g->runs(), t, st));
    HIPCHK(launch_to_caller_f32x3(g->n, g->d_orig, t, d, st));
    HIPCHK(hipFreeAsync(t, st));
    if (!d_out) {
        HIPCHK(hipMemcpyAsync(h_out, d, bytes, hipMemcpyDeviceToHost, st));
        HIPCHK(hipFreeAsync(d, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

extern "C" kad_status kad_mlp_create(kad_ctx *ctx, const float *h_params, kad_mlp **out)
{
    if (!ctx || !h_params || !out) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    kad_mlp *m = new kad_mlp();
    m->ctx = ctx;
    m->device = ctx->device;
    if (hipMalloc((void **)&m->params, 4 * 4481) != hipSuccess || hipMalloc((void **)&m->grad, 4 * 4481) != hipSuccess ||
        hipMalloc((void **)&m->m, 4 * 4481) != hipSuccess || hipMalloc((void **)&m->v, 4 * 4481) != hipSuccess ||
        hipMalloc((void **)&m->loss, 16) != hipSuccess) {
        delete m;
        return fail(KAD_ENOMEM, "mlp allocation failed");
    }
    HIPCHK(hipMemcpy(m->params, h_params, 4 * 4481, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(m->m, 0, 4 * 4481));
    HIPCHK(hipMemset(m->v, 0, 4 * 4481));
    *out = m;
    return KAD_OK;
}

extern "C" void kad_mlp_free(kad_mlp *m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(m->params);
    (void)hipFree(m->grad);
    (void)hipFree(m->m);
    (void)hipFree(m->v);
    (void)hipFree(m->loss);
    if (m->scratch) (void)hipFree(m->scratch);
    delete m;
}

extern "C" kad_status kad_mlp_get_params(const kad_mlp *m, float *h_params)
{
    if (!m || !h_params) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(m->ctx->device));
    HIPCHK(hipMemcpyAsync(h_params, m->params, 4 * 4481, hipMemcpyDeviceToHost, m->ctx->stream));
    HIPCHK(hipStreamSynchronize(m->ctx->stream));
    return KAD_OK;
}

static kad_status mlp_scratch(kad_mlp *m, int64_t rows)
{
    const size_t need = mlp_scratch_floats(rows);
    if (need > m->scratch_cap) {
        if (m->scratch) (void)hipFree(m->scratch);
        m->scratch = nullptr;
        if (hipMalloc((void **)&m->scratch, need * sizeof(float)) != hipSuccess)
            return fail(KAD_ENOMEM, "mlp scratch allocation failed");
        m->scratch_cap = need;
    }
    return KAD_OK;
}

extern "C" kad_status kad_mlp_loss_grad(kad_mlp *m, const float *d_x, const float *d_y, int64_t rows,
                                        float *h_loss, float *h_grad)
{
    if (!m || !d_x || !d_y || rows <= 0) return fail(KAD_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(m->ctx->device));
    kad_status r = mlp_scratch(m, rows);
    if (r != KAD_OK) return r;
    hipStream_t st = m->ctx->stream;
    HIPCHK(launch_mlp_loss_grad(m->params, d_x, d_y, rows, m->grad, m->loss, m->scratch, st));
    if (h_grad) HIPCHK(hipMemcpyAsync(h_grad, m->grad, 4 * 4481, hipMemcpyDeviceToHost, st));
    if (h_loss) HIPCHK(hipMemcpyAsync(h_loss, m->loss, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

extern "C" kad_status kad_mlp_train_step(kad_mlp *m, const float *d_x, const float *d_y, int64_t rows,
                                         float lr, float *h_loss)
{
    if (!m || !d_x || !d_y || rows <= 0) return fail(KAD_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(m->ctx->device));
    kad_status r = mlp_scratch(m, rows);
    if (r != KAD_OK) return r;
    hipStream_t st = m->ctx->stream;
    HIPCHK(launch_mlp_loss_grad(m->params, d_x, d_y, rows, m->grad, m->loss, m->scratch, st));
    m->step += 1;
    HIPCHK(launch_adam(m->params, m->grad, m->m, m->v, 4481, m->step, lr, st));
    if (h_loss) {
        HIPCHK(hipMemcpyAsync(h_loss, m->loss, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return KAD_OK;
}

extern "C" kad_status kad_mlp_forward(kad_mlp *m, const float *d_x, int64_t rows, float *d_y, float *h_y)
{
    if (!m || !d_x || rows <= 0 || (!d_y && !h_y)) return fail(KAD_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    float *y = d_y;
    if (!y) HIPCHK(hipMallocAsync((void **)&y, sizeof(float) * (size_t)rows, st));
    HIPCHK(launch_mlp_forward(m->params, d_x, nullptr, rows, y, st));
    if (!d_y) {
        HIPCHK(hipMemcpyAsync(h_y, y, sizeof(float) * (size_t)rows, hipMemcpyDeviceToHost, st));
        HIPCHK(hipFreeAsync(y, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return KAD_OK;
}

// Training of the prior network, everything on the device: features and
// targets of every graph's vertices (rows in graph order, vertices in the
// caller's numbering), the standardisation vector, the initialisation,
// then epochs of Adam steps on batches drawn from a Philox stream.
extern "C" kad_status kad_mlp_train(kad_ctx *ctx, const kad_graph *const *graphs, const double *const *h_btilde,
                                    const double *h_omega, int32_t ngraphs, const kad_train_opts *o,
                                    float *h_params, float *h_norm, float *h_losses)
{
    if (!ctx || !graphs || !h_btilde || !h_omega || !o || !h_params || !h_norm)
        return fail(KAD_EINVAL, "null argument");
    if (ngraphs < 1 || o->epochs < 1 || o->batch < 1 || !(o->lr > 0.0f) || o->lr_halve_every < 0)
        return fail(KAD_EINVAL, "bad training options");
    int64_t rows = 0;
    for (int32_t i = 0; i < ngraphs; ++i) {
        if (!graphs[i] || !h_btilde[i] || !(h_omega[i] > 0.0)) return fail(KAD_EINVAL, "bad graph, b~ or omega");
        if (graphs[i]->device != ctx->device) return fail(KAD_EINVAL, "graph on another device");
        rows += graphs[i]->n;
    }
    if (rows * 3 >= (int64_t)1 << 31) return fail(KAD_EOVERFLOW, "too many training rows");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    float *X = nullptr, *Y = nullptr, *XB = nullptr, *YB = nullptr, *norm = nullptr, *feat = nullptr;
    double *bt = nullptr, *mom = nullptr, *acc = nullptr;
    kad_mlp *m = nullptr;
    kad_status r = KAD_OK;
    int32_t nmax = 0;
    for (int32_t i = 0; i < ngraphs; ++i) nmax = std::max(nmax, graphs[i]->n);
    const size_t B = (size_t)o->batch;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        void *ps[] = {X, Y, XB, YB, norm, feat, bt, mom, acc};
        for (void *q : ps)
            if (q) (void)hipFree(q);
        if (m) kad_mlp_free(m);
    };
    if (hipMalloc((void **)&X, 12ull * rows) != hipSuccess || hipMalloc((void **)&Y, 4ull * rows) != hipSuccess ||
        hipMalloc((void **)&XB, 12ull * B) != hipSuccess || hipMalloc((void **)&YB, 4ull * B) != hipSuccess ||
        hipMalloc((void **)&norm, 64) != hipSuccess || hipMalloc((void **)&feat, 12ull * nmax) != hipSuccess ||
        hipMalloc((void **)&bt, 8ull * nmax) != hipSuccess ||
        hipMalloc((void **)&mom, 8 * moments_scratch_doubles()) != hipSuccess ||
        hipMalloc((void **)&acc, 8ull * o->epochs) != hipSuccess) {
        cleanup();
        return fail(KAD_ENOMEM, "training buffers");
    }
#define TRAIN_CHK(expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            cleanup();                                                                   \
            return fail(KAD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                                \
    } while (0)
    int64_t off = 0;
    for (int32_t i = 0; i < ngraphs; ++i) {
        const kad_graph *g = graphs[i];
        TRAIN_CHK(launch_features(g->dev(), g->runs(), feat, st));
        TRAIN_CHK(launch_to_caller_f32x3(g->n, g->d_orig, feat, X + 3 * off, st));
        TRAIN_CHK(hipMemcpyAsync(bt, h_btilde[i], 8ull * g->n, hipMemcpyHostToDevice, st));
        TRAIN_CHK(launch_target(g->n, bt, h_omega[i], Y + off, st));
        TRAIN_CHK(hipStreamSynchronize(st));   // bt is refilled for the next graph
        off += g->n;
    }
    TRAIN_CHK(launch_feature_norm(X, rows, mom, norm, st));
    TRAIN_CHK(launch_normalize((int32_t)rows, X, norm, st));
    TRAIN_CHK(launch_zero_words((uint32_t *)acc, 2ull * o->epochs, st));
    {
        std::vector<float> zero(4481, 0.0f);
        r = kad_mlp_create(ctx, zero.data(), &m);
        if (r != KAD_OK) { cleanup(); return r; }
    }
    TRAIN_CHK(launch_mlp_init(o->seed, m->params, st));
    r = mlp_scratch(m, o->batch);
    if (r != KAD_OK) { cleanup(); return r; }
    const int64_t steps_per_epoch = (rows + o->batch - 1) / o->batch;
    uint64_t step = 0;
    for (int32_t e = 0; e < o->epochs; ++e) {
        const int halvings = o->lr_halve_every > 0 ? e / o->lr_halve_every : 0;
        const float lr = o->lr * powf(0.5f, (float)halvings);
        for (int64_t j = 0; j < steps_per_epoch; ++j, ++step) {
            TRAIN_CHK(launch_gather_batch(o->seed, step, o->batch, rows, X, Y, XB, YB, st));
            TRAIN_CHK(launch_mlp_loss_grad(m->params, XB, YB, o->batch, m->grad, m->loss, m->scratch, st));
            TRAIN_CHK(launch_adam(m->params, m->grad, m->m, m->v, 4481, (int)(step + 1), lr, st));
            TRAIN_CHK(launch_acc_loss(m->loss, acc, e, st));
        }
    }
    std::vector<double> lsum((size_t)o->epochs);
    TRAIN_CHK(hipMemcpyAsync(h_params, m->params, 4 * 4481, hipMemcpyDeviceToHost, st));
    TRAIN_CHK(hipMemcpyAsync(h_norm, norm, 4 * 6, hipMemcpyDeviceToHost, st));
    TRAIN_CHK(hipMemcpyAsync(lsum.data(), acc, 8ull * o->epochs, hipMemcpyDeviceToHost, st));
    TRAIN_CHK(hipStreamSynchronize(st));
#undef TRAIN_CHK
    if (h_losses)
        for (int32_t e = 0; e < o->epochs; ++e) h_losses[e] = (float)(lsum[(size_t)e] / (double)steps_per_epoch);
    cleanup();
    return KAD_OK;
}

// ----------------------------------------------------------- device memory

extern "C" kad_status kad_device_alloc(kad_ctx *ctx, size_t bytes, void **d_out)
{
    if (!ctx || !d_out) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    if (hipMalloc(d_out, std::max<size_t>(bytes, 16)) != hipSuccess) return fail(KAD_ENOMEM, "hipMalloc failed");
    return KAD_OK;
}

extern "C" kad_status kad_device_free(kad_ctx *ctx, void *d_ptr)
{
    if (!ctx) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipFree(d_ptr));
    return KAD_OK;
}

extern "C" kad_status kad_memcpy_h2d(kad_ctx *ctx, void *d_dst, const void *h_src, size_t bytes)
{
    if (!ctx || (bytes && (!d_dst || !h_src))) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMemcpyAsync(d_dst, h_src, bytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return KAD_OK;
}

extern "C" kad_status kad_memcpy_d2h(kad_ctx *ctx, void *h_dst, const void *d_src, size_t bytes)
{
    if (!ctx || (bytes && (!d_src || !h_dst))) return fail(KAD_EINVAL, "null argument");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMemcpyAsync(h_dst, d_src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return KAD_OK;
}
