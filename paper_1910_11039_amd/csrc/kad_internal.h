// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kadabra.h"

namespace kad {

constexpr int KAD_INFO_WIDTH = 14;

// Per-vertex, per-slot record of the bidirectional BFS (16 bytes).
//   key   = (stamp << 32) | state; a record belongs to the current sample of
//           its slot only when stamp equals the slot's current stamp, so a
//           slot never has to clear its records between samples.
//   state = side << 31 | meet << 30 | depth (depth < 2^30).
//   sig   = number of shortest paths from the side's root (uint64, or the
//           bits of an FP64 value in FP mode).
struct Rec {
    uint32_t state;
    uint32_t stamp;
    uint64_t sig;
};
static_assert(sizeof(Rec) == 16, "record layout");

constexpr uint32_t SIDE_BIT = 1u << 31;
constexpr uint32_t MEET_BIT = 1u << 30;
constexpr uint32_t DEPTH_MASK = MEET_BIT - 1;

// Per-sample statistics accumulated by the sampler kernel (device).
struct SampleStats {
    unsigned long long edges;          // adjacency entries read by expansions (final attempt)
    unsigned long long expanded;       // frontier vertices expanded
    unsigned long long visited;        // vertices newly discovered
    unsigned long long pred_edges;     // predecessor edges summed into sigma
    unsigned long long path_vertices;  // interior vertices counted
    unsigned long long fp_samples;     // samples in FP mode
    unsigned long long samples;        // samples finished
    unsigned long long edges_all;      // adjacency entries read including redone attempts and rescans
    unsigned long long deferred;       // samples a hashed-state launch handed to the dense fallback
    int error;                         // nonzero: a sample found the graph disconnected (1), a path
                                       // outgrew max_len (2), no predecessor (3), defer list full (4),
                                       // a reached vertex missing from the hashed state (5)
    int pad[3];
};

// The graph as the kernels see it.  Vertices are renumbered at upload in
// descending degree (ties: ascending caller id), so that the visited-state
// records of the hubs, which most adjacency probes reach, share a few cache
// lines, and a wave's probes along a sorted row fall on neighbouring
// records.  Two copies of the adjacency:
//  * ci:  every row in ascending internal id (set-valued work: expansion,
//         integer path counts, adjacency tests, BFS);
//  * cci: every row in the caller's order, ascending caller id (steps whose
//         result depends on the order: predecessor picks, FP sums).
// Every rule that orders vertices by id compares caller ids (orig), so
// results are those of the caller's numbering.
struct DevGraph {
    int32_t n;
    int64_t nnz;
    const int64_t *rp;
    const int32_t *ci;
    const int32_t *orig;    // internal id -> caller id
    const int32_t *newid;   // caller id -> internal id
    const int32_t *cci;
    const uint32_t *deg;    // degree of every vertex (4 bytes: stays in cache)
};

// Relabelled CSR from the caller's (device) CSR: row i of the output is
// row orig[i] of the input with every entry mapped through newid.
hipError_t launch_relabel_rows(int32_t n, const int64_t *rp_in, const int32_t *ci_in, const int32_t *orig,
                               const int32_t *newid, const int64_t *rp_out, int32_t *ci_out, hipStream_t st);
// Per-vertex arrays between the two numberings: to_caller writes
// out[orig[i]] = in[i]; from_caller writes out[i] = in[orig[i]].
// deg[v] = rp[v + 1] - rp[v].
hipError_t launch_degrees(int32_t n, const int64_t *rp, uint32_t *deg, hipStream_t st);
// Clears `words` 32-bit words with a kernel.
hipError_t launch_zero_words(uint32_t *p, size_t words, hipStream_t st);
// Sorts every row of a CSR (int32 entries) into ascending order.
hipError_t sort_rows(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *in, int32_t *out, hipStream_t st);
hipError_t launch_to_caller_u32(int32_t n, const int32_t *orig, const uint32_t *in, uint32_t *out, hipStream_t st);
hipError_t launch_to_caller_f64(int32_t n, const int32_t *orig, const double *in, double *out, hipStream_t st);
hipError_t launch_to_caller_f32x3(int32_t n, const int32_t *orig, const float *in, float *out, hipStream_t st);
hipError_t launch_from_caller_f64(int32_t n, const int32_t *orig, const double *in, double *out, hipStream_t st);

// Arguments of one sampler launch.
struct SampleLaunch {
    DevGraph g;
    uint64_t seed;
    uint64_t stream;
    uint64_t first;                 // first sample index of the launch
    uint64_t count;                 // samples in the launch (from host), or
    const unsigned long long *dev_epoch;  // if non-null: the launch's epoch k, read on the device: samples
    unsigned long long E, cap;            // [kE, min((k+1)E, cap)) into sf[0] (replayed graphs)
    const uint64_t *dev_seed;             // if non-null: the Philox seed, read on the device
    uint32_t *sf[2];                // counter buffers (state frames)
    Rec *recs;                      // slots * n records
    int32_t *queues;                // slots * n frontier entries
    int32_t *mbufs;                 // slots * n meet-set entries
    unsigned long long *macc;       // slots * 2 * macc_cap meet-weight accumulators
    int32_t macc_cap;
    uint32_t *stamps;               // slots stamps
    unsigned long long *work_ctr;   // next sample to take (device counter)
    SampleStats *stats;
    const int32_t *stop_flag;       // if non-null and set: skip the launch
    int sigma_fp;                   // 1: FP mode for every sample
    int32_t *paths;                 // optional per-sample paths [count][max_len]
    int64_t *info;                  // optional per-sample info  [count][KAD_INFO_WIDTH]
    int32_t max_len;
    uint32_t *hist;                 // optional: histogram of the counters' values 1..hist_top,
    uint32_t hist_top;              // kept as they are counted (the calibration's)
    const int32_t *count_map;       // optional: counter index of a vertex (internal id -> caller id)
    // Visited state.  Dense (sparse == 0): recs, queues and mbufs hold n
    // entries per slot.  Sparse: each holds 2^vcap_log2 entries per slot and
    // recs is a hashed table; a sample that would claim more than
    // claim_limit vertices is appended to defer_list (at most defer_cap,
    // counted in *defer_count; error 4 beyond that) and left for a dense
    // launch.  A dense launch with defer_in set takes its samples from that
    // list (defer_in_count entries) instead of [0, count).
    int sparse;
    uint32_t vcap_log2;
    int32_t claim_limit;
    uint32_t *defer_list;
    unsigned long long *defer_count;
    uint32_t defer_cap;
    const uint32_t *defer_in;
    const unsigned long long *defer_in_count;
};

hipError_t launch_sampler(const SampleLaunch &a, int slots, int block, hipStream_t st);
int sampler_max_block();
int sampler_blocks_per_cu(int block, bool sparse);   // resident workgroups per CU

// Epoch merge + stop rule (FP64).
struct EpochState {
    unsigned long long tau;        // samples merged so far
    unsigned long long epoch;      // epochs merged so far
    int32_t stopped;               // 1 once the stop rule holds or tau hit the cap
    int32_t reason;                // KAD_STOP_*
    double max_f, max_g, min_margin;
    unsigned long long blocks_done;
    int32_t all_ok;                // reduction scratch for the epoch in flight
    int32_t pad;
    unsigned long long max_f_bits, max_g_bits, min_margin_bits;
    unsigned long long range[3];   // {first, count, sf_index} of the next epoch
};

// Mirror of the epoch verdict in pinned host memory, written by the merge
// kernel so the host can poll it without a device-to-host copy.
struct HostStatus {
    int32_t stopped, reason;
    unsigned long long epoch, tau;
};

hipError_t launch_merge_stop_impl(const DevGraph &g, uint32_t *c, uint32_t *sf0, uint32_t *sf1,
                                  const double *LL, const double *LU, double omega, double eps,
                                  unsigned long long cap, unsigned long long E, EpochState *es,
                                  unsigned long long *work_ctr, void *hist, int32_t hist_cap,
                                  HostStatus *hs, hipStream_t st, unsigned long long *pool_epoch = nullptr,
                                  int pools = 0, unsigned long long *defer_ctr = nullptr,
                                  const uint32_t *lcnt = nullptr, const double *ltab = nullptr);
size_t epoch_hist_bytes();   // per-epoch record: max_f, max_g, min_margin (f64), ok (i32), pad
size_t alloc_partials(int32_t n);
hipError_t launch_fg(int32_t n, const uint32_t *c, double tau, const double *LL, const double *LU,
                     double omega, double *f, double *g, hipStream_t st);
hipError_t launch_btilde(int32_t n, const uint32_t *c, double tau, double *b, hipStream_t st);
hipError_t launch_philox(uint64_t seed, uint64_t stream, uint64_t first, uint32_t count,
                         uint32_t nwords, uint64_t *out, hipStream_t st);

// Delta allocation from a prior (calibration counts or learned prior).
// prior(v) = counts[v] / tau0 when counts != null, else dense_prior[v].
struct AllocArgs {
    int32_t n;
    const uint32_t *counts;
    double tau0;
    const double *dense_prior;
    double delta, beta;
    double *lo_hi;       // device: {lo, hi, done}
    double *partials;    // device scratch, one per block
    double *LL, *LU;     // out
    uint32_t *hist;      // optional: histogram of the counts already built (bins 1..tau0)
    double *ltab;        // optional: room for tau0 + 1 doubles (L by count value)
    int lazy;            // with ltab: fill only the table (LL is built later by run_alloc_L)
};
hipError_t run_alloc(const AllocArgs &a, hipStream_t st, double *C_host);
// LL (= LU) from the count table that a lazy run_alloc filled.
hipError_t run_alloc_L(const AllocArgs &a, double C, hipStream_t st);
// Sum over v of delta_L(v) + delta_U(v) = e^-LL + e^-LU on the device
// (compensated per thread, pairwise across threads), and whether every L is
// finite and positive.
hipError_t alloc_budget(int32_t n, const double *LL, const double *LU, hipStream_t st, double *sum_out,
                        bool *finite_out);

// Vertex-diameter bracket by BFS sweeps on the device.
// cache (optional): BFS arrays kept between calls on the same graph.
struct BfsCache;
BfsCache *bfs_cache_create();
void bfs_cache_free(BfsCache *c, hipStream_t st);
hipError_t device_vd_bracket(const DevGraph &g, hipStream_t st, int64_t *vd_lo, int64_t *vd_hi,
                             BfsCache *cache = nullptr);
// Exact vertex diameter (eccentricity-bound refinement); with omega_only it
// stops once both ends of [vd_lo, vd_hi] give the same omega; after
// max_bfs BFS runs it stops with the bracket it has.  witness: a vertex
// (caller id) whose eccentricity is vd_lo - 1.
hipError_t device_exact_vd(const DevGraph &g, hipStream_t st, bool omega_only, double eps, double delta,
                           int64_t max_bfs, int64_t *vd_lo, int64_t *vd_hi, int32_t *witness, int64_t *bfs_runs);

// Learned prior.
// Runs of equal degree in the internal numbering: vertices are numbered by
// descending degree, so run k holds the vertices start[k] .. start[k+1]-1,
// all of degree deg[k], and deg[] descends.  A graph has at most a few
// thousand distinct degrees, so the feature pass finds a neighbour's degree
// by a search in a table held in LDS instead of a gather.
struct DegreeRuns {
    int32_t count;            // number of runs (distinct degrees)
    const int32_t *start;     // device, count + 1 entries, start[count] = n
    const uint32_t *deg;      // device, count entries
    const int32_t *h_start;   // host copy of start
};
hipError_t launch_features(const DevGraph &g, const DegreeRuns &runs, float *out, hipStream_t st);
size_t features_workspace_bytes(const DevGraph &g);
hipError_t launch_features_ws(const DevGraph &g, const DegreeRuns &runs, float *out, void *ws, hipStream_t st);
hipError_t launch_normalize(int32_t n, float *x, const float *norm, hipStream_t st);
// y = MLP(x) over rows of 3 features; with norm (mean[3], std[3]) the
// features are standardised on load.
hipError_t launch_mlp_forward(const float *params, const float *x, const float *norm, int64_t rows, float *y,
                              hipStream_t st);
hipError_t launch_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t rows,
                                float *grad, float *loss, float *scratch, hipStream_t st);
hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int count, int step,
                       float lr, hipStream_t st);
hipError_t launch_prior_from_mlp(int32_t n, const float *yhat, double omega, double *prior,
                                 hipStream_t st);
size_t mlp_scratch_floats(int64_t rows);
// Training: target ln(b~ + 1/omega); feature standardisation vector [mean,
// std] (FP64 sums, scratch of moments_scratch_doubles()); Philox-seeded
// initialisation; the rows of one Adam step; the per-epoch loss sum.
hipError_t launch_target(int32_t n, const double *btilde, double omega, float *y, hipStream_t st);
size_t moments_scratch_doubles();
hipError_t launch_feature_norm(const float *x, int64_t rows, double *scratch, float *norm, hipStream_t st);
hipError_t launch_mlp_init(uint64_t seed, float *params, hipStream_t st);
hipError_t launch_gather_batch(uint64_t seed, uint64_t step, int32_t batch, int64_t rows, const float *x,
                               const float *y, float *xb, float *yb, hipStream_t st);
hipError_t launch_acc_loss(const float *loss, double *acc, int e, hipStream_t st);

}  // namespace kad
