/*
 * kadabra.h -- C-ABI of the MI355X (gfx950) KADABRA sampling library.
 *
 * The library approximates betweenness centrality by adaptive sampling, the
 * method whose parallelisation is the subject of van der Grinten &
 * Meyerhenke, "Scaling Betweenness Approximation to Billions of Edges by
 * MPI-based Adaptive Sampling" (IPDPS 2020):
 *
 *   b(x) = 1/(n(n-1)) * sum over ordered pairs s != t of sigma_st(x)/sigma_st
 *   (Sec. I); a sample draws s != t, samples one shortest s-t path
 *   uniformly with a bidirectional BFS and adds one to c~(x) for the
 *   vertices on it; b~ = c~ / tau (Sec. III-A); sampling stops once the
 *   per-vertex bounds f and g are below eps for every vertex, checked once
 *   per epoch on a consistent snapshot of the counters (Sec. III-A, III-B,
 *   Alg. 2), or when tau reaches omega.
 *
 * Conventions for every entry point:
 *   - Status codes only (kad_status); nothing is thrown across the ABI.
 *     On failure a message is available from kad_last_error() (a
 *     thread-local string owned by the library, valid until the next call
 *     on the same thread).
 *   - Pointer arguments named h_* are host memory owned by the caller; the
 *     library copies what it needs before returning.  Pointers named d_*
 *     are device memory on the context's device, owned by the caller.
 *   - Outputs are written only when the call returns KAD_OK.
 *   - Handles are owned by the library and released by the matching
 *     *_free / kad_destroy.  Free graphs, samplers and MLPs before the
 *     context they were made with.  Calls on one sampler are not
 *     thread-safe; different samplers may be used from different threads.
 *   - Graphs: undirected, unweighted (Sec. III), CSR with row_ptr int64[n+1]
 *     and col_idx int32[nnz]; each row sorted ascending, no self loops, no
 *     duplicate edges, symmetric, connected.  Vertex ids are 0..n-1.
 *   - Work runs on the context's stream (the HIP stream given to
 *     kad_create, or one the context creates) and, for samplers, on three
 *     more streams that the context creates and owns: slot pools 1..3, the
 *     third also carrying the learned prior's network, which
 *     kad_sampler_reset leaves running and kad_run_to_stop waits for.
 *     Kernels are built for gfx950 only.
 */
#ifndef KADABRA_H
#define KADABRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KAD_OK = 0,
    KAD_EINVAL = -1,          /* bad argument or malformed graph                  */
    KAD_ENOMEM = -2,          /* device or host allocation failed                 */
    KAD_EDEVICE = -3,         /* a HIP call failed                                */
    KAD_ENOTCONNECTED = -4,   /* graph not connected (a sample found no path)     */
    KAD_ESTATE = -5,          /* call not valid in the sampler's current state     */
    KAD_EOVERFLOW = -6        /* a size exceeds what the kernels support          */
} kad_status;

typedef struct kad_ctx kad_ctx;
typedef struct kad_graph kad_graph;
typedef struct kad_sampler kad_sampler;

/* Random-number streams: the Philox key is (seed, stream).  Stream 5 is
 * used by the autotuner's trial samples, whose counts are discarded. */
enum { KAD_STREAM_ADS = 0, KAD_STREAM_CALIB = 1, KAD_STREAM_TUNE = 5 };

/* Allocation of the per-vertex failure probabilities delta_L, delta_U. */
enum {
    KAD_ALLOC_PLAIN = 0,      /* calibration samples, Sec. III-A phase 2          */
    KAD_ALLOC_EXPLICIT = 1,   /* caller passes the arrays (kad_set_delta)         */
    KAD_ALLOC_LEARNED = 2     /* prior from the MLP (kad_set_mlp_weights)         */
};

/* Path-count arithmetic. AUTO: uint64 with exact overflow detection, the
 * whole sample redone in FP64 (with per-layer 2^-400 rescaling) on overflow.
 * FP: always FP64. */
enum { KAD_SIGMA_AUTO = 0, KAD_SIGMA_FP = 1 };

enum { KAD_STOP_NONE = 0, KAD_STOP_COND = 1, KAD_STOP_OMEGA = 2 };

/* Per-sample visited state of the sampler's workgroups (kad_opts). */
enum { KAD_VISITED_AUTO = 0, KAD_VISITED_DENSE = 1, KAD_VISITED_HASHED = 2 };

enum { KAD_GRAPH_VALIDATE = 1u };

/* kad_create: bind a context to HIP device `device` and stream
 * `hip_stream` (a hipStream_t, borrowed, not owned; a torch.cuda stream
 * handle works; NULL: the context creates a stream of its own).  The
 * context also creates the three streams of the samplers' slot pools 1..3
 * right after its own, so that HIP, which deals its hardware queues (four
 * by default) to streams in creation order, gives every pool a queue;
 * samplers of one context share them.  kad_destroy releases them. */
kad_status kad_create(int device, void *hip_stream, kad_ctx **out);
void kad_destroy(kad_ctx *ctx);
const char *kad_last_error(void);

/* kad_graph_upload: copy a CSR graph (Sec. III: undirected, unweighted)
 * from host memory into HBM.  n >= 2, nnz = h_row_ptr[n] < 2^31.  With
 * flags & KAD_GRAPH_VALIDATE the CSR is checked on the host (sorted rows,
 * no loops or duplicates, symmetric; EINVAL) and for connectivity
 * (ENOTCONNECTED). */
kad_status kad_graph_upload(kad_ctx *ctx, int32_t n, int64_t nnz, const int64_t *h_row_ptr,
                            const int32_t *h_col_idx, uint32_t flags, kad_graph **out);
void kad_graph_free(kad_graph *g);

/* Sampler options.  Zero-initialise and set what is needed. */
typedef struct {
    uint64_t seed;                /* Philox seed                                  */
    double epsilon;               /* additive error bound, Sec. I                 */
    double delta;                 /* failure probability, Sec. I                  */
    uint32_t epoch_size;          /* samples per epoch; 0 = autotune: two rounds  */
                                  /* of the slot wave when a sample takes a slot  */
                                  /* over 10 ms at the trial's rate, else sixteen */
                                  /* rounds but at most omega / 16; rounded up to */
                                  /* a multiple of 256, within [256, 16384]       */
    int32_t alloc_mode;           /* KAD_ALLOC_*                                  */
    double omega_override;        /* > 0: use this omega instead of computing it  */
    int32_t sigma_mode;           /* KAD_SIGMA_*                                  */
    int32_t slots;                /* concurrent samples (workgroups); 0 = auto     */
    uint64_t visited_budget_bytes;/* cap on per-slot visited state; 0 = auto      */
    int32_t epochs_in_flight;     /* epochs queued ahead of the stop check; 0=auto */
    int32_t use_graphs;           /* 1: replay epochs from a captured hipGraph    */
    int32_t block_size;           /* threads per sampling workgroup (64, 128,     */
                                  /* 256, 512, 1024); 0 = autotune over 256, 512, */
                                  /* 1024 by a timed trial at kad_sampler_init    */
    int32_t timing;               /* 1: time every sampler launch with HIP events */
    int32_t pools;                /* slot pools = sampler launches that may       */
                                  /* overlap (1..4); 0 = as many as memory allows */
    int32_t exact_diameter;       /* 1: omega from the bracket refined as in      */
                                  /* kad_exact_vd until its ends give one omega   */
                                  /* (at most 64 BFS runs, then its upper end);   */
                                  /* 0: from the three-sweep bracket              */
    int32_t visited_mode;         /* per-sample visited state: 1 dense (a record  */
                                  /* per vertex in every slot), 2 hashed (a table */
                                  /* of 2^visited_log2 buckets per slot; samples  */
                                  /* that would fill it over 3/4 are finished on  */
                                  /* a dense slot per pool); 0 = auto: hashed     */
                                  /* when the dense state holds fewer than 1.25   */
                                  /* full waves of 1024-thread slots, the table   */
                                  /* is at most 1/8 of a dense slot and the       */
                                  /* bracket's vertex diameter is at most 32;     */
                                  /* else dense.  Hashed with block_size 0 uses   */
                                  /* 1024 threads                                 */
    int32_t visited_log2;         /* hashed table size; 0 = the power of two at   */
                                  /* or above n / 32 within [2^16, 2^22];         */
                                  /* else within [10, 26]                         */
} kad_opts;

typedef struct {
    uint64_t tau;                 /* adaptive samples at the stop                 */
    uint64_t tau0;                /* calibration samples (plain allocation)        */
    uint32_t epochs;              /* epochs run, the stop epoch included          */
    int32_t stop_reason;          /* KAD_STOP_*                                   */
    double omega;                 /* maximum number of samples used               */
    int64_t vd_lo, vd_hi;         /* vertex-diameter bracket behind omega         */
    double t_omega_ms, t_alloc_ms, t_ads_ms, t_total_ms;   /* phase wall times   */
    double t_sample_kernel_ms;    /* summed sampler-kernel time (HIP events)      */
    uint32_t sample_launches;     /* sampler-kernel launches behind that sum      */
    int64_t edges_scanned;        /* adjacency entries read by BFS expansions     */
    int64_t vertices_expanded;    /* frontier vertices expanded                   */
    int64_t vertices_visited;     /* vertices newly reached by the BFS            */
    int64_t pred_edges;           /* predecessor edges summed into sigma          */
    int64_t path_vertices;        /* interior vertices counted                    */
    int64_t fp_samples;           /* samples that used FP64 path counts           */
    double max_f, max_g;          /* at the stop epoch                            */
    double min_margin;            /* min over vertices of |eps - max(f, g)|       */
    uint32_t epoch_size;          /* epoch size actually used                     */
    int32_t slots;                /* concurrent samples actually used             */
    int64_t samples_run;          /* samples the kernels finished, speculative    */
                                  /* ones after the stop epoch included           */
    int32_t block_size;           /* workgroup size used by the sampler           */
    int32_t pools;                /* slot pools (epochs overlapped across them)   */
    int32_t visited_mode;         /* 1 dense, 2 hashed                            */
    int32_t visited_log2;         /* hashed table size used (0 when dense)        */
    int64_t deferred;             /* samples the hashed launches handed to the    */
                                  /* dense fallback                               */
} kad_result;

/* kad_sampler_init: allocate the sampler state for graph g and options o.
 * Computes omega (Sec. III-A phase 1: from a vertex-diameter bracket
 * obtained by BFS on the device, unless omega_override > 0).  The delta
 * allocation happens in kad_run_to_stop (PLAIN, LEARNED) or through
 * kad_set_delta (EXPLICIT). */
kad_status kad_sampler_init(kad_ctx *ctx, const kad_graph *g, const kad_opts *o,
                            kad_sampler **out);
void kad_sampler_free(kad_sampler *s);

/* kad_sampler_reset: start a new run of the same sampler with a new seed:
 * recomputes omega (phase 1, unless omega_override was given), clears the
 * counters, the epochs and the statistics, and drops a PLAIN or LEARNED
 * allocation (EXPLICIT arrays are kept).  No device memory is allocated. */
kad_status kad_sampler_reset(kad_sampler *s, uint64_t seed);

/* kad_set_delta: EXPLICIT allocation, h_delta_L/U float64[n] in (0, 1);
 * the sum over vertices of delta_L + delta_U must stay below delta / 2
 * (the other half of delta is spent on omega); checked, EINVAL otherwise.
 * Any such split is a valid allocation (Sec. III-A, footnote on delta_L,
 * delta_U).  The stop rule's L = ln(1/delta) is computed here, once per
 * vertex, on the host in FP64 with the C library's log. */
kad_status kad_set_delta(kad_sampler *s, const double *h_delta_L, const double *h_delta_U);

/* kad_set_mlp_weights: LEARNED allocation; h_params float32[4481] in the
 * layout W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3 (row-major,
 * out x in), h_norm float32[6] = feature means then standard deviations. */
kad_status kad_set_mlp_weights(kad_sampler *s, const float *h_params, const float *h_norm);

/* kad_step_epoch: run one epoch (samples [kE, min((k+1)E, ceil(omega)))),
 * merge it into c~ and evaluate the stop rule.  *stopped = 1 once the rule
 * holds or tau reached ceil(omega).  Allocates delta first if needed. */
kad_status kad_step_epoch(kad_sampler *s, int *stopped);

/* kad_run_to_stop: omega (if not yet known), delta allocation, then epochs
 * until the stop rule holds (Sec. III-A phase 3 on one GPU; the epoch
 * boundary is the consistent snapshot of Sec. III-B). */
kad_status kad_run_to_stop(kad_sampler *s, kad_result *out);

/* Results after a stop (or after any kad_step_epoch). */
kad_status kad_fetch_counts(const kad_sampler *s, uint32_t *h_c, uint64_t *h_tau);
kad_status kad_fetch_btilde(const kad_sampler *s, double *h_b);          /* c~ / tau, FP64 */
kad_status kad_fetch_fg(const kad_sampler *s, double *h_f, double *h_g); /* at current tau */
kad_status kad_fetch_delta(const kad_sampler *s, double *h_lnInvDL, double *h_lnInvDU);
kad_status kad_fetch_result(const kad_sampler *s, kad_result *out);

/* kad_fetch_history: for epochs [0, epochs) of the run so far, the largest
 * f, the largest g, the smallest |eps - max(f, g)| and the rule's verdict
 * (1.0 = all vertices below eps): h_hist float64[epochs][4]. */
kad_status kad_fetch_history(const kad_sampler *s, uint32_t epochs, double *h_hist);

/* kad_fetch_calibration: plain allocation's calibration counters c'
 * (uint32[n]), sample count tau0 and bisection constant C. */
kad_status kad_fetch_calibration(const kad_sampler *s, uint32_t *h_cprime, uint64_t *h_tau0,
                                 double *h_C);

/* kad_count_samples: add the counters of samples [first, first+count) of
 * Philox stream `stream` (no stop rule) into h_c (uint32[n], accumulated on
 * the host side: the library adds its device counts to what h_c holds). */
kad_status kad_count_samples(kad_sampler *s, uint64_t stream, uint64_t first, uint64_t count,
                             uint32_t *h_c);

/* kad_count_samples_noalloc: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Adds the counters of samples [first, first+count) of
 * Philox stream (seed, stream) into d_c (uint32[n], device memory owned by
 * the caller, indexed by the caller's vertex ids); sigma_mode is
 * KAD_SIGMA_AUTO or KAD_SIGMA_FP.  The same counts as kad_count_samples.
 * Calls no allocator: the samplers' visited state lives in a static device
 * scratch of KAD_NOALLOC_SCRATCH_BYTES per GPU (held until the process
 * ends), cleared by a kernel at the start of every call.  A graph whose one
 * sample slot (24 n + 16 min(n, 65536) + 4 bytes) does not fit returns
 * KAD_EOVERFLOW.  Every call on one GPU shares that GPU's scratch: calls
 * that overlap on one GPU (from several threads or streams) race.
 * Synchronous on the context's stream. */
#define KAD_NOALLOC_SCRATCH_BYTES (64ull << 20)
kad_status kad_count_samples_noalloc(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint64_t stream,
                                     uint64_t first, uint64_t count, int32_t sigma_mode, uint32_t *d_c);

/* kad_sample_paths: run samples [first, first+count) of `stream` and
 * return each path s..t: h_paths int32[count][max_len] (entries past d are
 * -1), h_info int64[count][14] = {s, t, d, w, fp_mode, meet_size, steps,
 * edges, duration_ns, attempts, expand_ns, meet_weights_ns, choose_ns,
 * walk_ns} (durations: wall time inside the sample's workgroup, in total
 * and per phase of the last attempt; attempts: 2 when integer path counts
 * overflowed and the sample was redone in FP64).  A path longer than max_len-1 edges returns KAD_EOVERFLOW. */
kad_status kad_sample_paths(kad_sampler *s, uint64_t stream, uint64_t first, uint32_t count,
                            int32_t max_len, int32_t *h_paths, int64_t *h_info);

/* kad_philox: words [0, nwords) of samples [first, first+count) of Philox
 * stream (seed, stream), computed on the device: h_out uint64[count][nwords]. */
kad_status kad_philox(kad_ctx *ctx, uint64_t seed, uint64_t stream, uint64_t first,
                      uint32_t count, uint32_t nwords, uint64_t *h_out);

/* kad_vd_bracket: device BFS sweeps bounding the vertex diameter of g
 * (Sec. III-A phase 1 needs it for omega): vd_lo <= VD <= vd_hi. */
kad_status kad_vd_bracket(kad_ctx *ctx, const kad_graph *g, int64_t *vd_lo, int64_t *vd_hi);

/* kad_exact_vd: the exact vertex diameter of g (the diameter phase of Sec.
 * III-A, computed exactly as in Sec. IV-F with a BFS-based exact algorithm):
 * bound refinement on the device -- every BFS from x bounds each vertex's
 * eccentricity by max(d, e - d) <= ecc <= e + d; sources are the bracket's
 * three sweeps, then alternately the vertex of smallest lower bound and the
 * vertex of largest upper bound, until the largest eccentricity found
 * equals the largest upper bound.  *h_vd = VD (edges of a longest shortest
 * path + 1); *h_witness (optional) = a vertex, caller id, of eccentricity
 * VD - 1; *h_bfs (optional) = BFS runs the search took.  KAD_EOVERFLOW when
 * 2000 BFS runs do not settle it (graphs with very many vertices of
 * near-diametral eccentricity, such as random hyperbolic graphs). */
kad_status kad_exact_vd(kad_ctx *ctx, const kad_graph *g, int64_t *h_vd, int32_t *h_witness, int64_t *h_bfs);

/* kad_omega: omega = 0.5/eps^2 * (floor(log2(VD-2)) + 1 + ln(2/delta)) for
 * the bracket [vd_lo, vd_hi] (the upper end unless both ends agree). */
double kad_omega(int64_t vd_lo, int64_t vd_hi, double eps, double delta);

/* ---- device memory plumbing (for callers without another HIP runtime):
 * kad_device_alloc returns `bytes` of device memory on the context's device
 * in *d_out (caller-owned, release with kad_device_free); the copies are
 * synchronous on the context's stream. */
kad_status kad_device_alloc(kad_ctx *ctx, size_t bytes, void **d_out);
kad_status kad_device_free(kad_ctx *ctx, void *d_ptr);
kad_status kad_memcpy_h2d(kad_ctx *ctx, void *d_dst, const void *h_src, size_t bytes);
kad_status kad_memcpy_d2h(kad_ctx *ctx, void *h_dst, const void *d_src, size_t bytes);

/* ---- learned prior (not in the paper: a learned replacement for the
 * calibration phase; delta_L/delta_U remain a valid split either way) ---- */

/* kad_features: per-vertex features [ln(1+deg v), mean over neighbours of
 * ln(1+deg u), ln(1+sum over neighbours of deg u)] into d_out float32[n][3]
 * (device memory, caller-owned), or h_out if d_out is NULL. */
kad_status kad_features(kad_ctx *ctx, const kad_graph *g, float *d_out, float *h_out);

typedef struct kad_mlp kad_mlp;

/* kad_mlp_create: a 3-64-64-1 ReLU MLP in FP32 on the device with Adam
 * state.  h_params float32[4481] (layout as kad_set_mlp_weights). */
kad_status kad_mlp_create(kad_ctx *ctx, const float *h_params, kad_mlp **out);
void kad_mlp_free(kad_mlp *m);
kad_status kad_mlp_get_params(const kad_mlp *m, float *h_params);

/* kad_mlp_loss_grad: mean squared error over rows of d_x float32[rows][3]
 * against d_y float32[rows], and its gradient (float32[4481], host). */
kad_status kad_mlp_loss_grad(kad_mlp *m, const float *d_x, const float *d_y, int64_t rows,
                             float *h_loss, float *h_grad);

/* kad_mlp_train_step: forward, backward and one Adam step (lr, beta1 =
 * 0.9, beta2 = 0.999, eps = 1e-8) on a batch; *h_loss = batch loss. */
kad_status kad_mlp_train_step(kad_mlp *m, const float *d_x, const float *d_y, int64_t rows,
                              float lr, float *h_loss);

/* kad_mlp_forward: predictions for d_x float32[rows][3] into d_y (device)
 * or h_y (host) when d_y is NULL. */
kad_status kad_mlp_forward(kad_mlp *m, const float *d_x, int64_t rows, float *d_y, float *h_y);

/* Training options of kad_mlp_train. */
typedef struct {
    int32_t epochs;           /* passes; each is ceil(rows / batch) Adam steps   */
    int32_t batch;            /* rows per step                                    */
    float lr;                 /* Adam step size of the first epochs               */
    int32_t lr_halve_every;   /* the step size halves every this many epochs      */
                              /* (0: constant)                                    */
    uint64_t seed;            /* Philox seed (stream 2) of the initialisation and */
                              /* of the batches                                   */
} kad_train_opts;

/* kad_mlp_train: trains the prior network on the vertices of ngraphs graphs.
 * The rows are the graphs' vertices, graph after graph, each graph's in its
 * caller numbering.  Row v of graph i: the features of kad_features, and
 * the target ln(b~ + 1/omega) with b~ = h_btilde[i][v] (float64[n_i], the
 * estimate a plain run gave) and omega = h_omega[i].  The features are
 * standardised with their mean and population standard deviation over all
 * rows (FP64 sums; a zero deviation is taken as 1).  Initialisation: weight
 * i (in the layout of kad_set_mlp_weights) is (2u - 1) sqrt(6 / fan_in),
 * u = unit53(draw 0 of Philox sample i of stream 2); biases 0.  Adam step j
 * (beta1 0.9, beta2 0.999, eps 1e-8; mean squared error) takes batch rows
 * floor(u_b rows / 2^64), u_b = draw b of Philox sample 2^32 + j (uniform
 * rows, with replacement).  Everything runs on the device.
 * Out: h_params float32[4481], h_norm float32[6] (means, then standard
 * deviations: the h_norm of kad_set_mlp_weights) and, unless NULL,
 * h_losses float32[epochs] (each epoch's mean batch loss). */
kad_status kad_mlp_train(kad_ctx *ctx, const kad_graph *const *graphs, const double *const *h_btilde,
                         const double *h_omega, int32_t ngraphs, const kad_train_opts *o, float *h_params,
                         float *h_norm, float *h_losses);

#ifdef __cplusplus
}
#endif
#endif
