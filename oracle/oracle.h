/*
 * Declarations of the CPU oracle (test infrastructure only; see oracle.c).
 * This header belongs to the oracle alone and is not shared with the HIP
 * library.
 */
#ifndef KAD_ORACLE_H
#define KAD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EDISCONNECTED = -4 };
enum { ORC_SIGMA_AUTO = 0, ORC_SIGMA_FP = 1 };
enum { ORC_STOP_NONE = 0, ORC_STOP_COND = 1, ORC_STOP_OMEGA = 2, ORC_STOP_PAUSED = 3 };
enum { ORC_STREAM_ADS = 0, ORC_STREAM_CALIB = 1 };
#define ORC_MLP_PARAMS 4481

typedef struct {
    int32_t n;
    const int64_t *row_ptr;   /* n + 1 */
    const int32_t *col_idx;   /* row_ptr[n], ascending per row */
} orc_graph;

typedef struct orc_ws orc_ws;

typedef struct {
    int32_t s, t, d, w;       /* pair, distance, chosen meet vertex          */
    int32_t side;             /* side that expanded last (0 = s, 1 = t)     */
    int32_t steps;            /* number of layer expansions                 */
    int32_t meet_size;
    int32_t fp_mode;          /* 1 if sigma was taken in FP mode            */
    int64_t edges;            /* adjacency entries scanned by expansions    */
    uint64_t draws;           /* random words consumed                      */
    uint64_t sigma_st_int;    /* integer mode: number of shortest s-t paths */
    double sigma_st;          /* FP mode: scaled count; sigma = this * 2^exp */
    int32_t sigma_exp;
    int32_t visited;          /* vertices reached by either side            */
} orc_sample_info;

typedef struct {
    uint64_t seed, stream;
    double eps, omega;
    uint64_t epoch;           /* samples per epoch                          */
    int sigma_mode;
    int32_t start_epoch;      /* resume: counters hold epochs [0, start)    */
    int32_t stop_after_epochs;/* > 0: pause after this many epochs          */
} orc_run_opts;

typedef struct {
    uint64_t tau;
    int32_t epochs;
    int32_t reason;
    int64_t edges;
} orc_run_result;

typedef struct {
    double max_f, max_g, min_abs_margin;
} orc_check_info;

void orc_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4]);
uint64_t orc_draw(uint64_t seed, uint64_t stream, uint64_t sample, uint64_t j);
void orc_pair(uint64_t seed, uint64_t stream, uint64_t sample, int32_t n, int32_t *s, int32_t *t);

orc_ws *orc_ws_create(int32_t n);
void orc_ws_free(orc_ws *w);
int orc_sample(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream, uint64_t sample,
               int sigma_mode, orc_sample_info *info);
int orc_sample_fixed(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream, uint64_t sample,
                     int sigma_mode, int32_t s, int32_t t, int32_t *path_out, orc_sample_info *info);
int orc_sample_path(const orc_graph *g, orc_ws *w, uint64_t seed, uint64_t stream, uint64_t sample,
                    int sigma_mode, int32_t *path_out, orc_sample_info *info);

double orc_f(double bt, double L, double omega, double tau);
double orc_g(double bt, double L, double omega, double tau);
double orc_omega(int64_t vd, double eps, double delta);
double orc_omega_bracket(int64_t vd_lo, int64_t vd_hi, double eps, double delta);
void orc_vd_bracket(const orc_graph *g, int64_t *vd_lo, int64_t *vd_hi);
int64_t orc_exact_vd(const orc_graph *g);
int32_t orc_eccentricity(const orc_graph *g, int32_t v);

int orc_check(int32_t n, const uint32_t *c, uint64_t tau, double omega, double eps,
              const double *LL, const double *LU, orc_check_info *ci);
int orc_run(const orc_graph *g, const orc_run_opts *o, const double *LL, const double *LU,
            uint32_t *c, orc_run_result *res, orc_check_info *per_epoch, int32_t max_epochs);
int orc_count(const orc_graph *g, uint64_t seed, uint64_t stream, uint64_t first, uint64_t count,
              int sigma_mode, uint32_t *c, int64_t *edges_out);

/* Threaded runner: every epoch's samples split over nthreads threads, each
 * with a state frame of its own, summed at the epoch boundary; results
 * equal orc_run / orc_count exactly. */
int orc_run_mt(const orc_graph *g, const orc_run_opts *o, const double *LL, const double *LU,
               uint32_t *c, orc_run_result *res, orc_check_info *per_epoch, int32_t max_epochs,
               int nthreads);
int orc_count_mt(const orc_graph *g, uint64_t seed, uint64_t stream, uint64_t first, uint64_t count,
                 int sigma_mode, uint32_t *c, int64_t *edges_out, int nthreads);
void orc_neglog(int32_t n, const double *delta, double *L);

double orc_alloc_constant(int32_t n, const double *prior, double delta);
void orc_alloc_delta(int32_t n, const double *prior, double C, double delta, double beta,
                     double *LL, double *LU);
int orc_calibrate(const orc_graph *g, uint64_t seed, double omega, double delta, int sigma_mode,
                  uint32_t *cprime, double *C_out, double *LL, double *LU);
int orc_calibrate_mt(const orc_graph *g, uint64_t seed, double omega, double delta, int sigma_mode,
                     uint32_t *cprime, double *C_out, double *LL, double *LU, int nthreads);

void orc_brandes(const orc_graph *g, double *bc);

void orc_features(const orc_graph *g, double *x);
void orc_prior_from_output(int64_t n, const double *y, double omega, double *prior);
void orc_mlp_forward(const double *p, const double *x, int64_t rows, double *y);
double orc_mlp_loss_grad(const double *p, const double *x, const double *target, int64_t rows,
                         double *grad);
void orc_adam_step(double *p, const double *grad, double *m, double *v, int64_t count, int64_t step,
                   double lr, double b1, double b2, double eps);
void orc_mlp_init(uint64_t seed, double *p);
void orc_batch_rows(uint64_t seed, uint64_t step, int32_t batch, int64_t rows, int64_t *out);
void orc_mlp_train(const double *x, const double *y, int64_t rows, int32_t epochs, int32_t batch, double lr,
                   int32_t halve_every, uint64_t seed, double *p, double *losses);

#ifdef __cplusplus
}
#endif
#endif
