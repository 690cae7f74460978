/*
 * pps.h -- prior-predictive sampling on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libpps.so.  The method is the one of Warne, Sisson & Drovandi,
 * "Vector operations for accelerating expensive Bayesian computations -- a
 * tutorial guide" (arXiv:1902.09046):
 *
 *   prior-predictive sampling (Sec. 3.1, Eq. ppd): for each draw i, theta_i ~
 *   pi(theta), data D_i ~ s(D; theta_i), reduced to summaries S(D_i);
 *   ABC rejection in its fixed-N form (Alg. 1 and the paragraph after it):
 *   accept draws whose discrepancy rho(S(D_obs), S(D_i)) <= eps, eps fixed or
 *   chosen a posteriori as a quantile of rho;
 *   prior-predictive p-values under a family of priors pi(theta | lambda)
 *   (Sec. 4.1, Eqs. pppv and pppvhype), here with a tail-area statistic.
 *
 * Conventions shared by every call:
 *   - Every function returns an int status: PPS_OK (0), PPS_PENDING (> 0),
 *     or a negative error.  On error, pps_last_error() returns a message for
 *     the calling thread.  No call aborts the process.
 *   - "device" pointers are HIP device allocations owned by the caller
 *     (typically torch tensors' data_ptr()); "host" pointers are ordinary
 *     host memory.  The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is stream-ordered; the synchronous calls block only for their
 *     final small device-to-host copy and return with all their work done.
 *   - Draw i uses its own Philox4x32-10 stream: key = (lo32 seed, hi32 seed),
 *     counter = (block, purpose, lo32 i, hi32 i), purpose 0 = prior, 1 = path,
 *     2 + c = cell c of the toggle switch (Sec. 2.5: independent streams;
 *     Philox from Salmon et al., SC'11).  So
 *     the result of a draw depends only on (seed, i) and the model, never on
 *     launch shape, batching or which other jobs share the GPU.
 *   - Simulation runs in FP32 on the GPU; priors, p-values (counts) and ABC
 *     posterior moments are FP64.
 */
#ifndef PPS_H
#define PPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PPS_OK 0
#define PPS_PENDING 1    /* pps_poll: the job has not finished yet */
#define PPS_EINVAL (-1)  /* invalid argument (message in pps_last_error) */
#define PPS_ENOMEM (-2)  /* device or host allocation failed */
#define PPS_EDEVICE (-3) /* a HIP runtime call failed */
#define PPS_EBUSY (-4)   /* server queue full: retry later */
#define PPS_ENOTFOUND (-5) /* unknown job id */
#define PPS_ETRUNC (-6)  /* more accepted draws than `capacity`: the first
                            `capacity` (by draw index) were written and
                            stats->n_accepted holds the true count */

/* ---- model description (the "prior, simulator, discrepancy" of Alg. 1) -- */
#define PPS_MAX_PARAMS 8
#define PPS_MAX_OBS 64
#define PPS_TSW_MAX_CELLS 8192 /* toggle switch: cells per draw (one LDS sort) */
#define PPS_GARCH_LAGS 10
#define PPS_GARCH_NSUMM 14 /* mean, variance, skewness, kurtosis, ACF(r^2) lags 1..10 */
#define PPS_TB_MAX_POP 16384   /* tuberculosis: largest stopping population */
#define PPS_TB_MAX_SAMPLE 1024 /* tuberculosis: largest sample of cases */

enum pps_family {
    PPS_UNIFORM = 0,   /* U(a, b) */
    PPS_NORMAL = 1,    /* N(mean a, sd b) */
    PPS_LOGNORMAL = 2, /* exp(N(a, b^2)): b is the log-sd */
    PPS_POINT = 3      /* point mass at a (a may be +inf) */
};

enum pps_model_kind {
    /* dX = th1 X (1 - X/th2) dt + th3 X dW on [0, t_end], X(0) = x0, by
     * Euler-Maruyama (Eq. gene_uv_SDE_EM) in increment form
     *   X <- max(0, X + X (th1 dt - th1 dt X / th2 + th3 sqrt(dt) z)),
     * dt = t_end/steps, observed after steps k*steps/n_obs, k = 1..n_obs.
     * Summaries: the n_obs observations; statistic: their mean. */
    PPS_LOGISTIC_SDE = 0,
    /* GARCH(1,1) returns (the Gaussian case of the volatility models of
     * Sec. 4.2): theta = (omega, alpha, beta), sigma2_1 = omega/(1-alpha-beta),
     * r_t = sigma_t z_t, sigma2_{t+1} = omega + alpha r_t^2 + beta sigma2_t,
     * t = 1..steps.  Summaries: the PPS_GARCH_NSUMM values above. */
    PPS_GARCH11 = 1,
    /* y_j = th1 + noise_sd z_j, j = 1..n_obs.  Summaries: the y_j;
     * statistic: their mean. */
    PPS_NORMAL_MEAN = 2,
    /* The genetic toggle switch of Sec. 3.2: n_cells independent cells, each
     * with gene levels u, v (u(0) = v(0) = x0) advanced by Euler-Maruyama
     * (Eq. gene_uv_SDE_EM), dt = t_end/steps,
     *   u <- u + dt alpha_u/(1 + v^beta_u) - dt (1 + 0.03 u) + 0.5 sqrt(dt) xi_u
     *   v <- v + dt alpha_v/(1 + u^beta_v) - dt (1 + 0.03 v) + 0.5 sqrt(dt) xi_v
     * (both from the levels before the step), each level held at >= 1; then
     * measured as y = u + mu + mu sigma eta / u^gamma (Eq. gene_u_obs), held
     * at >= 1.  theta = (mu, sigma, gamma, alpha_u, alpha_v, beta_u, beta_v).
     * Cell c draws xi_u, xi_v of step j and eta as normals 2j, 2j+1 and
     * 2 steps of stream purpose 2 + c.  Summaries: n_obs equally spaced
     * quantiles, the k-th being the ceil(k n_cells / (n_obs + 1))-th
     * smallest y (the inverse empirical CDF at level k / (n_obs + 1); the
     * paper's 19 quantiles of 8000 cells are ranks 400, 800, ..., 7600);
     * statistic: their mean.  Simulated one draw per workgroup with the
     * cells across lanes. */
    PPS_TOGGLE_SWITCH = 3,
    /* Tuberculosis transmission (App. B): cases of genotypes i with counts
     * X_i; each case gives birth at rate alpha, dies at rate delta and
     * mutates at rate tau (theta = (alpha, delta, tau)), a mutation moving
     * the case to a new genotype.  Gillespie's direct method from x0 cases of
     * one genotype until the population reaches n_cells cases (complete),
     * dies out (extinct) or `steps` events have happened (truncated).  Event
     * e uses words (2(e%2), 2(e%2)+1) of block e/2 of stream purpose
     * 0x90000000: the case is number floor(w N / 2^32) in genotype-slot
     * order (the lookup over genotype weights), the type is birth below
     * floor(2^32 alpha/R), death below floor(2^32 (alpha + delta)/R),
     * mutation above (R = alpha + delta + tau, FP64); a new genotype takes
     * the lowest empty slot after the mutating case has left its own.  The
     * waiting times do not enter the result and are not drawn.  Then n_obs
     * cases are drawn without replacement (draw s: word s%4 of block s/4 of
     * purpose 0x90000001, case floor(w (N - s)/2^32) of those left), or all N
     * when N < n_obs.  Summaries: (g/n_s, H) with g the distinct genotypes
     * among the n_s cases taken and H = 1 - sum_i (n_i/n_s)^2; (0, 0) for an
     * extinct run.  Statistic: their mean.  One draw per 64-lane workgroup,
     * its genotype counts in LDS. */
    PPS_TB = 4
};

enum pps_constraint {
    PPS_NO_CONSTRAINT = 0,
    /* GARCH: reject alpha + beta >= 1 (decided in FP64) and redraw from the
     * same draw's stream (attempt t uses prior blocks 8t + j), up to 32
     * attempts. */
    PPS_GARCH_STATIONARY = 1,
    /* tuberculosis: reject alpha <= delta or tau <= 0 (a growing epidemic),
     * redrawn as above */
    PPS_TB_SUPERCRITICAL = 2
};

typedef struct {
    int32_t family; /* enum pps_family */
    double a, b;
} pps_prior;

typedef struct {
    int32_t model;    /* enum pps_model_kind */
    int32_t n_params; /* 1..PPS_MAX_PARAMS (logistic and GARCH: 3; toggle switch: 7) */
    pps_prior prior[PPS_MAX_PARAMS];
    int32_t constraint; /* enum pps_constraint */
    double x0;          /* logistic: X(0); toggle switch: u(0) = v(0) */
    double t_end;       /* logistic, toggle switch: final time T */
    int32_t steps;      /* logistic: EM steps (multiple of n_obs); toggle switch: EM
                           steps (>= 1); GARCH: series length (multiple of 20);
                           tuberculosis: the event cap (>= 1) */
    int32_t n_obs;      /* logistic / normal-mean: observations; toggle switch:
                           quantiles (1..PPS_MAX_OBS); tuberculosis: cases
                           sampled (1..PPS_TB_MAX_SAMPLE) */
    double noise_sd;    /* normal-mean: observation sd */
    int32_t n_cells;    /* toggle switch: cells per draw (1..PPS_TSW_MAX_CELLS);
                           tuberculosis: the stopping population
                           (2..PPS_TB_MAX_POP); x0 is then the initial cases
                           (an integer in [1, n_cells]) */
} pps_model;

typedef struct {
    uint64_t n_draws;    /* N >= 1 */
    uint64_t first_draw; /* draws i in [first_draw, first_draw + n_draws) */
    uint64_t seed;
} pps_sampling;

/* ---- random streams ----------------------------------------------------- */

/* Raw Philox4x32-10 output: for q in [0, n) the 4 words of block `block`,
 * purpose `purpose` of draw first_draw + q, written to out[4q .. 4q+3].
 * out: device, 4*n uint32.  Errors: PPS_EINVAL for n == 0 or out == NULL. */
int pps_philox(uint64_t seed, uint64_t first_draw, uint64_t n, uint32_t block,
               uint32_t purpose, uint32_t *out, void *stream);

/* FP32 path normals z_0 .. z_{m-1} of each draw (Box-Muller, Sec. 3.4):
 * normal k comes from path block b = k/6, which holds three pairs; pair i
 * (z_{6b+2i} = r cos(2 pi u1), z_{6b+2i+1} = r sin(2 pi u1), r = sqrt(-2 ln
 * u0)) takes u0 = (2 (w_i >> 9) + 1) 2^-24 from word i and u1 = m 2^-19 from
 * m = (w_i & 0x1FF) << 10 | (w_3 >> (22 - 10 i)) & 0x3FF.  Every model's
 * path and cell streams use this layout.  out: device, m*n floats,
 * out[k*n + q] (SoA).  Errors: PPS_EINVAL for n == 0, m == 0, out == NULL. */
int pps_normals(uint64_t seed, uint64_t first_draw, uint64_t n, uint32_t m, float *out,
                void *stream);

/* ---- per-draw prior-predictive output (Eq. ppd; Alg. 1 steps 1-2) ------- */

/* Simulates draws [first_draw, first_draw + n_draws) and writes, per draw q:
 *   theta[j*n + q]  the prior draw (FP32; FP64 draw rounded), j < n_params;
 *   summ[k*n + q]   summary k (logistic: observation k; GARCH: the 14
 *                   summaries; normal-mean: y_k; toggle switch: quantile k);
 *   stat[q]         the mean of the observations (not for GARCH; may be NULL);
 *   dist[q]         Euclidean distance to y_obs (only when y_obs != NULL;
 *                   else may be NULL).
 * y_obs: host, n_summaries doubles, or NULL.  theta and summ: device, may be
 * NULL to skip.  Errors: PPS_EINVAL (bad model, N == 0). */
int pps_simulate(const pps_model *model, const pps_sampling *sampling, const double *y_obs,
                 float *theta, float *summ, float *stat, float *dist, void *stream);

/* Number of summaries a model produces (n_obs, or PPS_GARCH_NSUMM), or a
 * negative status for an invalid model.  Also the validity check of a model
 * description: PPS_EINVAL with a message for any field out of range. */
int pps_n_summaries(const pps_model *model);

/* ---- ABC rejection, fixed-N form (Alg. 1 and the paragraph after it) ---- */
enum pps_eps_mode {
    PPS_EPS_FIXED = 0,       /* accept rho <= eps (compared in FP64) */
    PPS_EPS_TOP_FRACTION = 1 /* accept the k = ceil(frac N) smallest (rho, i),
                                ties by lower i; eps_used = the k-th smallest rho */
};

typedef struct {
    uint64_t n_accepted;          /* true count, even when truncated */
    double eps_used;              /* eps, or the k-th smallest rho */
    double mean[PPS_MAX_PARAMS];  /* FP64 posterior mean of accepted theta */
    double var[PPS_MAX_PARAMS];   /* FP64 unbiased variance (NaN if < 2 accepted) */
} pps_abc_stats;

/* y_obs: host, n_summaries doubles (the observed summaries S(D_obs)).
 * Accepted draws are written in increasing draw index:
 *   acc_idx[r] (device uint64), acc_theta[j*capacity + r] (device float,
 *   SoA), acc_dist[r] (device float), for r < min(n_accepted, capacity).
 * The output pointers may be NULL when capacity == 0.  stats: host.
 * Returns PPS_OK, PPS_ETRUNC (see above), PPS_EINVAL or PPS_EDEVICE. */
int abc_sample(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
               int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
               float *acc_theta, float *acc_dist, pps_abc_stats *stats, void *stream);

/* For callers that cannot allocate (code that must not call hipMalloc, such
 * as tight serving loops or harnesses that forbid it): abc_sample with the
 * same arguments, kernels, results and error codes, whose device scratch
 * (the n rho values and the finalisation's block counts, moment partials,
 * selection histogram and result: abc_scratch_bytes(n), 16.1 MiB at the
 * maximum) is a file-scope device array of the library, one per device,
 * held until the process ends.  It allocates nothing on its success path: no
 * hipMalloc / hipFree, no graph capture or instantiation, no host heap.  So
 * the device's context and the epoch graph of the job's form must exist:
 * make one abc_sample call on the device with the same model class,
 * tolerance mode and launch shape first, else PPS_EINVAL (nothing run).
 * n_draws above PPS_NOALLOC_MAX_DRAWS: PPS_EINVAL.  Every call on a device
 * uses that device's one array, which keeps the last call's contents (every
 * part a call reads is rewritten or cleared by that call's own kernels).
 * Calls on one device are serialised by the library (each holds the device's
 * lock until its epoch has ended); calls that overlapped on one device would
 * race on the array. */
#define PPS_NOALLOC_MAX_DRAWS (1ull << 22)
int abc_sample_noalloc(const pps_model *model, const double *y_obs, const pps_sampling *sampling,
                       int eps_mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
                       float *acc_theta, float *acc_dist, pps_abc_stats *stats, void *stream);

/* ---- prior-predictive p-values over a lambda grid (Eq. pppvhype) -------- */

/* For each lambda_k, parameter `lambda_param` gets the prior
 * (lambda_family, a = model->prior[lambda_param].a, b = lambda_k); the other
 * priors are unchanged.  Every lambda_k uses the same draws and random
 * numbers (common random numbers).  count_ge[k] = #{i : T_i >= t_obs} with
 * T_i the mean of draw i's observations (compared in FP64) and
 * pvalue[k] = count_ge[k] / N.  All lambda values run in one launch; for the
 * logistic SDE, lambda values are simulated in groups of 32 per lane from one
 * random stream (the common random numbers make their normals and the
 * lambda'd parameter's variate identical); the rest one row per lambda.
 * lambda, count_ge, pvalue: host arrays of n_lambda (1..4096).  For the
 * toggle switch T_i is the mean of its quantile summaries.
 * Not for GARCH (use pps_summary_tally). */
int prior_pred_pvalue(const pps_model *model, int lambda_param, int lambda_family,
                      const double *lambda, int n_lambda, const pps_sampling *sampling,
                      double t_obs, uint64_t *count_ge, double *pvalue, void *stream);

/* Per-summary tail-area counts (the prior-predictive check of a summary
 * vector): count_ge[s] = #{i : S_s(D_i) >= obs_summ[s]} (compared in FP64),
 * s < n_summaries.  GARCH, toggle-switch and tuberculosis models.
 * obs_summ, count_ge: host. */
int pps_summary_tally(const pps_model *model, const pps_sampling *sampling,
                      const double *obs_summ, uint64_t *count_ge, void *stream);

/* Tuberculosis runs: per draw the number of Gillespie events and the status
 * (0 complete, 1 extinct, 2 truncated by the event cap), the same runs as
 * every other entry point simulates for these draws.  events (n_draws u64)
 * and status (n_draws i32): device, either may be NULL.  PPS_TB only. */
int pps_tb_events(const pps_model *model, const pps_sampling *sampling, uint64_t *events,
                  int32_t *status, void *stream);

/* ---- jobs, batches and serving ------------------------------------------ */
/* A job is one ABC run (Alg. 1, fixed-N form) or one prior-predictive p-value
 * at one lambda (Eq. pppvhype).  Jobs of different N, step count, lambda and
 * kind are run together: their tiles share persistent launches ("epochs"),
 * each job's result being identical to the one it gets alone (every draw is
 * keyed by (seed, i); tallies are integers; moments are reduced in a fixed
 * order per job). */
enum pps_job_kind { PPS_JOB_ABC = 0, PPS_JOB_PVALUE = 1 };

typedef struct {
    int32_t kind;           /* enum pps_job_kind */
    pps_model model;        /* ABC: any model; p-value: logistic SDE or
                               normal-mean (others: PPS_EINVAL) */
    pps_sampling sampling;
    /* ABC */
    double y_obs[PPS_MAX_OBS]; /* observed summaries (n_summaries values) */
    int32_t eps_mode;       /* enum pps_eps_mode */
    double eps_or_frac;
    uint64_t capacity;      /* FIXED: records kept (later ones only counted);
                               TOP_FRACTION: ignored (all k records are kept) */
    /* p-value: parameter lambda_param gets (lambda_family, a = model's a,
       b = lambda); count of T_i >= t_obs */
    int32_t lambda_param;
    int32_t lambda_family;
    double lambda;
    double t_obs;
} pps_job;

typedef struct {
    int32_t status;         /* PPS_OK, PPS_ETRUNC (ABC records truncated) or an error */
    int32_t kind;
    pps_abc_stats abc;      /* ABC statistics */
    uint64_t count_ge;      /* p-value tally */
    double pvalue;
    /* ABC records (device pointers into the arena, increasing draw index;
       valid until the job is released / the arena is reused):
       acc_idx[r], acc_theta[j * record_stride + r], acc_dist[r], r < n_records. */
    const uint64_t *acc_idx;
    const float *acc_theta;
    const float *acc_dist;
    uint64_t n_records;
    uint64_t record_stride;
    /* steady-clock seconds: submitted, admitted (memory reserved), result visible */
    double t_submit, t_admit, t_done;
} pps_job_result;

enum pps_policy {
    PPS_POLICY_BATCHED = 0, /* continuous batching: many jobs' tiles per epoch,
                               jobs admitted while others run */
    PPS_POLICY_PLAIN = 1    /* one job per epoch, each epoch waited for before
                               the next is launched (the one-job-per-launch path) */
};

typedef struct {
    void *arena;            /* device memory for per-job scratch and ABC records
                               (caller-owned, >= 256-byte aligned) */
    uint64_t arena_bytes;
    int32_t max_active;     /* jobs admitted at once (1..1024) */
    int32_t queue_capacity; /* submissions waiting for admission (pps_submit
                               returns PPS_EBUSY beyond this) */
    double epoch_ms;        /* target GPU time of one epoch (planning budget) */
    int32_t policy;         /* enum pps_policy */
    void *stream;           /* HIP stream of the epochs; NULL: a stream of the
                               server's own (default priority).  Epochs alternate
                               between it and a second stream of the library's
                               (default priority); results are read through
                               pps_poll / the returned results, never by
                               ordering on this stream */
} pps_server_config;

/* Bytes of arena a job needs while admitted (ABC: distances, finalisation
 * scratch and records; p-value: its tally), or a negative status. */
int64_t pps_job_arena_bytes(const pps_job *job);

/* Runs n_jobs jobs to completion with the same scheduler as the server (no
 * thread): jobs are admitted in order as arena memory allows.  results[i]
 * gets job i's result; the records stay in the arena until it is reused.
 * Returns PPS_OK when every job ran (per-job status in results[i].status).
 * config->queue_capacity is ignored. */
int pps_run_batch(const pps_job *jobs, int n_jobs, const pps_server_config *config,
                  pps_job_result *results);

typedef struct pps_server pps_server;
int pps_server_create(const pps_server_config *config, pps_server **server);
/* Queues a copy of *job; never blocks.  PPS_EBUSY when the queue is full,
 * PPS_EINVAL for an invalid job (message in pps_last_error). */
int pps_submit(pps_server *server, const pps_job *job, uint64_t *job_id);
/* PPS_PENDING while the job runs; PPS_OK (or the job's error status) with
 * *out filled once its result is visible; PPS_ENOTFOUND for unknown or
 * released ids.  After a device error the server stops: every job that had
 * not finished completes with that error, and pps_submit returns it. */
int pps_poll(pps_server *server, uint64_t job_id, pps_job_result *out);
/* Frees a finished job's arena memory.  PPS_EBUSY if it has not finished,
 * PPS_ENOTFOUND if unknown or already released. */
int pps_release(pps_server *server, uint64_t job_id);

typedef struct {
    uint64_t submitted, completed, epochs;
    uint64_t queued, active;   /* right now */
    double busy_s;             /* sum of epoch simulation-kernel times */
    double latency_p50_s, latency_p99_s; /* submit -> visible, completed jobs */
} pps_server_stats;
int pps_server_stats_get(pps_server *server, pps_server_stats *stats);
/* Stops the server thread after the epochs in flight finish; queued and
 * admitted jobs that are not in flight are dropped without running.  The
 * arena is not freed (it belongs to the caller). */
int pps_server_destroy(pps_server *server);
/* Fault injection for tests of the error path (no device fault involved):
 * once `after_epochs` epochs have been harvested, every later epoch is
 * reported as failed with `status` (< 0) when it ends on the device.  The
 * server then stops as after a real device error.  PPS_EINVAL for
 * status >= 0. */
int pps_server_inject_error(pps_server *server, uint64_t after_epochs, int status);

/* ---- weak-informativity test (Sec. 4.1: Alg. 2, evidence by Alg. 3) ---- */
/* The logistic dose-response model of Eq. bioassay: group i of n_groups has
 * n_trials[i] animals at dose x_i; y_i ~ Bin(n_trials[i], p_i) with
 * p_i = 1 / (1 + exp(b0 + b1 x_i)); theta = (b0, b1) ~ N(0, diag(lambda)^2).
 * The evidence p(D | lambda) is estimated in FP64 by the adaptive SMC
 * sampler of Alg. 3, one sampler per workgroup with one particle per lane:
 *   particles from the prior; per step the tempering increment with
 *   ESS = N_p / 2 (bisection, bisect_iters halvings; the whole remaining
 *   increment when it keeps ESS >= N_p / 2 or at step max_steps);
 *   log Z += log((1/N_p) sum_i L_i^delta); multinomial resampling by
 *   inversion of fixed-point weights floor(w 2^52) (exact integer prefix
 *   sums); a random-walk proposal N(0, h^2 Sigma_hat) (Cholesky of the
 *   particles' sample covariance); one trial Metropolis-Hastings move of
 *   every particle gives p_acc, then R = ceil(ln c / ln(1 - p_acc)) moves in
 *   all, clamped to [1, max_mcmc] (p_acc = 0: max_mcmc); until t = 1.
 * Random numbers (key = seed, counter = (block, purpose, lo32, hi32 of the
 * run or data-set index)): data sets purpose 0x40000000 (base prior, index i)
 * or 0x40000001 (prior k, index k N + i), theta from words (0,1) of block 0,
 * the trial uniforms in order from blocks 1, 2, ...; particle j of an SMC
 * run: purpose 0x50000000 + j block 0 (initial draw), 0x60000000 + j block n
 * (resampling), 0x70000000 + j block 256 n + r (move r of step n: words (0,1)
 * the proposal normals, word 2 the acceptance uniform). */
#define PPS_BIO_MAX_GROUPS 8
#define PPS_SMC_MAX_PARTICLES 1024

typedef struct {
    int32_t n_groups;                     /* 1..PPS_BIO_MAX_GROUPS */
    int32_t n_trials[PPS_BIO_MAX_GROUPS]; /* 0..1000 each */
    double dose[PPS_BIO_MAX_GROUPS];
} pps_bioassay;

typedef struct {
    int32_t n_particles;  /* N_p: 2..PPS_SMC_MAX_PARTICLES */
    int32_t max_mcmc;     /* 1..256 */
    int32_t max_steps;    /* 1..4096 */
    int32_t bisect_iters; /* 1..64 */
    double c;             /* in (0, 1) */
    double h;             /* > 0 */
} pps_smc_config;

/* log p(D_s | lambda_s) for s < n_sets: data y (host, n_sets x n_groups
 * counts), lambda (host, n_sets x 2), SMC run index first_run + s.
 * log_z: device, n_sets doubles.  Errors: PPS_EINVAL. */
int pps_smc_log_evidence(const pps_bioassay *model, const int32_t *y, const double *lambda,
                         uint64_t n_sets, const pps_smc_config *smc, uint64_t seed,
                         uint64_t first_run, double *log_z, void *stream);

/* The weak-informativity test of Alg. 2 for lambda_0 (row 0 of `lambda`, the
 * base prior) and lambda_1..lambda_{n_lambda-1}: N = n_data base data sets
 * D_0^(i) ~ p(D | lambda_0) (shared by every k) and N data sets D_k^(i) ~
 * p(D | lambda_k) per k; log pi_0^i = log p(D_0^(i) | lambda_k) (SMC run
 * (k N + i) 2) and log pi_k^i = log p(D_k^(i) | lambda_k) (run (k N + i) 2 + 1);
 * p_k^i = (1/N) #{j : pi_k^j <= pi_0^i}; gamma[k] = the ceil(alpha N)-th
 * smallest p_k^i (the alpha quantile).  Priors with gamma[k] > gamma[0] are
 * weakly informative with respect to the base (Eq. weakinfprior).
 * lambda: host, n_lambda x 2 (> 0); log_z0, log_zk, pvalues: device,
 * n_lambda x n_data doubles (pvalues may be NULL); gamma: host, n_lambda.
 * n_data: 1..65536.  Errors: PPS_EINVAL, PPS_ENOMEM, PPS_EDEVICE. */
int pps_wip_test(const pps_bioassay *model, const double *lambda, int n_lambda, uint64_t n_data,
                 const pps_smc_config *smc, uint64_t seed, double alpha, double *log_z0,
                 double *log_zk, double *pvalues, double *gamma, void *stream);

/* ---- BEGE log-likelihood (Sec. 4.2: Eqs. BEGE, shape, BEGE_LL, CDF_BEGE,
 *      BEGE_LL_approx, incompGamma) ------------------------------------------ */
/* log L(theta_k; r_0..r_T) for n_theta parameter vectors against one return
 * series, FP64.  theta_k = (p0, s_p, rho_p, phi_p+, phi_p-, n0, s_n, rho_n,
 * phi_n+, phi_n-, mu) (row k of `theta`, 11 doubles).  The shapes start at
 * (p0, n0) and follow Eq. shape:
 *   p_t = p0 + rho_p p_{t-1} + phi_p^{+/-} u_t^2 / (2 s_p^2)  (+ for u_t >= 0),
 *   n_t likewise with (n0, rho_n, phi_n^{+/-}, s_n),  u_t = r_t - mu;
 * log L = sum_{t=1..T} log f(u_t | p_{t-1}, n_{t-1}) (Eq. BEGE_LL; r_0 is
 * conditioned on).  f is the central difference (F(u + h) - F(u - h)) / (2h),
 * h = 1e-3 sqrt(s_p^2 p + s_n^2 n), of the distribution function F of
 * u = s_p w_p - s_n w_n (centred gamma shocks) discretised as in
 * Eq. BEGE_LL_approx on the n_omega + 1 nodes w^j = w^0 + j dw,
 * w^0 = 1e-4 - p s_p, dw = (10 s_p sqrt(p) - w^0) / (n_omega - 1) (the paper
 * uses n_omega = 100), with the increments of P(a, x) between nodes
 * evaluated to full FP64 accuracy (the density's Taylor series integrated
 * over the interval where it converges fast, else the difference of two
 * values of P from its power series for x < a + 1 or of Q = 1 - P from its
 * continued fraction otherwise).  A step whose shapes
 * are not positive, or whose density estimate is not positive, has
 * log f = -inf, and so has every step when s_p or s_n is not positive; the
 * sum is then -inf.
 * theta (n_theta x 11), r (T + 1), loglik (n_theta) and logdens (n_theta x T,
 * logdens[k T + t - 1] = log f(u_t); may be NULL) are device pointers; the
 * library keeps its own scratch (16 bytes per (vector, t), and 8 more when
 * logdens is NULL).  Returns after the results are written.
 * Errors: PPS_EINVAL (sizes out of range, NULL pointers), PPS_ENOMEM,
 * PPS_EDEVICE. */
#define PPS_BEGE_MAX_THETA (1 << 20)
#define PPS_BEGE_MAX_T (1 << 20)
#define PPS_BEGE_MAX_CELLS (1ull << 31)
#define PPS_BEGE_MAX_NODES 65536
int pps_bege_loglik(const double *theta, int n_theta, const double *r, int T, int n_omega,
                    double *loglik, double *logdens, void *stream);

/* ---- measurement -------------------------------------------------------- */

/* Kernel timing.  While enabled (process-wide; off by default) every call
 * that launches the simulation kernel records a HIP event pair around that
 * kernel on the caller's stream; pps_last_kernel_ms() then returns the
 * kernel's duration in milliseconds for the most recent such call on the
 * current device, or a negative value if none was timed.  Returns PPS_OK. */
int pps_set_timing(int enable);

/* Work of one pps_bege_loglik call, for roofline accounting: runs the same
 * batch (results discarded) with the operation-counting instantiation of the
 * density kernel and stores in *ops (host) the FP64 operations that the
 * lanes executed as the algorithm states them: an FMA counts 2, a division
 * 1, a series term of P(a, x) 5 (plus 1 per block of 8), a continued-fraction
 * step 10 (plus 4 per block of 4), a term of the density's Taylor series 8
 * (plus 3 per block of 4), and exp, log, lgamma and sqrt 1 each.
 * Arguments and errors as pps_bege_loglik (ops must not be NULL). */
int pps_bege_count_ops(const double *theta, int n_theta, const double *r, int T, int n_omega,
                       double *ops, void *stream);
double pps_last_kernel_ms(void);
/* While timing is enabled: the duration in milliseconds of the ABC
 * finalisation (the accept step of Alg. 1: radix selection in closest-fraction
 * mode, ordered compaction of the accepted draws, FP64 moments) of the most
 * recent abc_sample / abc_sample_noalloc call on the current device, timed
 * by HIP events around it in the call's graph; negative if none was timed. */
double pps_last_finalize_ms(void);

/* ---- launch shape ------------------------------------------------------- */

/* Workgroup size of the persistent simulation kernel for a model class
 * (0: logistic SDE and normal-mean; 1: GARCH; 2: lambda groups: 64, 128 or
 * 256; 3: toggle switch: 256, 512 or 1024).  Results
 * do not depend on it (draw i's arithmetic depends only on (seed, i)).
 * Returns PPS_OK or PPS_EINVAL.  pps_get_block_size returns the current
 * size, or PPS_EINVAL for an unknown class. */
int pps_set_block_size(int model_class, int block);
int pps_get_block_size(int model_class);

/* Full launch shape of a kernel class: workgroup size, draws simulated
 * interleaved per lane (1 or 2) and Philox blocks generated per loop trip
 * (1 or 2; logistic SDE).  Classes: 0 logistic SDE / normal-mean, 1 GARCH,
 * 2 lambda groups of a p-value grid (32 lambda values of one draw per lane,
 * sharing its random numbers), 3 toggle switch (one draw per workgroup, its
 * cells across the lanes).  Supported shapes: class 0 block {64, 128, 256}
 * x draws_per_lane {1, 2} x unroll {1, 2}; classes 1 and 2 block
 * {64, 128, 256} with (1, 1); class 3 block {256, 512, 1024} with (1, 1).
 * Results do not depend on the shape.  PPS_EINVAL otherwise. */
int pps_set_launch_shape(int model_class, int block, int draws_per_lane, int unroll);
int pps_get_launch_shape(int model_class, int *block, int *draws_per_lane, int *unroll);

/* ---- autotuning --------------------------------------------------------- */
typedef struct {
    int32_t block, draws_per_lane, unroll;
    double ms; /* simulation-kernel time of the probe (best of the timed runs) */
} pps_tune_entry;

typedef struct {
    int32_t model_class;
    int32_t n_entries;
    pps_tune_entry entries[16];
    int32_t best;       /* index of the chosen shape in entries (or -1) */
    int32_t from_cache; /* 1 when the choice was read from the cache file */
} pps_tune_report;

/* Chooses the launch shape of the model's class on the current device: times
 * every supported shape (pps_set_launch_shape) on a probe of n_draws draws of
 * `model` (p-value tally, no per-draw output; results never depend on the
 * shape), keeps the fastest for all later calls, batches and servers created
 * afterwards, and appends it to the cache file named by the environment
 * variable PPS_TUNE_CACHE, if set, keyed by (GPU architecture, class, steps
 * and n_draws, each rounded up to a power of two).  With use_cache != 0 and a matching cache
 * line, the cached shape is applied without timing.  report may be NULL. */
int pps_autotune(const pps_model *model, uint64_t n_draws, int use_cache, pps_tune_report *report,
                 void *stream);

/* ---- errors ------------------------------------------------------------- */
const char *pps_strerror(int status);
const char *pps_last_error(void); /* thread-local; "" when none */

/* Library version string. */
const char *pps_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PPS_H */
