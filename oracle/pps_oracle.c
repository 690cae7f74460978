/*
 * FP64 CPU oracle for prior-predictive sampling (Warne, Sisson & Drovandi,
 * "Vector operations for accelerating expensive Bayesian computations -- a
 * tutorial guide", arXiv:1902.09046).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Nothing in the product path may link,
 * load or call it; it shares no code, header or constant table with the HIP
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.
 *
 * What it computes, following the paper:
 *   - prior-predictive sampling (Sec. 3.1, Eq. ppd): draw theta from the
 *     prior, simulate data given theta;
 *   - ABC rejection in its fixed-N form (Alg. 1 and the paragraph after it):
 *     generate N (theta, D) pairs, then accept by a tolerance epsilon that is
 *     either fixed or chosen a posteriori from the empirical distribution of
 *     the discrepancy;
 *   - the prior-predictive p-value under a family of priors pi(theta|lambda)
 *     (Sec. 4.1, Eqs. pppv and pppvhype), with a tail-area statistic in place
 *     of the predictive density;
 *   - Euler-Maruyama time stepping (Sec. 3.3, Eq. gene_uv_SDE_EM) applied to
 *     the paper's genetic toggle switch (Sec. 3.2, Eqs. gene_uv_SDE and
 *     gene_u_obs; 19 quantiles of the cell measurements as summaries) and to
 *     a stochastic logistic SDE; a GARCH(1,1) recursion (the Gaussian special
 *     case of the volatility family of Sec. 4.2); a normal-mean model;
 *   - independent random streams per draw (Sec. 2.5, option (ii) taken to
 *     the limit): the counter-based Philox4x32-10 generator of Salmon, Moraes,
 *     Dror and Shaw (SC'11), keyed by the seed, with the draw index in the
 *     counter, so that every draw is reproducible on its own;
 *   - a static partition of draws over threads (Listing of the multithreaded
 *     sampler in Sec. 3.4; Appendix B discussion of static scheduling).
 *
 * Everything is IEEE double except the 32-bit integer RNG.  Where the paper is
 * silent (observation times, uniform/normal generation, stream layout,
 * boundary handling, GARCH summaries) the readings are listed in the design
 * notes and restated at each function below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 5 "Philox").                    */
/* One round maps (c0,c1,c2,c3) with key (k0,k1) to                          */
/*   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))        */
/* and the key is bumped by the Weyl constants between rounds.               */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream layout (reading of "keyed by (seed, i)"): key = (lo32 seed, hi32
 * seed); counter = (block b, purpose, lo32 i, hi32 i).  Purpose 0 = prior
 * draws, 1 = the simulated path, 2 + c = cell c of a multi-cell model (the
 * toggle switch simulates every cell of a draw from its own stream).        */
enum { OR_PURPOSE_PRIOR = 0, OR_PURPOSE_PATH = 1, OR_PURPOSE_CELL0 = 2 };

void or_stream_block(uint64_t seed, uint64_t draw, uint32_t block, uint32_t purpose,
                     uint32_t out[4])
{
    uint32_t ctr[4] = { block, purpose, (uint32_t)draw, (uint32_t)(draw >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    or_philox4x32_10(ctr, key, out);
}

/* Uniform on the open interval: the top 23 bits of a word select the cell
 * midpoint (2k+1)/2^24, so the value is never 0 or 1 and is exact in both
 * float and double.                                                          */
double or_uniform(uint32_t word)
{
    double k = (double)(word >> 9);
    return (2.0 * k + 1.0) / 16777216.0;
}

/* Box-Muller transform (the paper's MKL generator uses the Box-Muller method,
 * Sec. 3.4): two uniforms give two independent standard normals.            */
void or_box_muller(uint32_t w0, uint32_t w1, double *z0, double *z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = or_uniform(w0);
    double u1 = or_uniform(w1);
    double radius = sqrt(-2.0 * log(u0));
    *z0 = radius * cos(two_pi * u1);
    *z1 = radius * sin(two_pi * u1);
}

/* Path normals of one draw: block b of the stream holds normals 6b .. 6b+5
 * as three Box-Muller pairs (reading of Sec. 3.4: the generator's 128 bits
 * serve three pairs, 42 bits each).  Pair i (i = 0, 1, 2) gives normals
 * 6b + 2i (cosine) and 6b + 2i + 1 (sine):
 *   radius uniform u0 from word i: its top 23 bits k, u0 = (2k+1)/2^24;
 *   angle uniform u1 from 19 further bits: the low 9 bits of word i followed
 *   by bits 22 - 10i .. 31 - 10i of word 3 form m, u1 = m/2^19 (2^19 equally
 *   spaced angles from 0; unlike u0, the angle may be 0).
 * The 126 bits used are disjoint.                                           */
#define OR_NORMALS_PER_BLOCK 6

double or_angle_uniform(uint32_t word_i, uint32_t word3, int i)
{
    const uint32_t m = ((word_i & 0x1FFu) << 10) | ((word3 >> (22 - 10 * i)) & 0x3FFu);
    return (double)m / 524288.0;
}

/* One Box-Muller pair from its two uniforms.                                */
static void box_muller_u(double u0, double u1, double *z0, double *z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double radius = sqrt(-2.0 * log(u0));
    *z0 = radius * cos(two_pi * u1);
    *z1 = radius * sin(two_pi * u1);
}

static void normals_block(uint64_t seed, uint64_t draw, uint32_t block, uint32_t purpose,
                          double z[OR_NORMALS_PER_BLOCK])
{
    uint32_t w[4];
    or_stream_block(seed, draw, block, purpose, w);
    for (int i = 0; i < 3; ++i)
        box_muller_u(or_uniform(w[i]), or_angle_uniform(w[i], w[3], i), &z[2 * i], &z[2 * i + 1]);
}

void or_path_block(uint64_t seed, uint64_t draw, uint32_t block, double z[OR_NORMALS_PER_BLOCK])
{
    normals_block(seed, draw, block, OR_PURPOSE_PATH, z);
}

double or_path_normal(uint64_t seed, uint64_t draw, uint64_t n)
{
    double z[OR_NORMALS_PER_BLOCK];
    or_path_block(seed, draw, (uint32_t)(n / OR_NORMALS_PER_BLOCK), z);
    return z[n % OR_NORMALS_PER_BLOCK];
}

/* Normal n of cell `cell` of a draw (same block layout, purpose 2 + cell).  */
double or_cell_normal(uint64_t seed, uint64_t draw, uint32_t cell, uint64_t n)
{
    double z[OR_NORMALS_PER_BLOCK];
    normals_block(seed, draw, (uint32_t)(n / OR_NORMALS_PER_BLOCK), OR_PURPOSE_CELL0 + cell, z);
    return z[n % OR_NORMALS_PER_BLOCK];
}

/* Sequential reader of the normals z_0, z_1, ... of one stream of a draw.  */
typedef struct {
    uint64_t seed, draw;
    uint32_t purpose;
    uint64_t next;
    double buf[OR_NORMALS_PER_BLOCK];
} normal_reader;

static void reader_init_purpose(normal_reader *r, uint64_t seed, uint64_t draw, uint32_t purpose)
{
    r->seed = seed;
    r->draw = draw;
    r->purpose = purpose;
    r->next = 0;
}

static void reader_init(normal_reader *r, uint64_t seed, uint64_t draw)
{
    reader_init_purpose(r, seed, draw, OR_PURPOSE_PATH);
}

static double reader_next(normal_reader *r)
{
    if (r->next % OR_NORMALS_PER_BLOCK == 0)
        normals_block(r->seed, r->draw, (uint32_t)(r->next / OR_NORMALS_PER_BLOCK), r->purpose,
                      r->buf);
    return r->buf[r->next++ % OR_NORMALS_PER_BLOCK];
}

/* ------------------------------------------------------------------------ */
/* Model description (plain data; independent of the GPU library's structs). */
/* ------------------------------------------------------------------------ */
enum { OR_UNIFORM = 0, OR_NORMAL = 1, OR_LOGNORMAL = 2, OR_POINT = 3 };
enum { OR_LOGISTIC = 0, OR_GARCH11 = 1, OR_NORMAL_MEAN = 2, OR_TOGGLE_SWITCH = 3, OR_TB = 4 };
enum { OR_NO_CONSTRAINT = 0, OR_GARCH_STATIONARY = 1, OR_TB_SUPERCRITICAL = 2 };
#define OR_MAX_PARAMS 8
#define OR_MAX_ATTEMPTS 32
#define OR_GARCH_LAGS 10
#define OR_GARCH_NSUMM (4 + OR_GARCH_LAGS)

typedef struct {
    int32_t family;
    double a, b;
} or_prior;

typedef struct {
    int32_t model;
    int32_t n_params;
    or_prior prior[OR_MAX_PARAMS];
    int32_t constraint;
    double x0;        /* logistic: initial state; toggle switch: u(0) = v(0) */
    double t_end;     /* logistic, toggle switch: final time T */
    int32_t steps;    /* logistic, toggle switch: Euler-Maruyama steps S;
                         GARCH: series length */
    int32_t n_obs;    /* logistic: observations; normal-mean: sample size;
                         toggle switch: number of quantiles; tuberculosis:
                         cases sampled at the end */
    double noise_sd;  /* normal-mean: observation sd */
    int32_t n_cells;  /* toggle switch: cells C; tuberculosis: the population
                         size at which a run stops */
} or_model;

/* One prior value from PRIOR block (8*attempt + j): uniform from word 0,
 * normal from words (0,1) through Box-Muller (first output).                */
static double prior_value(const or_prior *p, uint64_t seed, uint64_t draw, int j, int attempt)
{
    uint32_t w[4];
    or_stream_block(seed, draw, (uint32_t)(8 * attempt + j), OR_PURPOSE_PRIOR, w);
    double z0, z1;
    switch (p->family) {
    case OR_UNIFORM:
        return p->a + (p->b - p->a) * or_uniform(w[0]);
    case OR_NORMAL:
        or_box_muller(w[0], w[1], &z0, &z1);
        return p->a + p->b * z0;
    case OR_LOGNORMAL:
        or_box_muller(w[0], w[1], &z0, &z1);
        return exp(p->a + p->b * z0);
    case OR_POINT:
    default:
        return p->a;
    }
}

/* theta ~ pi(theta) (Alg. 1, first step).  With the GARCH stationarity
 * constraint, an attempt whose (alpha, beta) = (theta[1], theta[2]) has
 * alpha + beta >= 1 is rejected and the next attempt of the same draw's
 * stream is used; after OR_MAX_ATTEMPTS the last attempt is kept.
 * Returns the number of attempts used.                                      */
int or_prior_draw(const or_model *m, uint64_t seed, uint64_t draw, double *theta)
{
    int attempt = 0;
    for (;;) {
        for (int j = 0; j < m->n_params; ++j)
            theta[j] = prior_value(&m->prior[j], seed, draw, j, attempt);
        int ok = 1;
        if (m->constraint == OR_GARCH_STATIONARY)
            ok = theta[1] + theta[2] < 1.0;
        else if (m->constraint == OR_TB_SUPERCRITICAL)
            ok = theta[0] > theta[1] && theta[2] > 0.0;
        if (ok || attempt + 1 == OR_MAX_ATTEMPTS)
            return attempt + 1;
        ++attempt;
    }
}

/* ------------------------------------------------------------------------ */
/* Simulators.                                                               */
/* ------------------------------------------------------------------------ */

/* Stochastic logistic SDE dX = th1 X (1 - X/th2) dt + th3 X dW, integrated by
 * Euler-Maruyama (Eq. gene_uv_SDE_EM) with dt = T/S:
 *   X <- X + X (a - b X + c z),  a = th1 dt, b = th1 dt / th2, c = th3 sqrt(dt)
 * then absorbed at zero, X <- max(X, 0) (the paper clamps its gene levels at a
 * boundary the same way).  Observation k (k = 1..n_obs) is X after step
 * k*S/n_obs.  S must be a multiple of n_obs.                                  */
static void simulate_logistic(const or_model *m, const double *theta, uint64_t seed,
                              uint64_t draw, double *obs)
{
    const double dt = m->t_end / (double)m->steps;
    const double a = theta[0] * dt;
    const double b = theta[0] * dt / theta[1];
    const double c = theta[2] * sqrt(dt);
    const int stride = m->steps / m->n_obs;
    double x = m->x0;
    int k = 0;
    normal_reader rd;
    reader_init(&rd, seed, draw);
    for (int n = 0; n < m->steps; ++n) {
        double z = reader_next(&rd);
        x = x + x * (a - b * x + c * z);
        if (x < 0.0)
            x = 0.0;
        if ((n + 1) % stride == 0)
            obs[k++] = x;
    }
}

/* Normal-mean model: y_j = mu + sd * z_j for j = 1..n_obs, mu = theta[0].    */
static void simulate_normal_mean(const or_model *m, const double *theta, uint64_t seed,
                                 uint64_t draw, double *obs)
{
    normal_reader rd;
    reader_init(&rd, seed, draw);
    for (int j = 0; j < m->n_obs; ++j)
        obs[j] = theta[0] + m->noise_sd * reader_next(&rd);
}

/* GARCH(1,1) returns: sigma2_1 = omega / (1 - alpha - beta), then for
 * t = 1..L:  r_t = sqrt(sigma2_t) z_t,  sigma2_{t+1} = omega + alpha r_t^2 +
 * beta sigma2_t, z_t the t-th path normal.  No mean, no burn-in.              */
static void simulate_garch_series(const or_model *m, const double *theta, uint64_t seed,
                                  uint64_t draw, double *r)
{
    const double omega = theta[0], alpha = theta[1], beta = theta[2];
    double sigma2 = omega / (1.0 - alpha - beta);
    normal_reader rd;
    reader_init(&rd, seed, draw);
    for (int t = 0; t < m->steps; ++t) {
        double z = reader_next(&rd);
        r[t] = sqrt(sigma2) * z;
        sigma2 = omega + alpha * r[t] * r[t] + beta * sigma2;
    }
}

/* GARCH summaries by their definitions, two-pass:
 *   s[0] mean, s[1] variance (1/L), s[2] skewness m3/m2^1.5,
 *   s[3] kurtosis m4/m2^2 (not excess),
 *   s[4+k-1] = sum_{t<=L-k} (a_t - abar)(a_{t+k} - abar) / sum_t (a_t - abar)^2
 *   for the squared returns a_t = r_t^2, lags k = 1..10.                     */
static void garch_summaries(const double *r, int len, double *s)
{
    double mean = 0.0;
    for (int t = 0; t < len; ++t)
        mean += r[t];
    mean /= len;
    double m2 = 0.0, m3 = 0.0, m4 = 0.0;
    for (int t = 0; t < len; ++t) {
        double d = r[t] - mean;
        m2 += d * d;
        m3 += d * d * d;
        m4 += d * d * d * d;
    }
    m2 /= len; m3 /= len; m4 /= len;
    s[0] = mean;
    s[1] = m2;
    s[2] = m3 / pow(m2, 1.5);
    s[3] = m4 / (m2 * m2);
    double abar = 0.0;
    for (int t = 0; t < len; ++t)
        abar += r[t] * r[t];
    abar /= len;
    double den = 0.0;
    for (int t = 0; t < len; ++t)
        den += (r[t] * r[t] - abar) * (r[t] * r[t] - abar);
    for (int k = 1; k <= OR_GARCH_LAGS; ++k) {
        double num = 0.0;
        for (int t = 0; t + k < len; ++t)
            num += (r[t] * r[t] - abar) * (r[t + k] * r[t + k] - abar);
        s[4 + k - 1] = num / den;
    }
}

/* Genetic toggle switch (Sec. 3.2): expression levels u, v of two genes in
 * each of C independent cells follow the coupled SDEs of Eq. gene_uv_SDE,
 * integrated by Euler-Maruyama as in Eq. gene_uv_SDE_EM with dt = T/S:
 *   u <- u + dt alpha_u / (1 + v^beta_u) - dt (1 + 0.03 u) + 0.5 sqrt(dt) xi_u
 *   v <- v + dt alpha_v / (1 + u^beta_v) - dt (1 + 0.03 v) + 0.5 sqrt(dt) xi_v
 * both right-hand sides evaluated at the levels before the step; then each
 * level is held at the boundary 1 (the model keeps u, v >= 1).  After S steps
 * the cell is measured with the error model of Eq. gene_u_obs,
 *   y = u + mu + mu sigma eta / u^gamma,
 * and y is held at >= 1 like the levels.  theta = (mu, sigma, gamma, alpha_u,
 * alpha_v, beta_u, beta_v); u(0) = v(0) = x0.  Cell c uses the normals of
 * stream 2 + c: xi_u of step j is z_{2j}, xi_v is z_{2j+1}, eta is z_{2S}.   */
static void toggle_cell(const or_model *m, const double *theta, uint64_t seed, uint64_t draw,
                        int cell, double *u_out, double *v_out, double *y_out)
{
    const double mu = theta[0], sigma = theta[1], gamma = theta[2];
    const double alpha_u = theta[3], alpha_v = theta[4];
    const double beta_u = theta[5], beta_v = theta[6];
    const double dt = m->t_end / (double)m->steps;
    const double noise = 0.5 * sqrt(dt);
    double u = m->x0, v = m->x0;
    normal_reader rd;
    reader_init_purpose(&rd, seed, draw, OR_PURPOSE_CELL0 + (uint32_t)cell);
    for (int j = 0; j < m->steps; ++j) {
        const double xi_u = reader_next(&rd);
        const double xi_v = reader_next(&rd);
        const double u_next = u + dt * alpha_u / (1.0 + pow(v, beta_u)) - dt * (1.0 + 0.03 * u) +
                              noise * xi_u;
        const double v_next = v + dt * alpha_v / (1.0 + pow(u, beta_v)) - dt * (1.0 + 0.03 * v) +
                              noise * xi_v;
        u = u_next < 1.0 ? 1.0 : u_next;
        v = v_next < 1.0 ? 1.0 : v_next;
    }
    const double eta = reader_next(&rd);
    double y = u + mu + mu * sigma * eta / pow(u, gamma);
    if (y < 1.0)
        y = 1.0;
    *u_out = u;
    *v_out = v;
    *y_out = y;
}

static int cmp_double(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/* Rank (1-based) of the k-th of K equally spaced quantiles of C values: the
 * empirical quantile at level k/(K+1) taken as the inverse of the empirical
 * distribution function, i.e. the ceil(k C / (K+1))-th smallest value.  For
 * the paper's 19 quantiles of 8000 cells the levels are 0.05, ..., 0.95 and
 * the ranks 400, 800, ..., 7600.                                             */
static int64_t quantile_rank(int k, int n_quantiles, int n_cells)
{
    return ((int64_t)k * n_cells + n_quantiles) / (n_quantiles + 1);
}

/* Summaries of one toggle-switch draw (Sec. 3.2, following Vo et al.): the
 * n_obs equally spaced quantiles of the C measurements.  work: C doubles.   */
static void simulate_toggle(const or_model *m, const double *theta, uint64_t seed, uint64_t draw,
                            double *summ, double *work)
{
    for (int c = 0; c < m->n_cells; ++c) {
        double u, v;
        toggle_cell(m, theta, seed, draw, c, &u, &v, &work[c]);
    }
    qsort(work, (size_t)m->n_cells, sizeof(double), cmp_double);
    for (int k = 1; k <= m->n_obs; ++k)
        summ[k - 1] = work[quantile_rank(k, m->n_obs, m->n_cells) - 1];
}

/* Number of summaries (the "data" D of one draw) a model produces.          */
/* ------------------------------------------------------------------------ */
/* Tuberculosis transmission (App. B): a birth-death process of cases with  */
/* mutation to new genotypes, simulated event by event by the Gillespie     */
/* direct method.                                                           */
/* ------------------------------------------------------------------------ */
enum { OR_PURPOSE_TB_EVENT = 0x90000000u, OR_PURPOSE_TB_SAMPLE = 0x90000001u };
enum { OR_TB_COMPLETE = 0, OR_TB_EXTINCT = 1, OR_TB_TRUNCATED = 2 };

/* The genotype holding case m (0 <= m < sum X) in slot order: the lookup
 * over the genotype weights, i.e. the smallest i with X_0 + ... + X_i > m.   */
int or_tb_select(const uint32_t *X, int S, uint64_t m)
{
    uint64_t acc = 0;
    for (int i = 0; i < S; ++i) {
        acc += X[i];
        if (acc > m)
            return i;
    }
    return -1;
}

/* The lowest slot holding no case (where a new genotype is founded).        */
int or_tb_lowest_empty(const uint32_t *X, int S)
{
    for (int i = 0; i < S; ++i)
        if (X[i] == 0)
            return i;
    return -1;
}

/* A uniform integer in [0, n) from a 32-bit word: floor(w n / 2^32).       */
static uint64_t tb_scale(uint32_t w, uint64_t n)
{
    return ((uint64_t)w * n) >> 32;
}

/* Event-type thresholds on a 32-bit word: birth below floor(2^32 alpha/R),
 * death below floor(2^32 (alpha + delta)/R), mutation above; R = alpha +
 * delta + tau.  The sums and quotients are single IEEE FP64 operations.      */
void or_tb_thresholds(const double *theta, uint64_t *t_birth, uint64_t *t_death)
{
    const double ad = theta[0] + theta[1];
    const double r = ad + theta[2];
    *t_birth = (uint64_t)floor(ldexp(theta[0] / r, 32));
    *t_death = (uint64_t)floor(ldexp(ad / r, 32));
}

/* One run at theta = (alpha, delta, tau) (event rates per case: birth,
 * death, mutation).  X (n_stop slots, zeroed here) receives the final case
 * counts per genotype slot.  Start: x0 cases of one genotype in slot 0.
 * While 0 < N < n_stop and fewer than max_events events have happened:
 * event e draws words (w_case, w_type) = words (2(e%2), 2(e%2)+1) of block
 * e/2 of stream purpose 0x90000000; the case is number floor(w_case N/2^32)
 * and its genotype the lookup above; the event type follows the thresholds;
 * birth adds a case to the genotype, death removes one, mutation removes one
 * and founds a new genotype with one case in the lowest empty slot (after
 * the removal).  The waiting times of the direct method do not enter the
 * stopped state and are not drawn.  Returns the status (complete: N reached
 * n_stop; extinct; truncated) and the number of events.                      */
int or_tb_run(const double *theta, int n_stop, double x0, uint64_t max_events, uint64_t seed,
              uint64_t draw, uint32_t *X, uint64_t *events, uint64_t *n_final)
{
    for (int i = 0; i < n_stop; ++i)
        X[i] = 0;
    uint64_t tb, td;
    or_tb_thresholds(theta, &tb, &td);
    uint64_t N = (uint64_t)x0;
    if (N > (uint64_t)n_stop)
        N = (uint64_t)n_stop;
    X[0] = (uint32_t)N;
    uint64_t e = 0;
    uint32_t w[4] = {0, 0, 0, 0};
    int status;
    for (;;) {
        if (N >= (uint64_t)n_stop) {
            status = OR_TB_COMPLETE;
            break;
        }
        if (N == 0) {
            status = OR_TB_EXTINCT;
            break;
        }
        if (e >= max_events) {
            status = OR_TB_TRUNCATED;
            break;
        }
        if (e % 2 == 0)
            or_stream_block(seed, draw, (uint32_t)(e / 2), OR_PURPOSE_TB_EVENT, w);
        const uint32_t w_case = w[2 * (e % 2)], w_type = w[2 * (e % 2) + 1];
        const int i = or_tb_select(X, n_stop, tb_scale(w_case, N));
        if ((uint64_t)w_type < tb) {
            X[i] += 1;
            N += 1;
        } else if ((uint64_t)w_type < td) {
            X[i] -= 1;
            N -= 1;
        } else {
            X[i] -= 1;
            X[or_tb_lowest_empty(X, n_stop)] = 1;
        }
        ++e;
    }
    *events = e;
    *n_final = N;
    return status;
}

/* Summaries of the final population: n cases drawn without replacement
 * (draw s: word s%4 of block s/4 of stream purpose 0x90000001, the case
 * floor(w (N - s)/2^32) of those left, looked up as above), or all N cases
 * when N < n; g = the number of distinct genotypes among them and
 * H = 1 - sum_i (n_i/n_s)^2 (the gene diversity), n_s the cases taken.
 * summ = (g/n_s, H); (0, 0) for an empty population.  X is consumed; Y
 * (n_stop slots) is workspace.                                               */
void or_tb_summaries(uint32_t *X, uint32_t *Y, int n_stop, uint64_t N, int n, uint64_t seed,
                     uint64_t draw, double *summ)
{
    if (N == 0) {
        summ[0] = 0.0;
        summ[1] = 0.0;
        return;
    }
    uint64_t ns;
    if (N >= (uint64_t)n) {
        ns = (uint64_t)n;
        for (int i = 0; i < n_stop; ++i)
            Y[i] = 0;
        uint32_t w[4];
        for (uint64_t s = 0; s < ns; ++s) {
            if (s % 4 == 0)
                or_stream_block(seed, draw, (uint32_t)(s / 4), OR_PURPOSE_TB_SAMPLE, w);
            const int i = or_tb_select(X, n_stop, tb_scale(w[s % 4], N - s));
            X[i] -= 1;
            Y[i] += 1;
        }
    } else {
        ns = N;
        for (int i = 0; i < n_stop; ++i)
            Y[i] = X[i];
    }
    uint64_t g = 0, sq = 0;
    for (int i = 0; i < n_stop; ++i) {
        g += Y[i] > 0;
        sq += (uint64_t)Y[i] * Y[i];
    }
    summ[0] = (double)g / (double)ns;
    summ[1] = 1.0 - (double)sq / ((double)ns * (double)ns);
}

static void simulate_tb(const or_model *m, const double *theta, uint64_t seed, uint64_t draw,
                        double *summ, double *work)
{
    uint32_t *X = (uint32_t *)work;
    uint32_t *Y = X + m->n_cells;
    uint64_t events, N;
    or_tb_run(theta, m->n_cells, m->x0, (uint64_t)(uint32_t)m->steps, seed, draw, X, &events, &N);
    or_tb_summaries(X, Y, m->n_cells, N, m->n_obs, seed, draw, summ);
}

/* Per draw: theta, status, events, final N and summaries (for tests and the
 * event-rate figures).                                                       */
int or_tb_simulate(const or_model *m, uint64_t seed, uint64_t first, uint64_t n, double *theta,
                   int32_t *status, uint64_t *events, uint64_t *n_final, double *summ)
{
    if (m->model != OR_TB || m->n_params != 3 || m->n_cells < 1 || m->n_obs < 1)
        return -1;
    int oom = 0;
#pragma omp parallel
    {
        uint32_t *X = (uint32_t *)malloc(2 * (size_t)m->n_cells * sizeof(uint32_t));
        if (!X) {
#pragma omp atomic write
            oom = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (uint64_t q = 0; q < n; ++q) {
            if (!X)
                continue;
            const uint64_t draw = first + q;
            double *th = &theta[q * 3];
            or_prior_draw(m, seed, draw, th);
            uint64_t ev, N;
            status[q] = or_tb_run(th, m->n_cells, m->x0, (uint64_t)(uint32_t)m->steps, seed, draw, X,
                                  &ev, &N);
            events[q] = ev;
            n_final[q] = N;
            or_tb_summaries(X, X + m->n_cells, m->n_cells, N, m->n_obs, seed, draw, &summ[q * 2]);
        }
        free(X);
    }
    return oom ? -2 : 0;
}

int or_n_summaries(const or_model *m)
{
    if (m->model == OR_GARCH11)
        return OR_GARCH_NSUMM;
    if (m->model == OR_TB)
        return 2;
    return m->n_obs;
}

/* D ~ s(D; theta) reduced to its summaries (Alg. 1, second step).           */
static void simulate_summaries(const or_model *m, const double *theta, uint64_t seed,
                               uint64_t draw, double *summ, double *work)
{
    switch (m->model) {
    case OR_LOGISTIC:
        simulate_logistic(m, theta, seed, draw, summ);
        break;
    case OR_NORMAL_MEAN:
        simulate_normal_mean(m, theta, seed, draw, summ);
        break;
    case OR_TOGGLE_SWITCH:
        simulate_toggle(m, theta, seed, draw, summ, work);
        break;
    case OR_TB:
        simulate_tb(m, theta, seed, draw, summ, work);
        break;
    case OR_GARCH11:
    default:
        simulate_garch_series(m, theta, seed, draw, work);
        garch_summaries(work, m->steps, summ);
        break;
    }
}

/* Euclidean discrepancy rho(S(D_obs), S(D)) between summary vectors.        */
double or_distance(const double *x, const double *y, int n)
{
    double acc = 0.0;
    for (int k = 0; k < n; ++k)
        acc += (x[k] - y[k]) * (x[k] - y[k]);
    return sqrt(acc);
}

/* Tail-area statistic: the mean of the observations.                         */
double or_mean_stat(const double *x, int n)
{
    double acc = 0.0;
    for (int k = 0; k < n; ++k)
        acc += x[k];
    return acc / n;
}

static int model_ok(const or_model *m)
{
    if (m->n_params < 1 || m->n_params > OR_MAX_PARAMS)
        return 0;
    if (m->model == OR_LOGISTIC)
        return m->n_params >= 3 && m->n_obs > 0 && m->steps > 0 && m->steps % m->n_obs == 0;
    if (m->model == OR_NORMAL_MEAN)
        return m->n_obs > 0;
    if (m->model == OR_GARCH11)
        return m->n_params >= 3 && m->steps > OR_GARCH_LAGS;
    if (m->model == OR_TOGGLE_SWITCH)
        return m->n_params == 7 && m->steps > 0 && m->t_end > 0.0 && m->n_cells > 0 &&
               m->n_obs > 0;
    if (m->model == OR_TB)
        return m->n_params == 3 && m->n_cells > 0 && m->n_obs > 0 && m->x0 >= 1.0;
    return 0;
}

static size_t work_len(const or_model *m)
{
    if (m->model == OR_GARCH11)
        return (size_t)m->steps;
    if (m->model == OR_TOGGLE_SWITCH)
        return (size_t)m->n_cells;
    if (m->model == OR_TB)
        return (size_t)m->n_cells;  /* two uint32 arrays of n_cells */
    return 1;
}

/* Per-draw prior-predictive output for draws i in [first, first + n):
 *   theta[(i-first)*n_params + j], summ[(i-first)*ns + k],
 *   stat[i-first] = mean of the summaries (logistic / normal-mean) or NaN,
 *   dist[i-first] = distance to y_obs (when y_obs != NULL) or NaN,
 *   attempts[i-first] = prior attempts used (optional).
 * Returns 0, or -1 for an invalid model.                                    */
int or_simulate(const or_model *m, uint64_t seed, uint64_t first, uint64_t n,
                const double *y_obs, double *theta, double *summ, double *stat,
                double *dist, int32_t *attempts)
{
    if (!model_ok(m))
        return -1;
    const int np = m->n_params;
    const int ns = or_n_summaries(m);
    const size_t wl = work_len(m);
    int oom = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(wl * sizeof(double));
        if (!work) {
#pragma omp atomic write
            oom = 1;
        }
#pragma omp for schedule(static)
        for (int64_t q = 0; q < (int64_t)n; ++q) {
            if (!work)
                continue;
            uint64_t draw = first + (uint64_t)q;
            double *th = theta + (size_t)q * np;
            double *s = summ + (size_t)q * ns;
            int at = or_prior_draw(m, seed, draw, th);
            if (attempts)
                attempts[q] = at;
            simulate_summaries(m, th, seed, draw, s, work);
            if (stat)
                stat[q] = (m->model == OR_GARCH11) ? NAN : or_mean_stat(s, ns);
            if (dist)
                dist[q] = y_obs ? or_distance(s, y_obs, ns) : NAN;
        }
        free(work);
    }
    return oom ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* ABC rejection, fixed-N form (Alg. 1 and the paragraph after it).          */
/* ------------------------------------------------------------------------ */
enum { OR_EPS_FIXED = 0, OR_EPS_TOP_FRACTION = 1 };

typedef struct {
    double d;
    uint64_t i;
} dist_index;

static int cmp_dist_index(const void *pa, const void *pb)
{
    const dist_index *a = (const dist_index *)pa, *b = (const dist_index *)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    if (a->i < b->i) return -1;
    if (a->i > b->i) return 1;
    return 0;
}

static int cmp_u64(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

/* Accepted count for the top-fraction mode: k = ceil(frac * N), at least 1
 * and at most N.                                                             */
uint64_t or_top_count(double frac, uint64_t n)
{
    double k = ceil(frac * (double)n);
    if (k < 1.0) k = 1.0;
    if (k > (double)n) k = (double)n;
    return (uint64_t)k;
}

/* Accepts draws i in [first, first+n):
 *   FIXED:        rho <= eps;
 *   TOP_FRACTION: the k = ceil(frac N) smallest (rho, i) pairs, ordered by
 *                 rho then by i, with eps_used = the k-th smallest rho.
 * Outputs the accepted indices in increasing order with their theta (row
 * major, n_params per row) and rho, up to `capacity` rows; *n_acc is the true
 * count.  Posterior moments of the accepted theta: mean and unbiased variance
 * (NaN when fewer than 2 draws), summed in index order.
 * Returns 0, 1 when the output was truncated to capacity, -1 on bad input.  */
int or_abc(const or_model *m, const double *y_obs, uint64_t seed, uint64_t first, uint64_t n,
           int mode, double eps_or_frac, uint64_t capacity, uint64_t *acc_idx,
           double *acc_theta, double *acc_dist, uint64_t *n_acc, double *eps_used,
           double *mean, double *var)
{
    if (!model_ok(m) || n == 0)
        return -1;
    const int np = m->n_params;
    const int ns = or_n_summaries(m);
    double *theta = (double *)malloc((size_t)n * np * sizeof(double));
    double *summ = (double *)malloc((size_t)n * ns * sizeof(double));
    double *dist = (double *)malloc((size_t)n * sizeof(double));
    /* accepted positions q (relative to first), in increasing order */
    uint64_t *acc = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    int rc = (theta && summ && dist && acc) ? or_simulate(m, seed, first, n, y_obs, theta, summ,
                                                          NULL, dist, NULL)
                                            : -2;
    free(summ);
    if (rc != 0) {
        free(acc);
        free(dist);
        free(theta);
        return -2;
    }
    uint64_t count = 0;
    double eps;
    if (mode == OR_EPS_FIXED) {
        eps = eps_or_frac;
        for (uint64_t q = 0; q < n; ++q)
            if (dist[q] <= eps)
                acc[count++] = q;
    } else {
        uint64_t k = or_top_count(eps_or_frac, n);
        dist_index *order = (dist_index *)malloc((size_t)n * sizeof(dist_index));
        if (!order) {
            free(acc);
            free(dist);
            free(theta);
            return -2;
        }
        for (uint64_t q = 0; q < n; ++q) {
            order[q].d = dist[q];
            order[q].i = q;
        }
        qsort(order, (size_t)n, sizeof(dist_index), cmp_dist_index);
        eps = order[k - 1].d;
        for (uint64_t r = 0; r < k; ++r)
            acc[count++] = order[r].i;
        free(order);
        qsort(acc, (size_t)count, sizeof(uint64_t), cmp_u64);
    }

    for (uint64_t r = 0; r < count && r < capacity; ++r) {
        uint64_t q = acc[r];
        acc_idx[r] = first + q;
        for (int j = 0; j < np; ++j)
            acc_theta[r * np + j] = theta[q * np + j];
        acc_dist[r] = dist[q];
    }
    for (int j = 0; j < np; ++j) {
        double s = 0.0;
        for (uint64_t r = 0; r < count; ++r)
            s += theta[acc[r] * np + j];
        double mu = count > 0 ? s / (double)count : NAN;
        double ss = 0.0;
        for (uint64_t r = 0; r < count; ++r) {
            double d = theta[acc[r] * np + j] - mu;
            ss += d * d;
        }
        mean[j] = mu;
        var[j] = count > 1 ? ss / (double)(count - 1) : NAN;
    }
    *n_acc = count;
    *eps_used = eps;
    free(acc);
    free(dist);
    free(theta);
    return count > capacity ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Prior-predictive p-values over a hyperparameter grid (Eq. pppvhype).      */
/* ------------------------------------------------------------------------ */

/* For each lambda_k the prior of parameter `lambda_param` becomes
 * (lambda_family, a = the model's a for that parameter, b = lambda_k); the
 * other priors are unchanged.  Draw i uses the same random numbers under
 * every lambda_k (common random numbers).  count_ge[k] = #{i : T_i >= t_obs}
 * with T the mean of the observations; pvalue[k] = count_ge[k] / n.         */
int or_pvalue(const or_model *m, int lambda_param, int lambda_family, const double *lambda,
              int n_lambda, uint64_t seed, uint64_t first, uint64_t n, double t_obs,
              uint64_t *count_ge, double *pvalue)
{
    if (!model_ok(m) || m->model == OR_GARCH11 || lambda_param < 0 ||
        lambda_param >= m->n_params || n_lambda < 1 || n == 0)
        return -1;
    const int ns = or_n_summaries(m);
    int oom = 0;
    for (int k = 0; k < n_lambda; ++k) {
        or_model mk = *m;
        mk.prior[lambda_param].family = lambda_family;
        mk.prior[lambda_param].b = lambda[k];
        uint64_t count = 0;
#pragma omp parallel reduction(+ : count)
        {
            double theta[OR_MAX_PARAMS];
            double *summ = (double *)malloc((size_t)ns * sizeof(double));
            double *work = (double *)malloc(work_len(m) * sizeof(double));
            const int ok = summ && work;
            if (!ok) {
#pragma omp atomic write
                oom = 1;
            }
#pragma omp for schedule(static)
            for (int64_t q = 0; q < (int64_t)n; ++q) {
                if (!ok)
                    continue;
                uint64_t draw = first + (uint64_t)q;
                or_prior_draw(&mk, seed, draw, theta);
                simulate_summaries(&mk, theta, seed, draw, summ, work);
                if (or_mean_stat(summ, ns) >= t_obs)
                    ++count;
            }
            free(work);
            free(summ);
        }
        count_ge[k] = count;
        pvalue[k] = (double)count / (double)n;
    }
    return oom ? -2 : 0;
}

/* Per-summary tail-area tallies for a summary-vector model (the
 * prior-predictive check of the GARCH, toggle-switch and tuberculosis
 * summaries; the tail-area form of Eq. pppv per summary):
 * count_ge[s] = #{i : S_s(D_i) >= obs[s]}, the comparison inclusive.
 * Returns 0, -1 for an invalid model, -2 when a buffer cannot be allocated. */
int or_summary_tally(const or_model *m, uint64_t seed, uint64_t first, uint64_t n,
                     const double *obs_summ, uint64_t *count_ge)
{
    if (!model_ok(m))
        return -1;
    const int ns = or_n_summaries(m);
    const size_t wl = work_len(m);
    for (int s = 0; s < ns; ++s)
        count_ge[s] = 0;
    int oom = 0;
#pragma omp parallel
    {
        double theta[OR_MAX_PARAMS];
        double *summ = (double *)malloc((size_t)ns * sizeof(double));
        double *work = (double *)malloc(wl * sizeof(double));
        uint64_t *local = (uint64_t *)calloc((size_t)ns, sizeof(uint64_t));
        const int ok = summ && work && local;
        if (!ok) {
#pragma omp atomic write
            oom = 1;
        }
#pragma omp for schedule(static)
        for (int64_t q = 0; q < (int64_t)n; ++q) {
            if (!ok)
                continue;
            uint64_t draw = first + (uint64_t)q;
            or_prior_draw(m, seed, draw, theta);
            simulate_summaries(m, theta, seed, draw, summ, work);
            for (int s = 0; s < ns; ++s)
                if (summ[s] >= obs_summ[s])
                    ++local[s];
        }
#pragma omp critical
        if (ok)
            for (int s = 0; s < ns; ++s)
                count_ge[s] += local[s];
        free(local);
        free(work);
        free(summ);
    }
    return oom ? -2 : 0;
}

/* The full path of one draw at every step (for convergence checks):
 * path[n] = X after step n+1, n = 0..S-1 (logistic only).                   */
int or_logistic_path(const or_model *m, const double *theta, uint64_t seed, uint64_t draw,
                     double *path)
{
    if (m->model != OR_LOGISTIC || m->steps < 1)
        return -1;
    const double dt = m->t_end / (double)m->steps;
    const double a = theta[0] * dt;
    const double b = theta[0] * dt / theta[1];
    const double c = theta[2] * sqrt(dt);
    double x = m->x0;
    normal_reader rd;
    reader_init(&rd, seed, draw);
    for (int n = 0; n < m->steps; ++n) {
        double z = reader_next(&rd);
        x = x + x * (a - b * x + c * z);
        if (x < 0.0)
            x = 0.0;
        path[n] = x;
    }
    return 0;
}

/* The GARCH return series of one draw (for checks of the summaries).        */
int or_garch_series(const or_model *m, const double *theta, uint64_t seed, uint64_t draw,
                    double *r)
{
    if (m->model != OR_GARCH11)
        return -1;
    simulate_garch_series(m, theta, seed, draw, r);
    return 0;
}

/* Every cell of one toggle-switch draw at a given theta (for checks of the
 * dynamics, the measurement model and the quantiles): final levels u, v and
 * the measurement y of cell c, c < C, in cell order.                         */
int or_toggle_cells(const or_model *m, const double *theta, uint64_t seed, uint64_t draw,
                    double *u, double *v, double *y)
{
    if (m->model != OR_TOGGLE_SWITCH || !model_ok(m))
        return -1;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < m->n_cells; ++c)
        toggle_cell(m, theta, seed, draw, c, &u[c], &v[c], &y[c]);
    return 0;
}

/* Summaries of a given return series (exposes garch_summaries for checks).  */
void or_garch_summaries(const double *r, int len, double *s)
{
    garch_summaries(r, len, s);
}

int or_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
