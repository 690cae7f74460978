/*
 * FP64 CPU oracle for the weak-informativity test of Sec. 4.1 (Warne, Sisson &
 * Drovandi, arXiv:1902.09046): prior-predictive p-values of the evidence
 * p(D | lambda) over a family of priors, with the evidence estimated by the
 * adaptive SMC sampler of Alg. 3, on the logistic dose-response model of
 * Eq. bioassay.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against; nothing in the product path may link, load
 * or call it, and it shares no code with the HIP library.  It uses the random
 * streams of pps_oracle.c (same library).
 *
 * Readings where the paper leaves a choice open are stated at each function;
 * the design notes list them all.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from pps_oracle.c */
void or_stream_block(uint64_t seed, uint64_t draw, uint32_t block, uint32_t purpose,
                     uint32_t out[4]);
double or_uniform(uint32_t word);
void or_box_muller(uint32_t w0, uint32_t w1, double *z0, double *z1);

#define OR_BIO_MAX_GROUPS 8
#define OR_SMC_BLOCKS_PER_STEP 256 /* MCMC blocks reserved per SMC step */

/* Stream purposes of the test (counter word 1); the draw word is a data set
 * or an SMC run index.                                                       */
enum {
    OR_P_DATA_BASE = 0x40000000, /* D_0^(i) from the base prior, draw = i */
    OR_P_DATA_K = 0x40000001,    /* D_k^(i) from prior k, draw = k N + i */
    OR_P_INIT = 0x50000000,      /* + particle: initial particle, block 0 */
    OR_P_RESAMPLE = 0x60000000,  /* + particle: resampling uniform, block = step */
    OR_P_MCMC = 0x70000000       /* + particle: MCMC move, block = step 256 + r */
};

typedef struct {
    int32_t n_groups;                   /* M */
    int32_t n_trials[OR_BIO_MAX_GROUPS]; /* n_i */
    double dose[OR_BIO_MAX_GROUPS];     /* x_i */
} or_bioassay;

typedef struct {
    int32_t n_particles;  /* N_p */
    int32_t max_mcmc;     /* cap on R_n (<= 256) */
    int32_t max_steps;    /* cap on tempering steps */
    int32_t bisect_iters; /* bisection iterations for the ESS condition */
    double c;             /* R_n = ceil(ln c / ln(1 - p_acc)) */
    double h;             /* proposal scale: N(0, h^2 Sigma_hat) */
} or_smc_config;

/* Success probability of group i (Eq. bioassay): 1 / (1 + exp(b0 + b1 x_i)). */
static double bio_prob(double b0, double b1, double x)
{
    return 1.0 / (1.0 + exp(b0 + b1 * x));
}

/* D ~ p(D | lambda): theta = (lambda_1 z0, lambda_2 z1) from Box-Muller on
 * words (0, 1) of block 0; then y_i counts the trials r < n_i whose uniform is
 * below p_i, the uniforms taken in order (group by group, trial by trial) from
 * the words of blocks 1, 2, ... of the same stream.                          */
void or_bio_simulate(const or_bioassay *b, const double lambda[2], uint64_t seed, uint64_t id,
                     uint32_t purpose, int32_t *y, double theta[2])
{
    uint32_t w[4];
    or_stream_block(seed, id, 0, purpose, w);
    double z0, z1;
    or_box_muller(w[0], w[1], &z0, &z1);
    theta[0] = lambda[0] * z0;
    theta[1] = lambda[1] * z1;
    uint32_t k = 0; /* uniform index */
    for (int i = 0; i < b->n_groups; ++i) {
        const double p = bio_prob(theta[0], theta[1], b->dose[i]);
        int32_t count = 0;
        for (int r = 0; r < b->n_trials[i]; ++r, ++k) {
            if (k % 4 == 0)
                or_stream_block(seed, id, 1 + k / 4, purpose, w);
            if (or_uniform(w[k % 4]) < p)
                ++count;
        }
        y[i] = count;
    }
}

/* log L(theta; D) of Eq. bioassay: sum_i [log C(n_i, y_i) + y_i log p_i +
 * (n_i - y_i) log(1 - p_i)], written with log p_i = -log(1 + e^eta_i) and
 * log(1 - p_i) = eta_i - log(1 + e^eta_i), eta_i = b0 + b1 x_i.              */
double or_bio_loglik(const or_bioassay *b, const int32_t *y, double b0, double b1)
{
    double ll = 0.0;
    for (int i = 0; i < b->n_groups; ++i) {
        const double n = b->n_trials[i], k = y[i];
        const double eta = b0 + b1 * b->dose[i];
        const double softplus = eta > 0.0 ? eta + log1p(exp(-eta)) : log1p(exp(eta));
        ll += lgamma(n + 1.0) - lgamma(k + 1.0) - lgamma(n - k + 1.0) - k * softplus +
              (n - k) * (eta - softplus);
    }
    return ll;
}

/* log pi(theta | lambda) for theta ~ N(0, diag(lambda)^2).                   */
double or_bio_logprior(const double lambda[2], double b0, double b1)
{
    const double a = b0 / lambda[0], c = b1 / lambda[1];
    return -0.5 * (a * a + c * c) - log(6.283185307179586476925286766559 * lambda[0] * lambda[1]);
}

/* Effective sample size of the incremental weights exp(delta (l_i - l_max)). */
static double ess(const double *ll, int np, double lmax, double delta)
{
    double s = 0.0, s2 = 0.0;
    for (int i = 0; i < np; ++i) {
        const double w = exp(delta * (ll[i] - lmax));
        s += w;
        s2 += w * w;
    }
    return s * s / s2;
}

/* Tempering increment of one step (the ESS condition of Alg. 3): delta in
 * (0, 1 - t] with ESS(delta) = N_p / 2.  If the whole remaining increment
 * keeps ESS >= N_p / 2, or this is step `max_steps`, delta = 1 - t; otherwise
 * bisection on [0, 1 - t] for `bisect_iters` halvings, keeping the end with
 * ESS >= N_p / 2 (delta = that end).                                         */
double or_smc_temper(const double *ll, int np, double t, int step, const or_smc_config *cfg)
{
    double lmax = ll[0];
    for (int i = 1; i < np; ++i)
        if (ll[i] > lmax)
            lmax = ll[i];
    const double rest = 1.0 - t;
    if (step >= cfg->max_steps || ess(ll, np, lmax, rest) >= 0.5 * np)
        return rest;
    double lo = 0.0, hi = rest;
    for (int it = 0; it < cfg->bisect_iters; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ess(ll, np, lmax, mid) >= 0.5 * np)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

/* Multinomial resampling by inversion (the "look-up method"): fixed-point
 * weights q_i = floor(w_i 2^52) (w_i <= 1), running totals c_i = q_0 + ... +
 * q_i; particle i draws r = words (0, 1) of stream OR_P_RESAMPLE + i, block
 * `step` as a 64-bit integer, U = floor(r total / 2^64), and takes the first
 * ancestor a with c_a > U.  Integer arithmetic, so any summation order gives
 * the same ancestors.                                                        */
void or_smc_resample(const double *w, int np, uint64_t seed, uint64_t run, uint32_t step,
                     int32_t *ancestor)
{
    uint64_t *cum = (uint64_t *)malloc(sizeof(uint64_t) * np);
    uint64_t total = 0;
    for (int i = 0; i < np; ++i) {
        total += (uint64_t)floor(w[i] * 4503599627370496.0); /* 2^52 */
        cum[i] = total;
    }
    uint32_t words[4];
    for (int i = 0; i < np; ++i) {
        or_stream_block(seed, run, step, OR_P_RESAMPLE + (uint32_t)i, words);
        const uint64_t r64 = ((uint64_t)words[1] << 32) | words[0];
        const uint64_t u = (uint64_t)(((unsigned __int128)r64 * total) >> 64);
        int a = 0;
        while (cum[a] <= u)
            ++a;
        ancestor[i] = a;
    }
    free(cum);
}

/* MCMC moves of a step from the trial acceptance rate p = accepted / N_p:
 * R = ceil(ln c / ln(1 - p)) clamped to [1, max_mcmc]; p = 0 (no trial move
 * accepted) gives max_mcmc and p = 1 gives 1 (the limits of the formula).   */
int or_smc_moves(int accepted, int np, const or_smc_config *cfg)
{
    if (accepted <= 0)
        return cfg->max_mcmc;
    if (accepted >= np)
        return 1;
    const double p_acc = (double)accepted / np;
    const double rn = ceil(log(cfg->c) / log(1.0 - p_acc));
    if (rn < 1.0)
        return 1;
    return rn > cfg->max_mcmc ? cfg->max_mcmc : (int)rn;
}

/* Lower Cholesky factor (l11, l21, l22) of h^2 Sigma_hat, Sigma_hat the sample
 * covariance (divisor N_p - 1) of the particles; a zero variance gives a zero
 * column.                                                                    */
void or_smc_proposal(const double *b0, const double *b1, int np, double h, double l[3])
{
    double m0 = 0.0, m1 = 0.0;
    for (int i = 0; i < np; ++i) {
        m0 += b0[i];
        m1 += b1[i];
    }
    m0 /= np;
    m1 /= np;
    double s00 = 0.0, s01 = 0.0, s11 = 0.0;
    for (int i = 0; i < np; ++i) {
        const double d0 = b0[i] - m0, d1 = b1[i] - m1;
        s00 += d0 * d0;
        s01 += d0 * d1;
        s11 += d1 * d1;
    }
    s00 /= (np - 1);
    s01 /= (np - 1);
    s11 /= (np - 1);
    const double h2 = h * h;
    l[0] = s00 > 0.0 ? sqrt(h2 * s00) : 0.0;
    l[1] = s00 > 0.0 ? h2 * s01 / l[0] : 0.0;
    const double r22 = h2 * s11 - l[1] * l[1];
    l[2] = r22 > 0.0 ? sqrt(r22) : 0.0;
}

/* The adaptive SMC sampler of Alg. 3 for log p(D | lambda), in its steps:
 *   init: particles from the prior (OR_P_INIT + i, block 0, Box-Muller), equal
 *     weights, t = 0, log Z = 0;
 *   repeat (step n = 1, 2, ...):
 *     tempering: delta from or_smc_temper;
 *     evidence: log Z += log((1/N_p) sum_i L_i^delta) (equal weights before
 *       the step, as after every resampling), evaluated as delta l_max +
 *       log((1/N_p) sum_i exp(delta (l_i - l_max)));
 *     multinomial resampling (or_smc_resample) with those weights;
 *     proposal N(0, h^2 Sigma_hat) of the resampled particles
 *       (or_smc_proposal);
 *     MCMC: one trial Metropolis-Hastings move of every particle gives
 *       p_acc = accepted / N_p; R_n = ceil(ln c / ln(1 - p_acc)) clamped to
 *       [1, max_mcmc] moves in all (the trial counts as the first).  Move r of
 *       particle i uses OR_P_MCMC + i, block n 256 + r: words (0, 1) for the
 *       two proposal normals, word 2 for the acceptance uniform; accept if
 *       log u < t (l* - l) + log pi(theta*) - log pi(theta) (the random-walk
 *       kernel is symmetric);
 *   until t = 1.
 * Returns log Z; *n_steps = the number of tempering steps.                   */
double or_smc_log_evidence(const or_bioassay *b, const int32_t *y, const double lambda[2],
                           const or_smc_config *cfg, uint64_t seed, uint64_t run,
                           int32_t *n_steps, double *trace /* optional: 4 per step */)
{
    const int np = cfg->n_particles;
    double *b0 = (double *)malloc(sizeof(double) * np);
    double *b1 = (double *)malloc(sizeof(double) * np);
    double *ll = (double *)malloc(sizeof(double) * np);
    double *nb0 = (double *)malloc(sizeof(double) * np);
    double *nb1 = (double *)malloc(sizeof(double) * np);
    double *nll = (double *)malloc(sizeof(double) * np);
    double *wts = (double *)malloc(sizeof(double) * np);
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * np);
    uint32_t w[4];
    for (int i = 0; i < np; ++i) {
        double z0, z1;
        or_stream_block(seed, run, 0, OR_P_INIT + (uint32_t)i, w);
        or_box_muller(w[0], w[1], &z0, &z1);
        b0[i] = lambda[0] * z0;
        b1[i] = lambda[1] * z1;
        ll[i] = or_bio_loglik(b, y, b0[i], b1[i]);
    }
    double t = 0.0, log_z = 0.0;
    int n = 0;
    while (t < 1.0) {
        ++n;
        const double delta = or_smc_temper(ll, np, t, n, cfg);
        const double rest = 1.0 - t;
        double lmax = ll[0];
        for (int i = 1; i < np; ++i)
            if (ll[i] > lmax)
                lmax = ll[i];
        /* incremental weights and the evidence factor */
        double sum_w = 0.0;
        for (int i = 0; i < np; ++i) {
            wts[i] = exp(delta * (ll[i] - lmax));
            sum_w += wts[i];
        }
        log_z += delta * lmax + log(sum_w / np);
        t = (delta == rest) ? 1.0 : t + delta;
        /* multinomial resampling */
        or_smc_resample(wts, np, seed, run, (uint32_t)n, anc);
        for (int i = 0; i < np; ++i) {
            nb0[i] = b0[anc[i]];
            nb1[i] = b1[anc[i]];
            nll[i] = ll[anc[i]];
        }
        memcpy(b0, nb0, sizeof(double) * np);
        memcpy(b1, nb1, sizeof(double) * np);
        memcpy(ll, nll, sizeof(double) * np);
        /* proposal covariance h^2 Sigma_hat and its Cholesky factor */
        double lf[3];
        or_smc_proposal(b0, b1, np, cfg->h, lf);
        const double l11 = lf[0], l21 = lf[1], l22 = lf[2];
        /* MCMC moves targeting L^t pi(theta | lambda) */
        int accepted = 0, moves = 1;
        for (int r = 0; r < moves; ++r) {
            int acc_r = 0;
            for (int i = 0; i < np; ++i) {
                or_stream_block(seed, run, (uint32_t)(n * OR_SMC_BLOCKS_PER_STEP + r),
                                OR_P_MCMC + (uint32_t)i, w);
                double z0, z1;
                or_box_muller(w[0], w[1], &z0, &z1);
                const double p0 = b0[i] + l11 * z0;
                const double p1 = b1[i] + l21 * z0 + l22 * z1;
                const double pll = or_bio_loglik(b, y, p0, p1);
                const double log_alpha = t * (pll - ll[i]) + or_bio_logprior(lambda, p0, p1) -
                                         or_bio_logprior(lambda, b0[i], b1[i]);
                if (log(or_uniform(w[2])) < log_alpha) {
                    b0[i] = p0;
                    b1[i] = p1;
                    ll[i] = pll;
                    ++acc_r;
                }
            }
            if (r == 0) {
                accepted = acc_r;
                moves = or_smc_moves(accepted, np, cfg);
            }
        }
        if (trace) {
            trace[4 * (n - 1) + 0] = t;
            trace[4 * (n - 1) + 1] = delta;
            trace[4 * (n - 1) + 2] = (double)accepted / np;
            trace[4 * (n - 1) + 3] = moves;
        }
    }
    if (n_steps)
        *n_steps = n;
    free(b0); free(b1); free(ll); free(nb0); free(nb1); free(nll); free(wts); free(anc);
    return log_z;
}

/* The weak-informativity test of Alg. 2 for hyperparameters lambda_0 (row 0,
 * the base prior) .. lambda_K (rows 1..K of `lambdas`, 2 values each):
 *   D_0^(i) ~ p(D | lambda_0), i < N, stream (OR_P_DATA_BASE, draw i), shared
 *     by every k (reading: the listing regenerates them inside its k loop; one
 *     set of base data sets serves every k here);
 *   D_k^(i) ~ p(D | lambda_k), stream (OR_P_DATA_K, draw k N + i);
 *   log pi_0^i = log p(D_0^(i) | lambda_k) and log pi_k^i = log p(D_k^(i) |
 *     lambda_k) by Alg. 3, SMC run index (k N + i) 2 + 0 and (k N + i) 2 + 1;
 *   p_k^i = (1/N) #{j : pi_k^j <= pi_0^i};
 *   gamma_k = the alpha quantile of {p_k^i}: the ceil(alpha N)-th smallest.
 * log_z0, log_zk: n_lambda x N (row k); pvals: n_lambda x N; gamma: n_lambda.
 * The SMC runs are spread over threads (static partition).                  */
int or_wip_test(const or_bioassay *b, const double *lambdas, int n_lambda, uint64_t n_data,
                const or_smc_config *cfg, uint64_t seed, double alpha, double *log_z0,
                double *log_zk, double *pvals, double *gamma)
{
    if (b->n_groups < 1 || b->n_groups > OR_BIO_MAX_GROUPS || n_lambda < 1 || n_data < 1 ||
        cfg->n_particles < 2 || cfg->max_mcmc < 1 || cfg->max_mcmc > OR_SMC_BLOCKS_PER_STEP)
        return -1;
    const int m = b->n_groups;
    int32_t *y0 = (int32_t *)malloc(sizeof(int32_t) * m * n_data);
    int32_t *yk = (int32_t *)malloc(sizeof(int32_t) * m * n_data * n_lambda);
    double th[2];
    for (uint64_t i = 0; i < n_data; ++i)
        or_bio_simulate(b, &lambdas[0], seed, i, OR_P_DATA_BASE, &y0[i * m], th);
    for (int k = 0; k < n_lambda; ++k)
        for (uint64_t i = 0; i < n_data; ++i)
            or_bio_simulate(b, &lambdas[2 * k], seed, k * n_data + i, OR_P_DATA_K,
                            &yk[(k * n_data + i) * m], th);
    const int64_t runs = 2 * (int64_t)n_lambda * (int64_t)n_data;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < runs; ++r) {
        const int64_t ki = r / 2;
        const int kind = (int)(r % 2);
        const int k = (int)(ki / (int64_t)n_data);
        const uint64_t i = (uint64_t)(ki % (int64_t)n_data);
        const int32_t *y = kind == 0 ? &y0[i * m] : &yk[(k * n_data + i) * m];
        const double lz = or_smc_log_evidence(b, y, &lambdas[2 * k], cfg, seed, (uint64_t)r, NULL,
                                              NULL);
        if (kind == 0)
            log_z0[k * n_data + i] = lz;
        else
            log_zk[k * n_data + i] = lz;
    }
    const uint64_t rank = (uint64_t)ceil(alpha * (double)n_data);
    const uint64_t q = rank < 1 ? 1 : (rank > n_data ? n_data : rank);
    double *sorted = (double *)malloc(sizeof(double) * n_data);
    for (int k = 0; k < n_lambda; ++k) {
        for (uint64_t i = 0; i < n_data; ++i) {
            uint64_t count = 0;
            for (uint64_t j = 0; j < n_data; ++j)
                if (log_zk[k * n_data + j] <= log_z0[k * n_data + i])
                    ++count;
            pvals[k * n_data + i] = (double)count / (double)n_data;
            sorted[i] = pvals[k * n_data + i];
        }
        /* the q-th smallest p-value (selection by repeated minimum, plain) */
        for (uint64_t a = 0; a < q; ++a) {
            uint64_t best = a;
            for (uint64_t j = a + 1; j < n_data; ++j)
                if (sorted[j] < sorted[best])
                    best = j;
            const double tmp = sorted[a];
            sorted[a] = sorted[best];
            sorted[best] = tmp;
        }
        gamma[k] = sorted[q - 1];
    }
    free(sorted);
    free(y0);
    free(yk);
    return 0;
}
