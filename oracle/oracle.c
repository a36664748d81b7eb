/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY: the plain FP64 CPU sampler.  Only the
 * tests, the package's smoke check and the benchmark's CPU-baseline leg load
 * it; the HIP library never does.
 *
 * Landau & Niemi, "A fully Bayesian strategy for high-dimensional hierarchical
 * modeling using massively parallel computing" (arXiv 1606.06659).
 *   Model:         Section 4.1, Fig. 3.
 *   Gibbs scan:    Algorithm 1 and Section 4.2 (the order of the conditionals).
 *   Slice draws:   Algorithm 2 (Appendix A), Neal's stepping-out slice sampler,
 *                  in log space.
 *   Moments:       Section 3.1 (one-pass running mean and mean of squares).
 *
 * Everything is written the plain way: each log density is the full conditional
 * evaluated term by term (sums over all n, no grouping), each reduction is a
 * serial loop, and the conditionals are drawn in the order of Algorithm 1:
 * eps (all g, n), gamma (all g), nu, tau, beta (l = 1..L), theta, sigma^2.
 *
 * Readings where the paper is silent or garbled (each is also listed in the
 * design notes of the repository):
 *  - nu: the printed conditional carries nu/gamma_g inside the sum; the
 *    product of InvGamma(nu/2, nu tau/2) densities gives tau/gamma_g, which is
 *    used here, together with the U(0, d) support.
 *  - gamma_g: InvGamma(nu/2 + N/2, nu tau/2 + sum_n eps_gn^2 / 2) (scale form).
 *  - theta_l: Normal full conditional drawn directly (only non-normal
 *    conditionals are slice sampled, Section 4.2).
 *  - sigma_l: the prior is uniform on sigma_l, so sigma_l^2 has the truncated
 *    InvGamma((G-1)/2, sum_g (beta_gl - theta_l)^2 / 2) conditional on
 *    (0, s_l^2); it is slice sampled and sigma_l^2 is what is stored.
 *  - tau: its Gamma conditional is slice sampled like the other gamma-family
 *    conditionals (Section 4.2).
 *  - Growing the slice interval: the printed loop keeps testing after the first
 *    end outside the slice; stopping there gives the same interval and is what
 *    is done here.
 *  - The trial-point loop is capped at shrink_cap points; on the cap the draw
 *    keeps x0 and an error is counted.
 *  - Width adaptation uses the sweep index m, and a computed width that is not
 *    a positive finite number leaves w unchanged.
 *  - Moments cover sweeps m > M_B with divisor m - M_B.
 */
#include "oracle.h"

/* OR_MUTANT selects a deliberately wrong variant of one formula.  Mutant
 * libraries are built only by the tests, to show that each pin fails on a
 * plausible mistake; the default build (OR_MUTANT = 0) is the oracle. */
#ifndef OR_MUTANT
#define OR_MUTANT 0
#endif

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11)                  */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double u01(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }

/* The random words of one draw: a lazily extended Philox stream. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];     /* block index lives in the low 16 bits of ctr[3] */
    uint32_t block;      /* block currently in buf */
    uint32_t buf[4];
} rstream;

static void rs_init(rstream *s, uint64_t seed, uint32_t g, uint32_t kind, uint32_t sub,
                    uint32_t m, uint32_t chain)
{
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    s->ctr[0] = g;
    s->ctr[1] = (kind << 24) | sub;
    s->ctr[2] = m;
    s->ctr[3] = chain << 16;
    s->block = 0;
    or_philox4x32_10(s->ctr, s->key, s->buf);
}

static uint32_t rs_word(rstream *s, uint32_t q)
{
    uint32_t blk = q >> 2;
    if (blk != s->block) {
        uint32_t c[4] = { s->ctr[0], s->ctr[1], s->ctr[2], (s->ctr[3] & 0xFFFF0000u) | blk };
        or_philox4x32_10(c, s->key, s->buf);
        s->block = blk;
    }
    return s->buf[q & 3];
}

/* ------------------------------------------------------------------ */
/* Univariate slice sampling with a stepped-out interval               */
/* ------------------------------------------------------------------ */
/* The paper draws every conditional that is not normal with the univariate
 * slice sampler of Neal (2003, Ann. Statist. 31, Sections 4.1-4.2) in the
 * form of Algorithm 2 (Appendix A), including its adaptive width.  From the
 * current point x0:
 *   - an auxiliary level below f(x0) defines the slice {x : f(x) > level};
 *     in log space the level is z = log f(x0) - E with E ~ Exp(1), which is
 *     log of a uniform draw on (0, f(x0)) and cannot underflow;
 *   - an interval of width w is placed uniformly at random around x0 and
 *     grown by whole widths while its end lies in the slice, with a budget of
 *     K growth steps split uniformly at random between the two sides;
 *   - points drawn uniformly from the interval are tried until one lies in
 *     the slice; a rejected point becomes the end of the interval on its side
 *     of x0 (a point equal to x0 counts as the left side).
 * The result leaves f invariant for any fixed w (Neal 2003, Section 4.3).
 * During burn-in w adapts to the mean absolute move (see adapt_width).
 *
 * Random words (layout in oracle.h): word 0 gives E, word 1 the side budget
 * (low 4 bits) and the interval offset (high 28 bits), word t + 1 the t-th
 * trial point. */
typedef double (*logf_fn)(double x, const void *arg);

typedef struct {
    int32_t kl, nl, nr, nc;  /* left budget, left and right growth steps, trial points */
    double margin;           /* smallest |log f(x) - z| over the comparisons */
    int bad;                 /* non-finite log f(x0), or no point found */
} draw_info;

static void note_margin(draw_info *di, double fx, double z)
{
    double d = fabs(fx - z);
    if (isnan(d)) d = INFINITY;
    if (d < di->margin) di->margin = d;
}

/* Grows one end of the interval: while fewer than `budget` moves have been
 * made and the end is inside the slice, move it by `step`.  Returns the
 * number of moves; the loop ends at the first end outside the slice (further
 * tests could not move it any more). */
static int grow_end(logf_fn f, const void *arg, double z, double step, int budget, double *end, draw_info *di)
{
    int moves = 0;
    for (; moves < budget; ++moves) {
        const double fe = f(*end, arg);
        note_margin(di, fe, z);
        if (!(fe > z)) break;
        *end += step;
    }
    return moves;
}

/* Burn-in adaptation of the width (Appendix A): waux accumulates m |x1 - x0|
 * from the first sweep; once m > M_C the width becomes the weighted mean
 * waux / (m (m + 1) / 2).  A value that is not a positive finite number
 * leaves w as it is.  After burn-in w is frozen. */
static void adapt_width(double *w, double *waux, double x0, double x1, int64_t m, int64_t burnin,
                        int64_t tune_start)
{
    if (m > burnin) return;
    *waux += (double)m * fabs(x1 - x0);
    if (m > tune_start) {
        const double wn = *waux / (0.5 * (double)m * (double)(m + 1));
        if (wn > 0.0 && isfinite(wn)) *w = wn;
    }
}

static double slice_draw(logf_fn f, const void *arg, double x0, double *w, double *waux,
                         int64_t m, int64_t burnin, int64_t tune_start, int K, int cap,
                         rstream *rs, draw_info *di)
{
    di->margin = INFINITY;
    di->bad = 0;
    di->kl = di->nl = di->nr = di->nc = 0;
    const double fx0 = f(x0, arg);
    if (!isfinite(fx0)) { di->bad = 1; return x0; }
    const double z = fx0 - (-log(u01(rs_word(rs, 0))));
    /* the interval [lo, hi] of width w with x0 at a uniform offset from hi */
    const uint32_t r1 = rs_word(rs, 1);
    double off = (*w) * (((double)(r1 >> 4) + 0.5) * 0x1p-28);
    if (OR_MUTANT == 4) off = *w;           /* interval not placed at random */
    double lo = x0 - off;
    double hi = lo + (*w);
    /* the growth budget: kl steps to the left, K - kl to the right */
    di->kl = (int)(r1 & (uint32_t)K);
    di->nl = grow_end(f, arg, z, -(*w), di->kl, &lo, di);
    di->nr = grow_end(f, arg, z, *w, K - di->kl, &hi, di);
    /* uniform trial points, each rejection cutting the interval at the point */
    double x1 = x0;
    int found = 0;
    for (int t = 1; t <= cap && !found; ++t) {
        const double xt = lo + u01(rs_word(rs, (uint32_t)(t + 1))) * (hi - lo);
        const double ft = f(xt, arg);
        note_margin(di, ft, z);
        di->nc = t;
        if (ft > z) { x1 = xt; found = 1; }
        else if (xt > x0) hi = xt;
        else lo = xt;
    }
    if (!found) di->bad = 1;
    adapt_width(w, waux, x0, x1, m, burnin, tune_start);
    return x1;
}

/* ------------------------------------------------------------------ */
/* Exact conjugate draws (bit OR_KIND_EXACT of update_mask)            */
/* ------------------------------------------------------------------ */
/* Section 4.2 slice-samples the gamma and inverse-gamma conditionals only
 * because the paper's GPU library had no gamma generator, and names a
 * gamma sampler as the alternative.  This option draws them directly:
 *   gamma_g    = B / X,  X ~ Gamma(alpha),  alpha = nu/2 + N/2, B = nu tau/2 + S_g/2
 *   tau        = X / R,  X ~ Gamma(alpha),  alpha = a + G nu/2, R = b + (nu/2) sum 1/gamma
 *   sigma_l^2  = B / X,  X ~ Gamma(alpha),  alpha = (G-1)/2,    B = S_l/2,
 *                kept only when below s_l^2 (the truncation of its prior).
 * Gamma(alpha, 1) variates come from the method of Marsaglia and Tsang (ACM
 * TOMS 26(3), 2000): for alpha >= 1 put d = alpha - 1/3, c = 1/sqrt(9 d); a
 * standard normal x gives v = (1 + c x)^3, and d v is a variate when v > 0
 * and log u < x^2/2 + d - d v + d log v for a uniform u.  For alpha < 1 the
 * variate for alpha + 1 times U^(1/alpha) is one for alpha.
 * Random numbers: Philox counter (g, 12 << 24 | sub, m, chain << 16 | t) for
 * attempt t = 0, 1, ...: words 0 and 1 give x by Box-Muller, word 2 gives u,
 * word 3 the U of alpha < 1; sub = 0 for gamma_g, 1 for tau, 2 + l for
 * sigma_l^2.  An attempt fails when its candidate is rejected or falls outside
 * the support.  After OR_EXACT_TRIES failed attempts, or when alpha <= 0, the
 * parameter takes the slice draw of Algorithm 2 instead; whether that happens
 * does not depend on the parameter's current value, so the update remains a
 * mixture of two kernels that both leave the conditional invariant. */
#define OR_EXACT_TRIES 64

typedef struct {
    double alpha;    /* shape of the gamma variate X */
    double q;        /* B of an inverse gamma (value q / X) or R of a gamma (value X / q) */
    int inverse;     /* 1: value q / X, 0: value X / q */
    double upper;    /* values must lie below this bound (INFINITY: none) */
} exact_arg;

/* Returns the number of attempts used (1..OR_EXACT_TRIES) with *out set, or
 * 0 when no attempt succeeded.  di->margin gets the smallest gap of any
 * decision taken (the acceptance test in log space, the truncation on the
 * log scale). */
static int exact_draw(const exact_arg *e, uint64_t seed, uint32_t kind, uint32_t g, uint32_t sub, uint32_t m,
                      uint32_t chain, double *out, draw_info *di)
{
    di->margin = INFINITY;
    di->bad = 0;
    if (!(e->alpha > 0.0)) return 0;
    const int boost = e->alpha < 1.0;
    const double ab = boost ? e->alpha + 1.0 : e->alpha;
    const double d = (OR_MUTANT == 13 ? ab - 0.5 : ab - 1.0 / 3.0);
    const double c = 1.0 / sqrt(9.0 * d);
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int t = 0; t < OR_EXACT_TRIES; ++t) {
        const uint32_t ctr[4] = { g, (kind << 24) | sub, m, (chain << 16) | (uint32_t)t };
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        const double x = sqrt(-2.0 * log(u01(r[0]))) * cos(2.0 * M_PI * u01(r[1]));
        const double s = 1.0 + c * x;
        if (!(s > 0.0)) continue;
        const double v = s * s * s;
        const double lu = log(u01(r[2]));
        const double rhs = 0.5 * x * x + d - d * v + d * log(v);
        note_margin(di, lu, rhs);
        if (!(lu < rhs)) continue;
        double X = d * v;
        if (boost) X *= exp(log(u01(r[3])) / (OR_MUTANT == 14 ? ab : e->alpha));
        const double val = e->inverse ? e->q / X : X / e->q;
        if (!(val > 0.0) || !isfinite(val)) continue;
        if (isfinite(e->upper)) {
            note_margin(di, log(val), log(e->upper));
            if (!(val < e->upper)) continue;
        }
        *out = val;
        return t + 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Context                                                             */
/* ------------------------------------------------------------------ */
struct or_ctx {
    or_config cfg;
    int32_t *y;            /* [G][N] */
    double *X, *h, *c, *s; /* copies */
    /* state */
    double *eps, *gam, *beta;      /* [G][N], [G], [G][L] */
    double nu, tau, *theta, *sig2; /* [L], [L] */
    double *w_eps, *wa_eps, *w_gam, *wa_gam, *w_beta, *wa_beta;
    double w_nu, wa_nu, w_tau, wa_tau, *w_sig2, *wa_sig2;
    int64_t m;
    /* moments over parameters in the order eps, gamma, beta, hyp */
    double *mean, *msq;
    int64_t count;
    /* last-sweep records */
    int32_t *cnt;          /* 4 per slice draw, same order (hyp: nu, tau, sig2) */
    double *mrg;
    int64_t errors;
    double red[2 + 2 * 64];
    int nthreads;
    /* distinct rows of X in order of first appearance (features of the proposal) */
    int R;
    int *row_of;           /* [N] */
    /* learned beta proposal: owned copy of the model, fallback mask, records */
    int prop_on;
    or_mlp prop;
    double *prop_buf;
    int32_t *prop_mask;    /* [G]: 1 = slice fallback */
    int32_t *imh_acc;      /* [G]: last sweep, 1 = accepted, 0 = rejected, -1 = slice */
    double *imh_la;        /* [G]: log acceptance ratio of the last IMH step */
    /* posterior probabilities of contrast events (Section 3.2): event e is the
     * conjunction of the rows r with crow_event[r] == e, row r the inequality
     * sum_l cv[r][l] beta_gl > cb[r]; ev_count[g][e] counts the sweeps
     * m > max(M_B, ev_from) whose end-of-sweep beta_g satisfies event e */
    int n_ev, n_crow;
    int32_t *crow_event;
    double *cv, *cb;
    int64_t *ev_count;
    int64_t ev_from;
    /* prior mean of theta_l (0 unless a three-level driver sets it) */
    double theta_mean[OR_MAX_L];
};

static int64_t n_params(const or_ctx *c)
{
    int64_t G = c->cfg.G, N = c->cfg.N, L = c->cfg.L;
    return G * N + G + G * L + 2 + 2 * L;
}

static int64_t n_slice(const or_ctx *c)
{
    int64_t G = c->cfg.G, N = c->cfg.N, L = c->cfg.L;
    return G * N + G + G * L + 2 + L;
}

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

int or_create(or_ctx **out, const or_config *cfg)
{
    if (!out || !cfg) return -1;
    *out = NULL;
    if (cfg->G < 1 || cfg->N < 1 || cfg->L < 1 || cfg->L > OR_MAX_L) return -1;
    if (!(cfg->K == 0 || cfg->K == 1 || cfg->K == 3 || cfg->K == 7 || cfg->K == 15)) return -1;
    if (cfg->shrink_cap < 1) return -1;
    or_ctx *c = (or_ctx *)xcalloc(1, sizeof(or_ctx));
    if (!c) return -2;
    c->cfg = *cfg;
    int64_t G = cfg->G, N = cfg->N, L = cfg->L;
    c->y = (int32_t *)xcalloc((size_t)(G * N), sizeof(int32_t));
    c->X = (double *)xcalloc((size_t)(N * L), sizeof(double));
    c->h = (double *)xcalloc((size_t)N, sizeof(double));
    c->c = (double *)xcalloc((size_t)L, sizeof(double));
    c->s = (double *)xcalloc((size_t)L, sizeof(double));
    memcpy(c->y, cfg->y, sizeof(int32_t) * (size_t)(G * N));
    memcpy(c->X, cfg->X, sizeof(double) * (size_t)(N * L));
    memcpy(c->h, cfg->h, sizeof(double) * (size_t)N);
    memcpy(c->c, cfg->c, sizeof(double) * (size_t)L);
    memcpy(c->s, cfg->s, sizeof(double) * (size_t)L);
    c->cfg.y = c->y; c->cfg.X = c->X; c->cfg.h = c->h; c->cfg.c = c->c; c->cfg.s = c->s;
    c->eps = (double *)xcalloc((size_t)(G * N), sizeof(double));
    c->gam = (double *)xcalloc((size_t)G, sizeof(double));
    c->beta = (double *)xcalloc((size_t)(G * L), sizeof(double));
    c->theta = (double *)xcalloc((size_t)L, sizeof(double));
    c->sig2 = (double *)xcalloc((size_t)L, sizeof(double));
    c->w_eps = (double *)xcalloc((size_t)(G * N), sizeof(double));
    c->wa_eps = (double *)xcalloc((size_t)(G * N), sizeof(double));
    c->w_gam = (double *)xcalloc((size_t)G, sizeof(double));
    c->wa_gam = (double *)xcalloc((size_t)G, sizeof(double));
    c->w_beta = (double *)xcalloc((size_t)(G * L), sizeof(double));
    c->wa_beta = (double *)xcalloc((size_t)(G * L), sizeof(double));
    c->w_sig2 = (double *)xcalloc((size_t)L, sizeof(double));
    c->wa_sig2 = (double *)xcalloc((size_t)L, sizeof(double));
    c->mean = (double *)xcalloc((size_t)n_params(c), sizeof(double));
    c->msq = (double *)xcalloc((size_t)n_params(c), sizeof(double));
    c->cnt = (int32_t *)xcalloc((size_t)(4 * n_slice(c)), sizeof(int32_t));
    c->mrg = (double *)xcalloc((size_t)n_slice(c), sizeof(double));
    c->nthreads = 1;
    c->row_of = (int *)xcalloc((size_t)N, sizeof(int));
    c->prop_mask = (int32_t *)xcalloc((size_t)G, sizeof(int32_t));
    c->imh_acc = (int32_t *)xcalloc((size_t)G, sizeof(int32_t));
    c->imh_la = (double *)xcalloc((size_t)G, sizeof(double));
    if (!c->y || !c->eps || !c->mean || !c->msq || !c->cnt || !c->mrg || !c->row_of || !c->prop_mask ||
        !c->imh_acc || !c->imh_la) { or_destroy(c); return -2; }
    /* rows of X that are equal entry by entry share a row index */
    c->R = 0;
    for (int n = 0; n < N; ++n) {
        int found = -1;
        for (int q = 0; q < n && found < 0; ++q) {
            int same = 1;
            for (int l = 0; l < L; ++l) if (c->X[q * L + l] != c->X[n * L + l]) { same = 0; break; }
            if (same) found = c->row_of[q];
        }
        c->row_of[n] = found >= 0 ? found : c->R++;
    }
    if (c->R > OR_MAX_ROWS) { or_destroy(c); return -1; }
    for (int64_t i = 0; i < G * N; ++i) c->w_eps[i] = cfg->w0;
    for (int64_t i = 0; i < G; ++i) c->w_gam[i] = cfg->w0;
    for (int64_t i = 0; i < G * L; ++i) c->w_beta[i] = cfg->w0;
    for (int64_t l = 0; l < L; ++l) c->w_sig2[l] = cfg->w0;
    c->w_nu = cfg->w0;
    c->w_tau = cfg->w0;
    *out = c;
    return 0;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    free(c->y); free(c->X); free(c->h); free(c->c); free(c->s);
    free(c->eps); free(c->gam); free(c->beta); free(c->theta); free(c->sig2);
    free(c->w_eps); free(c->wa_eps); free(c->w_gam); free(c->wa_gam);
    free(c->w_beta); free(c->wa_beta); free(c->w_sig2); free(c->wa_sig2);
    free(c->mean); free(c->msq); free(c->cnt); free(c->mrg);
    free(c->row_of); free(c->prop_buf); free(c->prop_mask); free(c->imh_acc); free(c->imh_la);
    free(c->crow_event); free(c->cv); free(c->cb); free(c->ev_count);
    free(c);
}

int or_set_counts(or_ctx *c, const int32_t *y)
{
    if (!c || !y) return -1;
    memcpy(c->y, y, sizeof(int32_t) * (size_t)c->cfg.G * (size_t)c->cfg.N);
    return 0;
}

int or_set_update_mask(or_ctx *c, uint32_t mask) { if (!c) return -1; c->cfg.update_mask = mask; return 0; }

int or_set_top_priors(or_ctx *c, double b, const double *theta_mean)
{
    if (!c || !(b > 0.0) || !theta_mean) return -1;
    c->cfg.b = b;
    for (int l = 0; l < c->cfg.L; ++l) c->theta_mean[l] = theta_mean[l];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Three-level form (Section 2.3): the top-level draws                 */
/* ------------------------------------------------------------------ */
/* Groups k = 1..K are copies of the model of Section 4.1 with their own
 * hyperparameters phi_k = (nu_k, tau_k, theta_k, sigma_k^2), tied through
 * psi = (b, psi_1..psi_L):  tau_k ~ Gamma(a_k, rate b), theta_kl ~ N(psi_l,
 * c_kl^2), with b ~ Gamma(a_b, rate b_b) and psi_l ~ N(0, c0_l^2).  Given phi
 * the top level is independent of the genes, and its full conditionals are
 * conjugate (a reduction over the groups each):
 *   b     ~ Gamma(a_b + sum_k a_k, rate b_b + sum_k tau_k)
 *   psi_l ~ N(v_l sum_k theta_kl / c_kl^2, v_l),  v_l = 1 / (1/c0_l^2 + sum_k 1/c_kl^2)
 * Random numbers: Philox counter (0, 13 << 24 | sub, m, chain << 16 | j);
 * psi_l: sub = l, block 0, Box-Muller on words 0 and 1; b: sub = 128, the
 * gamma variate of exact_draw (attempt j in block j); if every attempt fails
 * b keeps its value (a state-independent identity step).  mask bit 0 draws
 * b, bit 1 the psi_l.  Sums run over k in order. */
int or_top_draw(int32_t K, int32_t L, const double *theta, const double *tau, const double *a, const double *c,
                double a_b, double b_b, const double *c0, uint64_t seed, int32_t chain, int64_t m, uint32_t mask,
                double *b, double *psi, int32_t *tries)
{
    if (K < 1 || L < 1 || L > OR_MAX_L || !theta || !tau || !a || !c || !c0 || !b || !psi) return -1;
    const uint32_t mm = (uint32_t)m;
    if (tries) *tries = 0;
    if (mask & 1u) {
        double sa = 0.0, st = 0.0;
        for (int k = 0; k < K; ++k) { sa += a[k]; st += tau[k]; }
        exact_arg e = { a_b + sa, OR_MUTANT == 18 ? st : b_b + st, 0, INFINITY };
        draw_info di;
        double v;
        int t = exact_draw(&e, seed, OR_KIND_TOP, 0, 128u, mm, (uint32_t)chain, &v, &di);
        if (t > 0) *b = v;
        if (tries) *tries = t;
    }
    if (mask & 2u) {
        const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
        for (int l = 0; l < L; ++l) {
            double prec = OR_MUTANT == 17 ? 0.0 : 1.0 / (c0[l] * c0[l]);
            double sw = 0.0;
            for (int k = 0; k < K; ++k) {
                const double ckl = c[k * L + l];
                prec += 1.0 / (ckl * ckl);
                sw += theta[k * L + l] / (ckl * ckl);
            }
            const double mean = sw / prec;
            const uint32_t ctr[4] = { 0, ((uint32_t)OR_KIND_TOP << 24) | (uint32_t)l, mm, (uint32_t)chain << 16 };
            uint32_t r[4];
            or_philox4x32_10(ctr, key, r);
            const double zn = sqrt(-2.0 * log(u01(r[0]))) * cos(2.0 * M_PI * u01(r[1]));
            psi[l] = mean + zn / sqrt(prec);
        }
    }
    return 0;
}

int or_set_threads(or_ctx *c, int32_t nthreads)
{
    if (!c || nthreads < 1) return -1;
    c->nthreads = nthreads;
    return 0;
}

int64_t or_error_count(const or_ctx *c) { return c ? c->errors : -1; }

/* ------------------------------------------------------------------ */
/* Full conditionals (log densities up to a constant)                  */
/* ------------------------------------------------------------------ */
typedef struct { const or_ctx *c; int64_t g; int n; } eps_arg;

/* eps_gn: y_gn eps - exp(h_n + eps + X_n beta_g) - eps^2 / (2 gamma_g) */
static double logf_eps(double x, const void *p)
{
    const eps_arg *a = (const eps_arg *)p;
    const or_ctx *c = a->c;
    int L = c->cfg.L, N = c->cfg.N;
    double eta = c->h[a->n];
    for (int l = 0; l < L; ++l) eta += c->X[a->n * L + l] * c->beta[a->g * L + l];
    double y = (double)c->y[a->g * N + a->n];
    if (OR_MUTANT == 6) return y * x - exp(eta - x) - x * x / (2.0 * c->gam[a->g]);
    return y * x - exp(eta + x) - x * x / (2.0 * c->gam[a->g]);
}

typedef struct { double alpha1, scale; } gam_arg;   /* alpha + 1, scale */

/* gamma_g: InvGamma(nu/2 + N/2, nu tau/2 + S_g/2) */
static double logf_gam(double x, const void *p)
{
    const gam_arg *a = (const gam_arg *)p;
    if (!(x > 0.0)) return -INFINITY;
    return -a->alpha1 * log(x) - a->scale / x;
}

typedef struct { double G, tau, sum_log, sum_inv, d; } nu_arg;

/* nu: -G lgamma(nu/2) + (G nu / 2) log(nu tau / 2) - (nu/2)(sum log gamma + tau sum 1/gamma) */
static double logf_nu(double x, const void *p)
{
    const nu_arg *a = (const nu_arg *)p;
    if (!(x > 0.0) || !(x < a->d)) return -INFINITY;
    return -a->G * lgamma(0.5 * x) + 0.5 * a->G * x * log(0.5 * x * a->tau)
           - 0.5 * x * (a->sum_log + (OR_MUTANT == 1 ? x : a->tau) * a->sum_inv);
}

typedef struct { double shape_m1, rate; } tau_arg;

/* tau: Gamma(a + G nu / 2, rate b + (nu/2) sum 1/gamma) */
static double logf_tau(double x, const void *p)
{
    const tau_arg *a = (const tau_arg *)p;
    if (!(x > 0.0)) return -INFINITY;
    return a->shape_m1 * log(x) - a->rate * x;
}

typedef struct { const or_ctx *c; int64_t g; int l; double Yl; double *bwork; } beta_arg;

/* beta_gl: beta Y_gl - sum_n exp(h_n + eps_gn + X_n beta_g) - (beta - theta_l)^2 / (2 sigma_l^2) */
static double logf_beta(double x, const void *p)
{
    const beta_arg *a = (const beta_arg *)p;
    const or_ctx *c = a->c;
    int L = c->cfg.L, N = c->cfg.N;
    a->bwork[a->l] = x;
    double sum = 0.0;
    for (int n = 0; n < N; ++n) {
        double eta = c->h[n] + c->eps[a->g * N + n];
        for (int l = 0; l < L; ++l) eta += c->X[n * L + l] * a->bwork[l];
        sum += exp(eta);
    }
    double dt = x - c->theta[a->l];
    return x * a->Yl - sum - dt * dt / (2.0 * c->sig2[a->l]);
}

typedef struct { double halfGp1, S, upper; } sig_arg;

/* sigma_l^2: -((G+1)/2) log v - S / (2 v) on 0 < v < s_l^2 */
static double logf_sig2(double x, const void *p)
{
    const sig_arg *a = (const sig_arg *)p;
    if (!(x > 0.0) || !(x < a->upper)) return -INFINITY;
    return -a->halfGp1 * log(x) - a->S / (2.0 * x);
}

/* ------------------------------------------------------------------ */
/* Learned proposal: features and the independence-MH step             */
/* ------------------------------------------------------------------ */
/* Features of gene g (definition in mlp.c): per distinct row r of X,
 * log((Y_r + 1/2) / A_r) and log(Y_r + 1/2), then theta and log sigma^2. */
static void gene_features(const or_ctx *c, int64_t g, double *phi, int F)
{
    const int N = c->cfg.N, L = c->cfg.L, R = c->R;
    double Y[OR_MAX_ROWS], A[OR_MAX_ROWS];
    for (int r = 0; r < R; ++r) { Y[r] = 0.0; A[r] = 0.0; }
    for (int n = 0; n < N; ++n) {
        Y[c->row_of[n]] += (double)c->y[g * N + n];
        A[c->row_of[n]] += exp(c->h[n] + c->eps[g * N + n]);
    }
    for (int i = 0; i < F; ++i) phi[i] = 0.0;
    for (int r = 0; r < R; ++r) {
        phi[r] = log((Y[r] + 0.5) / A[r]);
        phi[R + r] = log(Y[r] + 0.5);
    }
    for (int l = 0; l < L; ++l) {
        phi[2 * R + l] = c->theta[l];
        phi[2 * R + L + l] = log(c->sig2[l]);
    }
}

/* log of the beta_g full conditional at b, up to a constant:
 * sum_n [y_gn X_n b - exp(h_n + eps_gn + X_n b)] - sum_l (b_l - theta_l)^2 / (2 sigma_l^2) */
static double log_post_beta(const or_ctx *c, int64_t g, const double *b)
{
    const int N = c->cfg.N, L = c->cfg.L;
    double s = 0.0;
    for (int n = 0; n < N; ++n) {
        double xb = 0.0;
        for (int l = 0; l < L; ++l) xb += c->X[n * L + l] * b[l];
        s += (double)c->y[g * N + n] * xb - exp(c->h[n] + c->eps[g * N + n] + xb);
    }
    for (int l = 0; l < L; ++l) {
        const double d = b[l] - c->theta[l];
        s -= d * d / (2.0 * c->sig2[l]);
    }
    return s;
}

/* Cholesky factor of a symmetric positive definite L x L matrix: H = U U^T,
 * U lower triangular (row-major, zero above the diagonal). */
static void chol(const double *H, int L, double *U)
{
    for (int i = 0; i < L * L; ++i) U[i] = 0.0;
    for (int j = 0; j < L; ++j) {
        double d = H[j * L + j];
        for (int k = 0; k < j; ++k) d -= U[j * L + k] * U[j * L + k];
        U[j * L + j] = sqrt(d);
        for (int i = j + 1; i < L; ++i) {
            double s = H[i * L + j];
            for (int k = 0; k < j; ++k) s -= U[i * L + k] * U[j * L + k];
            U[i * L + j] = s / U[j * L + j];
        }
    }
}

/* x with H x = b, H = U U^T: forward then back substitution. */
static void chol_solve(const double *U, int L, const double *b, double *x)
{
    double t[OR_MAX_L];
    for (int i = 0; i < L; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= U[i * L + k] * t[k];
        t[i] = s / U[i * L + i];
    }
    for (int i = L - 1; i >= 0; --i) {
        double s = t[i];
        for (int k = i + 1; k < L; ++k) s -= U[k * L + i] * x[k];
        x[i] = s / U[i * L + i];
    }
}

/* The Laplace approximation of the beta_g conditional given eps_g, the base
 * of the learned proposal.  With Y_r and A_r the row sums of the counts and of
 * exp(h_n + eps_gn) over the samples of distinct row r (x_r) of X, the
 * conditional is
 *   log pi(b) = sum_r [Y_r x_r.b - A_r exp(x_r.b)] - sum_l (b_l - theta_l)^2 / (2 sigma_l^2).
 * Start: the weighted least-squares fit of log((Y_r + 1/2) / A_r) on x_r with
 * weights Y_r + 1/2 and the prior; then two Newton steps
 *   b += H^-1 [sum_r (Y_r - c_r) x_r - (b - theta) / sigma^2],
 *   H = sum_r c_r x_r x_r^T + diag(1 / sigma^2),  c_r = A_r exp(x_r.b).
 * Returns the last iterate bh and the lower Cholesky factor U of H at bh. */
static void laplace_base(const or_ctx *c, const double *Y, const double *A, double *bh, double *U)
{
    const int N = c->cfg.N, L = c->cfg.L, R = c->R;
    double xr[OR_MAX_ROWS * OR_MAX_L], H[OR_MAX_L * OR_MAX_L], rhs[OR_MAX_L], cr[OR_MAX_ROWS];
    for (int r = 0; r < R; ++r) {
        int n0 = 0;
        while (c->row_of[n0] != r) ++n0;
        for (int l = 0; l < L; ++l) xr[r * L + l] = c->X[n0 * L + l];
    }
    (void)N;
    /* weighted least squares start */
    for (int i = 0; i < L; ++i) {
        rhs[i] = c->theta[i] / c->sig2[i];
        for (int j = 0; j < L; ++j) H[i * L + j] = i == j ? 1.0 / c->sig2[i] : 0.0;
    }
    for (int r = 0; r < R; ++r) {
        const double w = Y[r] + 0.5, z = log(w / A[r]);
        for (int i = 0; i < L; ++i) {
            rhs[i] += w * z * xr[r * L + i];
            for (int j = 0; j < L; ++j) H[i * L + j] += w * xr[r * L + i] * xr[r * L + j];
        }
    }
    chol(H, L, U);
    chol_solve(U, L, rhs, bh);
    /* Newton steps, then the factor at the last iterate */
    for (int it = 0; it <= 2; ++it) {
        for (int r = 0; r < R; ++r) {
            double xb = 0.0;
            for (int l = 0; l < L; ++l) xb += xr[r * L + l] * bh[l];
            cr[r] = A[r] * exp(xb);
        }
        for (int i = 0; i < L; ++i) {
            rhs[i] = -(bh[i] - c->theta[i]) / c->sig2[i];
            for (int j = 0; j < L; ++j) H[i * L + j] = i == j ? 1.0 / c->sig2[i] : 0.0;
        }
        for (int r = 0; r < R; ++r)
            for (int i = 0; i < L; ++i) {
                rhs[i] += (Y[r] - cr[r]) * xr[r * L + i];
                for (int j = 0; j < L; ++j) H[i * L + j] += cr[r] * xr[r * L + i] * xr[r * L + j];
            }
        chol(H, L, U);
        if (it == 2) break;
        double step[OR_MAX_L];
        chol_solve(U, L, rhs, step);
        for (int l = 0; l < L; ++l) bh[l] += step[l];
    }
}

/* Row sums of gene g: Y_r (counts) and A_r (exp(h_n + eps_gn)). */
static void row_sums(const or_ctx *c, int64_t g, double *Y, double *A)
{
    const int N = c->cfg.N, R = c->R;
    for (int r = 0; r < R; ++r) { Y[r] = 0.0; A[r] = 0.0; }
    for (int n = 0; n < N; ++n) {
        Y[c->row_of[n]] += (double)c->y[g * N + n];
        A[c->row_of[n]] += exp(c->h[n] + c->eps[g * N + n]);
    }
}

/* One independence Metropolis-Hastings step for beta_g.  The proposal is the
 * Laplace approximation N(bh, H^-1) corrected by the network in whitened
 * coordinates w = U^T (b - bh): w ~ N(mu_w, Lw Lw^T) with the network's
 * outputs (mlp.c: mu_w = omean + oscale o, Lw = diag(oscale) Ls), so
 * beta* = bh + U^-T (mu_w + Lw z), z ~ N(0, I).  Up to a constant,
 * log q(x) = -sum_l ls_l - |u|^2 / 2 with Lw u = U^T (x - bh) - mu_w.
 * Random words come from counter (g, 8 << 24, m, chain << 16 | j): word 0 is
 * the acceptance uniform, words (1 + 2p, 2 + 2p) give the Box-Muller pair p of
 * normals (z_2p = rho cos(2 pi u_b), z_2p+1 = rho sin(2 pi u_b),
 * rho = sqrt(-2 log u_a)). */
static void imh_step(or_ctx *c, int64_t g, uint32_t mm)
{
    const int L = c->cfg.L, F = c->prop.F;
    const or_mlp *pm = &c->prop;
    double phi[OR_MLP_MAXW], o[OR_MLP_MAXW], Y[OR_MAX_ROWS], A[OR_MAX_ROWS];
    double bh[OR_MAX_L], U[OR_MAX_L * OR_MAX_L], mw[OR_MAX_L], z[OR_MAX_L], w[OR_MAX_L], bs[OR_MAX_L], d[OR_MAX_L],
        u[OR_MAX_L];
    gene_features(c, g, phi, F);
    or_mlp_outputs(pm, phi, o);
    row_sums(c, g, Y, A);
    laplace_base(c, Y, A, bh, U);
    for (int l = 0; l < L; ++l) mw[l] = pm->omean[l] + pm->oscale[l] * o[l];
    rstream rs;
    rs_init(&rs, c->cfg.seed, (uint32_t)g, OR_KIND_IMH, 0, mm, (uint32_t)c->cfg.chain);
    const double uacc = u01(rs_word(&rs, 0));
    for (int p = 0; 2 * p < L; ++p) {
        const double ua = u01(rs_word(&rs, (uint32_t)(1 + 2 * p)));
        const double ub = u01(rs_word(&rs, (uint32_t)(2 + 2 * p)));
        const double rho = sqrt(-2.0 * log(ua));
        z[2 * p] = rho * cos(2.0 * M_PI * ub);
        if (2 * p + 1 < L) z[2 * p + 1] = rho * sin(2.0 * M_PI * ub);
    }
    /* w = mu_w + Lw z; beta* = bh + v with U^T v = w (back substitution) */
    for (int l = 0; l < L; ++l) {
        double s = exp(o[L + l]) * z[l];
        for (int j = 0; j < l; ++j) s += o[2 * L + l * (l - 1) / 2 + j] * z[j];
        w[l] = mw[l] + pm->oscale[l] * s;
    }
    for (int i = L - 1; i >= 0; --i) {
        double s = w[i];
        for (int k = i + 1; k < L; ++k) s -= U[k * L + i] * (bs[k] - bh[k]);
        bs[i] = bh[i] + s / U[i * L + i];
    }
    const double *b = c->beta + g * L;
    double lq_new = 0.0, lq_old = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        const double *x = pass == 0 ? bs : b;
        for (int i = 0; i < L; ++i) {          /* d = U^T (x - bh) - mu_w */
            double s = 0.0;
            for (int k = i; k < L; ++k) s += U[k * L + i] * (x[k] - bh[k]);
            d[i] = s - mw[i];
        }
        or_mlp_solve(pm, L, o, d, u);
        double lq = 0.0;
        for (int l = 0; l < L; ++l) lq -= log(pm->oscale[l]) + o[L + l] + 0.5 * u[l] * u[l];
        if (pass == 0) lq_new = lq; else lq_old = lq;
    }
    const double la = (log_post_beta(c, g, bs) - log_post_beta(c, g, b)) - (OR_MUTANT == 9 ? 0.0 : lq_new - lq_old);
    c->imh_la[g] = la;
    if (log(uacc) < la) {
        for (int l = 0; l < L; ++l) c->beta[g * L + l] = bs[l];
        c->imh_acc[g] = 1;
    } else {
        c->imh_acc[g] = 0;
    }
}

/* The shift step (an addition to Algorithm 1, enabled by bit OR_KIND_SHIFT of
 * update_mask).  In the model of Section 4.1 the counts of gene g depend on
 * eps_g and beta_g only through the sums zeta_gn = eps_gn + X_n beta_g, so the
 * map beta_g -> beta_g + delta, eps_gn -> eps_gn - X_n delta leaves the
 * likelihood unchanged and has unit Jacobian.  Given zeta_g, gamma_g, theta
 * and sigma^2, delta has the Gaussian density proportional to
 *   exp(-sum_n (eps_gn - X_n delta)^2 / (2 gamma_g)
 *       - sum_l (beta_gl + delta_l - theta_l)^2 / (2 sigma_l^2)),
 * i.e. precision P = X^T X / gamma_g + diag(1 / sigma^2) and mean P^-1 c with
 * c = X^T eps_g / gamma_g - (beta_g - theta) / sigma^2.  The step draws delta
 * exactly: delta = P^-1 c + U^-T z, P = U U^T, z ~ N(0, I) from Box-Muller
 * pairs on words (2p, 2p + 1) of counter (g, 11 << 24, m, chain << 16 | j). */
static void shift_step(or_ctx *c, int64_t g, uint32_t mm)
{
    const int N = c->cfg.N, L = c->cfg.L;
    double P[OR_MAX_L * OR_MAX_L], U[OR_MAX_L * OR_MAX_L], cv[OR_MAX_L], mean[OR_MAX_L], z[OR_MAX_L], v[OR_MAX_L];
    const double ig = 1.0 / c->gam[g];
    for (int i = 0; i < L; ++i) {
        double s = 0.0;
        for (int n = 0; n < N; ++n) s += c->X[n * L + i] * c->eps[g * N + n];
        cv[i] = s * ig - (OR_MUTANT == 11 ? 0.0 : (c->beta[g * L + i] - c->theta[i]) / c->sig2[i]);
        for (int j = 0; j < L; ++j) {
            double x = 0.0;
            for (int n = 0; n < N; ++n) x += c->X[n * L + i] * c->X[n * L + j];
            P[i * L + j] = x * ig + (i == j ? 1.0 / c->sig2[i] : 0.0);
        }
    }
    chol(P, L, U);
    chol_solve(U, L, cv, mean);
    rstream rs;
    rs_init(&rs, c->cfg.seed, (uint32_t)g, OR_KIND_SHIFT, 0, mm, (uint32_t)c->cfg.chain);
    for (int p = 0; 2 * p < L; ++p) {
        const double ua = u01(rs_word(&rs, (uint32_t)(2 * p)));
        const double ub = u01(rs_word(&rs, (uint32_t)(2 * p + 1)));
        const double rho = sqrt(-2.0 * log(ua));
        z[2 * p] = rho * cos(2.0 * M_PI * ub);
        if (2 * p + 1 < L) z[2 * p + 1] = rho * sin(2.0 * M_PI * ub);
    }
    /* v = U^-T z (back substitution) */
    for (int i = L - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < L; ++k) s -= U[k * L + i] * v[k];
        v[i] = s / U[i * L + i];
    }
    double d[OR_MAX_L];
    for (int l = 0; l < L; ++l) {
        d[l] = mean[l] + v[l];
        c->beta[g * L + l] += d[l];
    }
    for (int n = 0; n < N; ++n) {
        double xd = 0.0;
        for (int l = 0; l < L; ++l) xd += c->X[n * L + l] * d[l];
        c->eps[g * N + n] -= (OR_MUTANT == 10 ? -xd : xd);
    }
}

int or_set_proposal(or_ctx *c, const or_mlp *m, const int32_t *fallback_mask)
{
    if (!c) return -1;
    if (!m) { c->prop_on = 0; return 0; }
    const int L = c->cfg.L;
    if (m->O != 2 * L + L * (L - 1) / 2 || m->F < 2 * c->R + 2 * L || m->F > OR_MLP_MAXW || m->H > OR_MLP_MAXW || m->H < 1)
        return -1;
    const size_t F = (size_t)m->F, H = (size_t)m->H, O = (size_t)m->O;
    const size_t total = 2 * F + F * H + H + H * H + H + H * O + O + 2 * (size_t)L;
    double *buf = (double *)malloc(sizeof(double) * total);
    if (!buf) return -2;
    double *p = buf;
    or_mlp cp = *m;
#define OR_TAKE(field, n) do { memcpy(p, m->field, sizeof(double) * (n)); cp.field = p; p += (n); } while (0)
    OR_TAKE(fmean, F); OR_TAKE(fscale, F);
    OR_TAKE(W1, F * H); OR_TAKE(b1, H); OR_TAKE(W2, H * H); OR_TAKE(b2, H);
    OR_TAKE(W3, H * O); OR_TAKE(b3, O); OR_TAKE(omean, (size_t)L); OR_TAKE(oscale, (size_t)L);
#undef OR_TAKE
    free(c->prop_buf);
    c->prop_buf = buf;
    c->prop = cp;
    for (int64_t g = 0; g < c->cfg.G; ++g) c->prop_mask[g] = fallback_mask ? fallback_mask[g] : 0;
    c->prop_on = 1;
    return 0;
}

int or_features(const or_ctx *c, int32_t F, double *phi)
{
    if (!c || !phi || F < 2 * c->R + 2 * c->cfg.L) return -1;
    for (int64_t g = 0; g < c->cfg.G; ++g) gene_features(c, g, phi + g * F, F);
    return 0;
}

int or_get_imh(const or_ctx *c, int32_t *acc, double *log_alpha)
{
    if (!c) return -1;
    if (acc) memcpy(acc, c->imh_acc, sizeof(int32_t) * (size_t)c->cfg.G);
    if (log_alpha) memcpy(log_alpha, c->imh_la, sizeof(double) * (size_t)c->cfg.G);
    return 0;
}

int or_num_rows(const or_ctx *c) { return c ? c->R : -1; }

/* ------------------------------------------------------------------ */
/* One sweep                                                           */
/* ------------------------------------------------------------------ */
static void record(or_ctx *c, int64_t idx, const draw_info *di)
{
    c->cnt[4 * idx + 0] = di->kl;
    c->cnt[4 * idx + 1] = di->nl;
    c->cnt[4 * idx + 2] = di->nr;
    c->cnt[4 * idx + 3] = di->nc;
    c->mrg[idx] = di->margin;
}

static void welford(double *mean, double *msq, double x, int64_t k)
{
    *mean += (x - *mean) / (double)k;
    *msq += (x * x - *msq) / (double)k;
}

/* eps_gn for every gene and sample: the Poisson log pmf of y_gn in eps
 * (without the term in y alone) plus the N(0, gamma_g) prior, given beta_g
 * and gamma_g.  The draws are independent across (g, n). */
static int64_t update_eps(or_ctx *c, int64_t m)
{
    const or_config *cf = &c->cfg;
    const int64_t G = cf->G;
    const int N = cf->N;
    int64_t errs = 0;
#pragma omp parallel for schedule(static) reduction(+:errs) num_threads(c->nthreads)
    for (int64_t g = 0; g < G; ++g) {
        for (int n = 0; n < N; ++n) {
            eps_arg a = { c, g, n };
            rstream rs;
            draw_info di;
            rs_init(&rs, cf->seed, (uint32_t)g, OR_KIND_EPS, (uint32_t)n, (uint32_t)m, (uint32_t)cf->chain);
            const int64_t i = g * N + n;
            c->eps[i] = slice_draw(logf_eps, &a, c->eps[i], &c->w_eps[i], &c->wa_eps[i], m,
                                   cf->burnin, cf->tune_start, cf->K, cf->shrink_cap, &rs, &di);
            record(c, i, &di);
            errs += di.bad;
        }
    }
    return errs;
}

/* gamma_g for every gene: InvGamma(nu/2 + N/2, nu tau/2 + sum_n eps_gn^2 / 2),
 * slice sampled, or drawn directly with the exact-draw option. */
static int64_t update_gamma(or_ctx *c, int64_t m)
{
    const or_config *cf = &c->cfg;
    const int64_t G = cf->G;
    const int N = cf->N;
    const int64_t off_gam = G * N;
    int64_t errs = 0;
#pragma omp parallel for schedule(static) reduction(+:errs) num_threads(c->nthreads)
    for (int64_t g = 0; g < G; ++g) {
        double S = 0.0;
        for (int n = 0; n < N; ++n) S += c->eps[g * N + n] * c->eps[g * N + n];
        gam_arg a = { 0.5 * c->nu + (OR_MUTANT == 2 ? 1.0 : 0.5) * N + 1.0,
                      0.5 * c->nu * c->tau + 0.5 * S };
        rstream rs;
        draw_info di;
        if (cf->update_mask & (1u << OR_KIND_EXACT)) {
            exact_arg e = { 0.5 * c->nu + 0.5 * N, (OR_MUTANT == 15 ? c->nu * c->tau : 0.5 * c->nu * c->tau) + 0.5 * S,
                            1, INFINITY };
            double v;
            int t = exact_draw(&e, cf->seed, OR_KIND_EXACT, (uint32_t)g, 0, (uint32_t)m, (uint32_t)cf->chain, &v, &di);
            if (t > 0) {
                c->gam[g] = v;
                di.kl = -1; di.nl = 0; di.nr = 0; di.nc = t;
                record(c, off_gam + g, &di);
                continue;
            }
        }
        rs_init(&rs, cf->seed, (uint32_t)g, OR_KIND_GAMMA, 0, (uint32_t)m, (uint32_t)cf->chain);
        c->gam[g] = slice_draw(logf_gam, &a, c->gam[g], &c->w_gam[g], &c->wa_gam[g], m,
                               cf->burnin, cf->tune_start, cf->K, cf->shrink_cap, &rs, &di);
        record(c, off_gam + g, &di);
        errs += di.bad;
    }
    return errs;
}

/* The sums over genes that the nu and tau conditionals need. */
static void gamma_sums(or_ctx *c)
{
    double sum_log = 0.0, sum_inv = 0.0;
    for (int64_t g = 0; g < c->cfg.G; ++g) { sum_log += log(c->gam[g]); sum_inv += 1.0 / c->gam[g]; }
    c->red[0] = sum_log;
    c->red[1] = sum_inv;
}

/* nu given gamma and tau: the product of the InvGamma(nu/2, nu tau/2)
 * densities of the gamma_g on the U(0, d) support (logf_nu). */
static int64_t update_nu(or_ctx *c, int64_t m)
{
    const or_config *cf = &c->cfg;
    nu_arg a = { (double)cf->G, c->tau, c->red[0], c->red[1], cf->d };
    rstream rs;
    draw_info di;
    rs_init(&rs, cf->seed, 0, OR_KIND_NU, 0, (uint32_t)m, (uint32_t)cf->chain);
    c->nu = slice_draw(logf_nu, &a, c->nu, &c->w_nu, &c->wa_nu, m, cf->burnin,
                       cf->tune_start, cf->K, cf->shrink_cap, &rs, &di);
    record(c, cf->G * cf->N + cf->G + cf->G * cf->L, &di);
    return di.bad;
}

/* tau given nu and gamma: Gamma(a + G nu / 2, rate b + (nu/2) sum_g 1/gamma_g). */
static int64_t update_tau(or_ctx *c, int64_t m)
{
    const or_config *cf = &c->cfg;
    tau_arg a = { cf->a + 0.5 * (double)cf->G * c->nu - 1.0,
                  cf->b + (OR_MUTANT == 8 ? 1.0 : 0.5) * c->nu * c->red[1] };
    rstream rs;
    draw_info di;
    int t = 0;
    if (cf->update_mask & (1u << OR_KIND_EXACT)) {
        exact_arg e = { a.shape_m1 + 1.0, a.rate, 0, INFINITY };
        double v;
        t = exact_draw(&e, cf->seed, OR_KIND_EXACT, 0, 1, (uint32_t)m, (uint32_t)cf->chain, &v, &di);
        if (t > 0) {
            c->tau = v;
            di.kl = -1; di.nl = 0; di.nr = 0; di.nc = t;
        }
    }
    if (t == 0) {
        rs_init(&rs, cf->seed, 0, OR_KIND_TAU, 0, (uint32_t)m, (uint32_t)cf->chain);
        c->tau = slice_draw(logf_tau, &a, c->tau, &c->w_tau, &c->wa_tau, m, cf->burnin,
                            cf->tune_start, cf->K, cf->shrink_cap, &rs, &di);
    }
    record(c, cf->G * cf->N + cf->G + cf->G * cf->L + 1, &di);
    return di.bad;
}

/* beta_g for every gene, one coefficient at a time (l = 1..L, each with the
 * latest values of the others); the genes are conditionally independent, so
 * gene-major order is the same chain.  Genes with the learned proposal on
 * take one independence Metropolis-Hastings step for the whole block. */
static int64_t update_beta(or_ctx *c, int64_t m)
{
    const or_config *cf = &c->cfg;
    const int64_t G = cf->G;
    const int N = cf->N, L = cf->L;
    const int64_t off_beta = G * N + G;
    int64_t errs = 0;
#pragma omp parallel for schedule(static) reduction(+:errs) num_threads(c->nthreads)
    for (int64_t g = 0; g < G; ++g) {
        if (c->prop_on && !c->prop_mask[g]) {
            imh_step(c, g, (uint32_t)m);
            continue;
        }
        c->imh_acc[g] = -1;
        for (int l = 0; l < L; ++l) {
            double bwork[OR_MAX_L];
            for (int i = 0; i < L; ++i) bwork[i] = c->beta[g * L + i];
            double Yl = 0.0;
            int lx = OR_MUTANT == 5 ? (l + 1) % L : l;
            for (int n = 0; n < N; ++n) Yl += (double)c->y[g * N + n] * c->X[n * L + lx];
            beta_arg a = { c, g, l, Yl, bwork };
            rstream rs;
            draw_info di;
            rs_init(&rs, cf->seed, (uint32_t)g, OR_KIND_BETA, (uint32_t)l, (uint32_t)m, (uint32_t)cf->chain);
            const int64_t i = g * L + l;
            c->beta[i] = slice_draw(logf_beta, &a, c->beta[i], &c->w_beta[i], &c->wa_beta[i], m,
                                    cf->burnin, cf->tune_start, cf->K, cf->shrink_cap, &rs, &di);
            record(c, off_beta + i, &di);
            errs += di.bad;
        }
    }
    return errs;
}

/* theta_l, then sigma_l^2, for each l: theta_l given beta and sigma_l^2 is
 * Normal and drawn directly (Box-Muller); sigma_l^2 given beta and the new
 * theta_l is InvGamma((G - 1)/2, sum_g (beta_gl - theta_l)^2 / 2) truncated
 * to (0, s_l^2), slice sampled or drawn directly with the exact-draw option. */
static int64_t update_theta_sigma(or_ctx *c, int64_t m)
{
    const or_config *cf = &c->cfg;
    const int64_t G = cf->G;
    const int L = cf->L;
    const uint32_t mask = cf->update_mask, mm = (uint32_t)m;
    const int64_t off_hyp = G * cf->N + G + G * L;
    int64_t errs = 0;
    for (int l = 0; l < L; ++l) {
        double sb = 0.0;
        for (int64_t g = 0; g < G; ++g) sb += c->beta[g * L + l];
        c->red[2 + 2 * l] = sb;
        if (mask & (1u << OR_KIND_THETA)) {
            double prec = (double)G / c->sig2[l] + 1.0 / (c->c[l] * c->c[l]);
            /* prior N(theta_mean_l, c_l^2): theta_mean = 0 in the model of Section 4.1,
             * psi_l of the top level in the three-level form (Section 2.3) */
            double mean = (sb / c->sig2[l] + (OR_MUTANT == 19 ? 0.0 : c->theta_mean[l] / (c->c[l] * c->c[l]))) / prec;
            uint32_t ctr[4] = { 0, ((uint32_t)OR_KIND_THETA << 24) | (uint32_t)l, mm,
                                (uint32_t)cf->chain << 16 };
            uint32_t key[2] = { (uint32_t)cf->seed, (uint32_t)(cf->seed >> 32) };
            uint32_t r[4];
            or_philox4x32_10(ctr, key, r);
            double zn = sqrt(-2.0 * log(u01(r[0]))) * cos(2.0 * M_PI * u01(r[1]));
            c->theta[l] = mean + zn / (OR_MUTANT == 7 ? prec : sqrt(prec));
        }
        double S = 0.0;
        for (int64_t g = 0; g < G; ++g) {
            double dv = c->beta[g * L + l] - c->theta[l];
            S += dv * dv;
        }
        c->red[3 + 2 * l] = S;
        if (mask & (1u << OR_KIND_SIG2)) {
            sig_arg a = { 0.5 * ((double)G + (OR_MUTANT == 3 ? 2.0 : 1.0)), S, c->s[l] * c->s[l] };
            rstream rs;
            draw_info di;
            int t = 0;
            if (mask & (1u << OR_KIND_EXACT)) {
                exact_arg e = { 0.5 * ((double)G - 1.0), 0.5 * S, 1,
                                OR_MUTANT == 16 ? INFINITY : c->s[l] * c->s[l] };
                double v;
                t = exact_draw(&e, cf->seed, OR_KIND_EXACT, 0, 2u + (uint32_t)l, mm, (uint32_t)cf->chain, &v, &di);
                if (t > 0) {
                    c->sig2[l] = v;
                    di.kl = -1; di.nl = 0; di.nr = 0; di.nc = t;
                }
            }
            if (t == 0) {
                rs_init(&rs, cf->seed, 0, OR_KIND_SIG2, (uint32_t)l, mm, (uint32_t)cf->chain);
                c->sig2[l] = slice_draw(logf_sig2, &a, c->sig2[l], &c->w_sig2[l], &c->wa_sig2[l], m,
                                        cf->burnin, cf->tune_start, cf->K, cf->shrink_cap, &rs, &di);
            }
            record(c, off_hyp + 2 + l, &di);
            errs += di.bad;
        }
    }
    return errs;
}

/* Running means and means of squares of every parameter (Section 3.1), over
 * the sweeps after burn-in. */
static void update_moments(or_ctx *c, int64_t m)
{
    const int64_t G = c->cfg.G;
    const int N = c->cfg.N, L = c->cfg.L;
    const int64_t off_gam = G * N, off_beta = G * N + G;
    const int64_t k = m - c->cfg.burnin;
    double *mu = c->mean, *sq = c->msq;
    for (int64_t i = 0; i < G * N; ++i) welford(&mu[i], &sq[i], c->eps[i], k);
    for (int64_t g = 0; g < G; ++g) welford(&mu[off_gam + g], &sq[off_gam + g], c->gam[g], k);
    for (int64_t i = 0; i < G * L; ++i) welford(&mu[off_beta + i], &sq[off_beta + i], c->beta[i], k);
    int64_t o = off_beta + G * L;
    welford(&mu[o], &sq[o], c->nu, k);
    welford(&mu[o + 1], &sq[o + 1], c->tau, k);
    for (int l = 0; l < L; ++l) welford(&mu[o + 2 + l], &sq[o + 2 + l], c->theta[l], k);
    for (int l = 0; l < L; ++l) welford(&mu[o + 2 + L + l], &sq[o + 2 + L + l], c->sig2[l], k);
    c->count = k;
}

/* Indicators of the contrast events (Section 3.2) at the end of the sweep. */
static void count_events(or_ctx *c)
{
    const int64_t G = c->cfg.G;
    const int L = c->cfg.L;
    for (int64_t g = 0; g < G; ++g) {
        for (int e = 0; e < c->n_ev; ++e) {
            int all = 1;
            for (int r = 0; r < c->n_crow; ++r) {
                if (c->crow_event[r] != e) continue;
                double sum = 0.0;
                for (int l = 0; l < L; ++l) sum += c->cv[r * L + l] * c->beta[g * L + l];
                if (OR_MUTANT == 12) { if (sum > c->cb[r]) all = 2; else if (all == 1) all = 0; }
                else if (!(sum > c->cb[r])) all = 0;
            }
            c->ev_count[g * c->n_ev + e] += all ? 1 : 0;
        }
    }
}

/* One sweep m = c->m + 1: the conditionals in the order of Algorithm 1
 * (eps, gamma, nu, tau, beta, theta and sigma^2), each step enabled by its
 * bit of update_mask; the shift step, when enabled, after beta. */
static int64_t sweep_once(or_ctx *c)
{
    const uint32_t mask = c->cfg.update_mask;
    const int64_t m = c->m + 1;
    int64_t errs = 0;
    if (mask & (1u << OR_KIND_EPS)) errs += update_eps(c, m);
    if (mask & (1u << OR_KIND_GAMMA)) errs += update_gamma(c, m);
    gamma_sums(c);
    if (mask & (1u << OR_KIND_NU)) errs += update_nu(c, m);
    if (mask & (1u << OR_KIND_TAU)) errs += update_tau(c, m);
    if (mask & (1u << OR_KIND_BETA)) errs += update_beta(c, m);
    if (mask & (1u << OR_KIND_SHIFT)) {
#pragma omp parallel for schedule(static) num_threads(c->nthreads)
        for (int64_t g = 0; g < c->cfg.G; ++g) shift_step(c, g, (uint32_t)m);
    }
    errs += update_theta_sigma(c, m);
    if (m > c->cfg.burnin) update_moments(c, m);
    if (c->n_ev > 0 && m > c->cfg.burnin && m > c->ev_from) count_events(c);
    c->m = m;
    return errs;
}

int or_set_contrasts(or_ctx *c, int32_t n_events, int32_t n_rows, const int32_t *row_event, const double *v,
                     const double *b)
{
    if (!c || n_events < 0 || n_rows < n_events || (n_rows > 0 && (!row_event || !v || !b))) return -1;
    for (int r = 0; r < n_rows; ++r)
        if (row_event[r] < 0 || row_event[r] >= n_events) return -1;
    for (int e = 0; e < n_events; ++e) {
        int seen = 0;
        for (int r = 0; r < n_rows; ++r) seen |= row_event[r] == e;
        if (!seen) return -1;
    }
    const int L = c->cfg.L;
    const int64_t G = c->cfg.G;
    free(c->crow_event); free(c->cv); free(c->cb); free(c->ev_count);
    c->crow_event = (int32_t *)xcalloc((size_t)n_rows, sizeof(int32_t));
    c->cv = (double *)xcalloc((size_t)n_rows * L, sizeof(double));
    c->cb = (double *)xcalloc((size_t)n_rows, sizeof(double));
    c->ev_count = (int64_t *)xcalloc((size_t)(G * (n_events ? n_events : 1)), sizeof(int64_t));
    if (!c->crow_event || !c->cv || !c->cb || !c->ev_count) return -2;
    if (n_rows) {
        memcpy(c->crow_event, row_event, sizeof(int32_t) * (size_t)n_rows);
        memcpy(c->cv, v, sizeof(double) * (size_t)n_rows * L);
        memcpy(c->cb, b, sizeof(double) * (size_t)n_rows);
    }
    c->n_ev = n_events;
    c->n_crow = n_rows;
    c->ev_from = c->m;
    return 0;
}

int or_event_counts(const or_ctx *c, int64_t *counts, int64_t *n_sweeps)
{
    if (!c) return -1;
    if (counts && c->n_ev) memcpy(counts, c->ev_count, sizeof(int64_t) * (size_t)(c->cfg.G * c->n_ev));
    if (n_sweeps) {
        const int64_t from = c->cfg.burnin > c->ev_from ? c->cfg.burnin : c->ev_from;
        *n_sweeps = c->m > from ? c->m - from : 0;
    }
    return 0;
}

int or_sweep(or_ctx *c, int64_t n)
{
    if (!c || n < 0) return -1;
    int64_t errs = 0;
    for (int64_t i = 0; i < n; ++i) errs += sweep_once(c);
    c->errors += errs;
    return errs ? -4 : 0;
}

/* ------------------------------------------------------------------ */
/* State access                                                        */
/* ------------------------------------------------------------------ */
static void cp(double *dst, const double *src, int64_t n)
{
    if (dst && src) memcpy(dst, src, sizeof(double) * (size_t)n);
}

int or_get_state(const or_ctx *c, double *eps, double *gam, double *beta, double *hyp,
                 double *w_eps, double *waux_eps, double *w_gam, double *waux_gam,
                 double *w_beta, double *waux_beta, double *w_hyp, double *waux_hyp, int64_t *m)
{
    if (!c) return -1;
    int64_t G = c->cfg.G, N = c->cfg.N, L = c->cfg.L;
    cp(eps, c->eps, G * N); cp(gam, c->gam, G); cp(beta, c->beta, G * L);
    if (hyp) {
        hyp[0] = c->nu; hyp[1] = c->tau;
        for (int l = 0; l < L; ++l) { hyp[2 + l] = c->theta[l]; hyp[2 + L + l] = c->sig2[l]; }
    }
    cp(w_eps, c->w_eps, G * N); cp(waux_eps, c->wa_eps, G * N);
    cp(w_gam, c->w_gam, G); cp(waux_gam, c->wa_gam, G);
    cp(w_beta, c->w_beta, G * L); cp(waux_beta, c->wa_beta, G * L);
    if (w_hyp) { w_hyp[0] = c->w_nu; w_hyp[1] = c->w_tau; for (int l = 0; l < L; ++l) w_hyp[2 + l] = c->w_sig2[l]; }
    if (waux_hyp) { waux_hyp[0] = c->wa_nu; waux_hyp[1] = c->wa_tau; for (int l = 0; l < L; ++l) waux_hyp[2 + l] = c->wa_sig2[l]; }
    if (m) *m = c->m;
    return 0;
}

static void cpin(double *dst, const double *src, int64_t n)
{
    if (dst && src) memcpy(dst, src, sizeof(double) * (size_t)n);
}

int or_set_state(or_ctx *c, const double *eps, const double *gam, const double *beta,
                 const double *hyp, const double *w_eps, const double *waux_eps,
                 const double *w_gam, const double *waux_gam, const double *w_beta,
                 const double *waux_beta, const double *w_hyp, const double *waux_hyp, int64_t m)
{
    if (!c || m < 0) return -1;
    int64_t G = c->cfg.G, N = c->cfg.N, L = c->cfg.L;
    cpin(c->eps, eps, G * N); cpin(c->gam, gam, G); cpin(c->beta, beta, G * L);
    if (hyp) {
        c->nu = hyp[0]; c->tau = hyp[1];
        for (int l = 0; l < L; ++l) { c->theta[l] = hyp[2 + l]; c->sig2[l] = hyp[2 + L + l]; }
    }
    cpin(c->w_eps, w_eps, G * N); cpin(c->wa_eps, waux_eps, G * N);
    cpin(c->w_gam, w_gam, G); cpin(c->wa_gam, waux_gam, G);
    cpin(c->w_beta, w_beta, G * L); cpin(c->wa_beta, waux_beta, G * L);
    if (w_hyp) { c->w_nu = w_hyp[0]; c->w_tau = w_hyp[1]; for (int l = 0; l < L; ++l) c->w_sig2[l] = w_hyp[2 + l]; }
    if (waux_hyp) { c->wa_nu = waux_hyp[0]; c->wa_tau = waux_hyp[1]; for (int l = 0; l < L; ++l) c->wa_sig2[l] = waux_hyp[2 + l]; }
    c->m = m;
    return 0;
}

int or_get_moments(const or_ctx *c, double *mean_eps, double *msq_eps, double *mean_gam,
                   double *msq_gam, double *mean_beta, double *msq_beta, double *mean_hyp,
                   double *msq_hyp, int64_t *count)
{
    if (!c) return -1;
    int64_t G = c->cfg.G, N = c->cfg.N, L = c->cfg.L;
    int64_t og = G * N, ob = og + G, oh = ob + G * L;
    cp(mean_eps, c->mean, G * N); cp(msq_eps, c->msq, G * N);
    cp(mean_gam, c->mean + og, G); cp(msq_gam, c->msq + og, G);
    cp(mean_beta, c->mean + ob, G * L); cp(msq_beta, c->msq + ob, G * L);
    cp(mean_hyp, c->mean + oh, 2 + 2 * L); cp(msq_hyp, c->msq + oh, 2 + 2 * L);
    if (count) *count = c->count;
    return 0;
}

int or_get_counts(const or_ctx *c, int32_t *cnt_eps, int32_t *cnt_gam, int32_t *cnt_beta,
                  int32_t *cnt_hyp, double *mrg_eps, double *mrg_gam, double *mrg_beta,
                  double *mrg_hyp)
{
    if (!c) return -1;
    int64_t G = c->cfg.G, N = c->cfg.N, L = c->cfg.L;
    int64_t og = G * N, ob = og + G, oh = ob + G * L;
    if (cnt_eps) memcpy(cnt_eps, c->cnt, sizeof(int32_t) * 4 * (size_t)(G * N));
    if (cnt_gam) memcpy(cnt_gam, c->cnt + 4 * og, sizeof(int32_t) * 4 * (size_t)G);
    if (cnt_beta) memcpy(cnt_beta, c->cnt + 4 * ob, sizeof(int32_t) * 4 * (size_t)(G * L));
    if (cnt_hyp) memcpy(cnt_hyp, c->cnt + 4 * oh, sizeof(int32_t) * 4 * (size_t)(2 + L));
    cp(mrg_eps, c->mrg, G * N); cp(mrg_gam, c->mrg + og, G);
    cp(mrg_beta, c->mrg + ob, G * L); cp(mrg_hyp, c->mrg + oh, 2 + L);
    return 0;
}

int or_get_reductions(const or_ctx *c, double *out)
{
    if (!c || !out) return -1;
    memcpy(out, c->red, sizeof(double) * (size_t)(2 + 2 * c->cfg.L));
    return 0;
}

/* ------------------------------------------------------------------ */
/* Default starting values                                             */
/* ------------------------------------------------------------------ */
/* Solve the L x L system A x = r by Gaussian elimination with partial pivoting. */
static int solve(double *A, double *r, int L)
{
    for (int k = 0; k < L; ++k) {
        int p = k;
        for (int i = k + 1; i < L; ++i) if (fabs(A[i * L + k]) > fabs(A[p * L + k])) p = i;
        if (fabs(A[p * L + k]) < 1e-12) return -1;
        if (p != k) {
            for (int j = 0; j < L; ++j) { double t = A[k * L + j]; A[k * L + j] = A[p * L + j]; A[p * L + j] = t; }
            double t = r[k]; r[k] = r[p]; r[p] = t;
        }
        for (int i = k + 1; i < L; ++i) {
            double f = A[i * L + k] / A[k * L + k];
            for (int j = k; j < L; ++j) A[i * L + j] -= f * A[k * L + j];
            r[i] -= f * r[k];
        }
    }
    for (int k = L - 1; k >= 0; --k) {
        double s = r[k];
        for (int j = k + 1; j < L; ++j) s -= A[k * L + j] * r[j];
        r[k] = s / A[k * L + k];
    }
    return 0;
}

int or_init_default(or_ctx *c)
{
    if (!c) return -1;
    const int64_t G = c->cfg.G;
    const int N = c->cfg.N, L = c->cfg.L;
    double XtX[OR_MAX_L * OR_MAX_L];
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
            double s = 0.0;
            for (int n = 0; n < N; ++n) s += c->X[n * L + i] * c->X[n * L + j];
            XtX[i * L + j] = s + (i == j ? 1e-8 : 0.0);
        }
    double sb[OR_MAX_L] = { 0 }, sbb[OR_MAX_L] = { 0 }, sg = 0.0;
    for (int64_t g = 0; g < G; ++g) {
        double A[OR_MAX_L * OR_MAX_L], r[OR_MAX_L];
        memcpy(A, XtX, sizeof(double) * (size_t)(L * L));
        for (int l = 0; l < L; ++l) {
            double s = 0.0;
            for (int n = 0; n < N; ++n)
                s += c->X[n * L + l] * (log1p((double)c->y[g * N + n]) - c->h[n]);
            r[l] = s;
        }
        if (solve(A, r, L) != 0) for (int l = 0; l < L; ++l) r[l] = 0.0;
        double rss = 0.0;
        for (int n = 0; n < N; ++n) {
            double e = log1p((double)c->y[g * N + n]) - c->h[n];
            for (int l = 0; l < L; ++l) e -= c->X[n * L + l] * r[l];
            rss += e * e;
        }
        double gm = N > L ? rss / (double)(N - L) : 0.1;
        if (gm < 0.01) gm = 0.01;
        c->gam[g] = gm;
        sg += gm;
        for (int l = 0; l < L; ++l) {
            c->beta[g * L + l] = r[l];
            sb[l] += r[l];
            sbb[l] += r[l] * r[l];
        }
        for (int n = 0; n < N; ++n) c->eps[g * N + n] = 0.0;
    }
    for (int l = 0; l < L; ++l) {
        double mu = sb[l] / (double)G;
        double v = sbb[l] / (double)G - mu * mu;
        double hi = 0.25 * c->s[l] * c->s[l];
        if (!(v > 1e-4)) v = 1e-4;
        if (v > hi) v = hi;
        c->theta[l] = mu;
        c->sig2[l] = v;
    }
    c->tau = sg / (double)G;
    c->nu = 10.0 < 0.5 * c->cfg.d ? 10.0 : 0.5 * c->cfg.d;
    c->m = 0;
    c->count = 0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Slice sampler on textbook targets (tests of Algorithm 2 alone)      */
/* ------------------------------------------------------------------ */
typedef struct { int kind; double p0, p1, p2; } test_arg;

static double logf_test(double x, const void *p)
{
    const test_arg *a = (const test_arg *)p;
    switch (a->kind) {
    case 0: { double z = (x - a->p0) / a->p1; return -0.5 * z * z; }
    case 1: if (!(x > 0.0)) return -INFINITY; return (a->p0 - 1.0) * log(x) - a->p1 * x;
    case 2: if (!(x > 0.0)) return -INFINITY; return -(a->p0 + 1.0) * log(x) - a->p1 / x;
    case 3: if (!(x > 0.0) || !(x < a->p2)) return -INFINITY; return -(a->p0 + 1.0) * log(x) - a->p1 / x;
    default: return NAN;
    }
}

int or_slice_test(int32_t target, const double *params, const double *x0, double *x1,
                  int64_t n, double w, int32_t K, uint64_t seed, uint32_t m, int32_t *counts)
{
    if (!params || !x0 || !x1 || n < 0 || target < 0 || target > 3) return -1;
    if (!(K == 0 || K == 1 || K == 3 || K == 7 || K == 15)) return -1;
    test_arg a = { target, params[0], params[1], target == 3 ? params[2] : 0.0 };
    int64_t errs = 0;
    for (int64_t i = 0; i < n; ++i) {
        rstream rs;
        draw_info di;
        double ww = w, wa = 0.0;
        rs_init(&rs, seed, (uint32_t)i, OR_KIND_TEST, 0, m, 0);
        /* burnin = 0: w stays frozen */
        x1[i] = slice_draw(logf_test, &a, x0[i], &ww, &wa, (int64_t)m, 0, 0, K, 1000, &rs, &di);
        if (counts) {
            counts[4 * i + 0] = di.kl; counts[4 * i + 1] = di.nl;
            counts[4 * i + 2] = di.nr; counts[4 * i + 3] = di.nc;
        }
        errs += di.bad;
    }
    return errs ? -4 : 0;
}
