/*
 * oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the fully Bayesian Gibbs sampler for
 * the Poisson-lognormal RNA-seq model (Section 4.1 and Fig. 3 of Landau & Niemi,
 * arXiv 1606.06659): the Gibbs scan of Algorithm 1, with every non-normal
 * conditional drawn by the univariate stepping-out slice sampler with an
 * adaptive width of Algorithm 2 (Appendix A).
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP path.
 *
 * Parameter kinds and their random-number counters
 * ------------------------------------------------
 * Every random word comes from Philox4x32-10 (Salmon et al., SC'11) keyed by
 * the 64-bit seed, with counter (c0, c1, c2, c3) =
 *   (gene g, kind << 24 | sub, sweep m, chain << 16 | block j).
 * Kinds: 1 eps (sub = n), 2 gamma, 3 nu, 4 tau, 5 beta (sub = l), 6 theta
 * (sub = l), 7 sigma^2 (sub = l), 8 independence-MH, 9 initial jitter,
 * 10 slice-sampler test targets.  g = 0 for the hyperparameters.
 *
 * One slice draw reads block 0: word 0 -> E = -log u (the slice height in log
 * space), word 1 -> K_L = word & K in its low 4 bits and the window offset
 * u = (word >> 4 + 1/2) 2^-28 in its high 28 bits, words 2 and 3 -> the first
 * two shrink candidates.  Candidate t >= 1 uses word q = t + 1 of the stream,
 * i.e. block q / 4, word q % 4.  A 32-bit word r maps to u = (r + 1/2) 2^-32.
 */
#ifndef FB_ORACLE_H
#define FB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OR_KIND_EPS = 1, OR_KIND_GAMMA = 2, OR_KIND_NU = 3, OR_KIND_TAU = 4,
    OR_KIND_BETA = 5, OR_KIND_THETA = 6, OR_KIND_SIG2 = 7, OR_KIND_IMH = 8,
    OR_KIND_INIT = 9, OR_KIND_TEST = 10, OR_KIND_SHIFT = 11, OR_KIND_EXACT = 12, OR_KIND_TOP = 13
};

/* bit (1 << kind) of update_mask enables that Gibbs step; the shift step
 * (kind 11) is an addition to Algorithm 1 and is not in OR_UPDATE_ALL.  Bit
 * OR_KIND_EXACT (also not in OR_UPDATE_ALL) replaces the slice draws of
 * gamma_g, tau and sigma_l^2 by direct draws from their conjugate full
 * conditionals (Section 4.2 names this alternative); see oracle.c. */
#define OR_UPDATE_ALL 0xFEu

/* Bounds of the work arrays: at most OR_MAX_L coefficients and OR_MAX_ROWS
 * distinct rows of X; or_create rejects larger designs (returns -1). */
#define OR_MAX_L 8
#define OR_MAX_ROWS 64

typedef struct {
    int32_t G, N, L;
    const int32_t *y;      /* [G][N] counts, row g = gene */
    const double *X;       /* [N][L] design */
    const double *h;       /* [N] offsets */
    double a, b, d;        /* tau ~ Gamma(a, rate b), nu ~ U(0, d) */
    const double *c;       /* [L] theta_l ~ N(0, c_l^2) */
    const double *s;       /* [L] sigma_l ~ U(0, s_l) */
    uint64_t seed;
    int32_t chain;
    int64_t burnin;        /* M_B: sweeps 1..M_B tune w and skip the moments */
    int64_t tune_start;    /* M_C: w is recomputed only for M_C < m <= M_B */
    int32_t K;             /* step-out budget, one of 0, 1, 3, 7, 15 */
    double w0;             /* initial slice width */
    uint32_t update_mask;  /* 1 << kind for each Gibbs step to run */
    int32_t shrink_cap;    /* maximum shrink candidates per draw */
} or_config;

typedef struct or_ctx or_ctx;

/* Sizes: hyp = [nu, tau, theta(L), sig2(L)] has 2 + 2L entries;
 * whyp (slice widths of the slice-sampled hyperparameters) = [nu, tau, sig2(L)]
 * has 2 + L entries. */
int  or_create(or_ctx **out, const or_config *cfg);
void or_destroy(or_ctx *c);
/* Replace the count matrix (same G, N). */
int  or_set_counts(or_ctx *c, const int32_t *y);
int  or_set_update_mask(or_ctx *c, uint32_t mask);
int  or_set_threads(or_ctx *c, int32_t nthreads);

/* Deterministic default starting values (per-gene least squares). */
int  or_init_default(or_ctx *c);

int  or_get_state(const or_ctx *c, double *eps, double *gam, double *beta, double *hyp,
                  double *w_eps, double *waux_eps, double *w_gam, double *waux_gam,
                  double *w_beta, double *waux_beta, double *w_hyp, double *waux_hyp,
                  int64_t *m);
int  or_set_state(or_ctx *c, const double *eps, const double *gam, const double *beta,
                  const double *hyp, const double *w_eps, const double *waux_eps,
                  const double *w_gam, const double *waux_gam, const double *w_beta,
                  const double *waux_beta, const double *w_hyp, const double *waux_hyp,
                  int64_t m);

/* Run n sweeps.  Returns 0, or -4 if a draw hit the shrink cap or met a
 * non-finite log density (the draw then keeps its old value). */
int  or_sweep(or_ctx *c, int64_t n);

int  or_get_moments(const or_ctx *c, double *mean_eps, double *msq_eps, double *mean_gam,
                    double *msq_gam, double *mean_beta, double *msq_beta, double *mean_hyp,
                    double *msq_hyp, int64_t *count);

/* Per-draw record of the last sweep: 4 int32 per slice draw
 * (K_L, left moves, right moves, shrink candidates) and the smallest
 * |log f(x) - z| over the draw's slice comparisons. */
int  or_get_counts(const or_ctx *c, int32_t *cnt_eps, int32_t *cnt_gam, int32_t *cnt_beta,
                   int32_t *cnt_hyp, double *mrg_eps, double *mrg_gam, double *mrg_beta,
                   double *mrg_hyp);
int64_t or_error_count(const or_ctx *c);

/* Reductions the hyperparameter steps of the last sweep used:
 * [sum log gamma, sum 1/gamma, then per l: sum beta_l, sum (beta_l - theta_l)^2]. */
int  or_get_reductions(const or_ctx *c, double *out);

/* ---- building blocks exposed for the tests ---- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* One slice step (w frozen) from each x0[i] for a test target:
 * kind 0: N(p0, p1^2); 1: Gamma(shape p0, rate p1); 2: InvGamma(shape p0, scale p1);
 * 3: InvGamma(shape p0, scale p1) truncated to (0, p2).
 * Draw i uses counter (i, 10 << 24, m, 0). counts may be NULL. */
int  or_slice_test(int32_t target, const double *params, const double *x0, double *x1,
                   int64_t n, double w, int32_t K, uint64_t seed, uint32_t m,
                   int32_t *counts);

/* ---- learned beta proposal (mlp.c) ---- */
#define OR_MLP_MAXW 256
typedef struct {
    int32_t F, H, O;              /* inputs, hidden width, outputs (= 2L) */
    const double *fmean, *fscale; /* [F] input standardisation */
    const double *W1, *b1;        /* [F][H], [H] */
    const double *W2, *b2;        /* [H][H], [H] */
    const double *W3, *b3;        /* [H][O], [O] */
    const double *omean, *oscale; /* [L] output affine map */
} or_mlp;

/* Number of coefficients L of a network with O = 2L + L(L-1)/2 outputs, or -1. */
int or_mlp_coefs(int O);
/* For feature rows phi [B][F]: mu, ls [B][L] (proposal means and log of the
 * factor's diagonal) and off [B][L(L-1)/2] (the strict lower triangle of the
 * factor in units of oscale, row-major); any output may be NULL. */
int or_mlp_forward(const or_mlp *m, const double *phi, int64_t B, double *mu, double *ls, double *off);
/* Raw outputs o [O] of one feature row; u with Lc u = d for outputs o. */
void or_mlp_outputs(const or_mlp *m, const double *phi, double *o);
void or_mlp_solve(const or_mlp *m, int L, const double *o, const double *d, double *u);
/* Mean Gaussian NLL of targets [B][L] and its gradients (any may be NULL). */
int or_mlp_loss_grad(const or_mlp *m, const double *phi, const double *target, int64_t B,
                     double *loss, double *gW1, double *gb1, double *gW2, double *gb2,
                     double *gW3, double *gb3);

/* Use the learned proposal for the beta draws: genes with fallback_mask[g] = 0 take
 * one independence Metropolis-Hastings step for beta_g (mlp.c describes the
 * features and the network); the others keep the slice steps.  The model is
 * copied.  m = NULL switches the proposal off. */
int or_set_proposal(or_ctx *c, const or_mlp *m, const int32_t *fallback_mask);
/* Features of every gene of the current state, [G][F]. */
int or_features(const or_ctx *c, int32_t F, double *phi);
/* Last sweep's IMH records per gene: acc (1 accepted, 0 rejected, -1 slice)
 * and the log acceptance ratio. */
int or_get_imh(const or_ctx *c, int32_t *acc, double *log_alpha);
/* Number of distinct rows of X. */
int or_num_rows(const or_ctx *c);

/* Posterior probabilities of contrast events (Section 3.2): event e holds
 * when every row r with row_event[r] == e has sum_l v[r][l] beta_gl > b[r]
 * (v is [n_rows][L]).  Counting starts with the sweeps after this call and
 * after burn-in; or_event_counts returns counts [G][n_events] and the number
 * of sweeps counted. */
int or_set_contrasts(or_ctx *c, int32_t n_events, int32_t n_rows, const int32_t *row_event, const double *v,
                     const double *b);
int or_event_counts(const or_ctx *c, int64_t *counts, int64_t *n_sweeps);

/* Three-level form (Section 2.3), see oracle.c: or_set_top_priors sets the
 * rate b of tau's Gamma prior and the prior means of theta (both fixed by the
 * top level psi); or_top_draw draws b and psi (arrays theta [K][L], tau [K],
 * a [K], c [K][L], c0 [L]); b and psi are in/out; tries gets the attempts of
 * the b draw (0: none succeeded, b kept). */
int or_set_top_priors(or_ctx *c, double b, const double *theta_mean);
int or_top_draw(int32_t K, int32_t L, const double *theta, const double *tau, const double *a, const double *c,
                double a_b, double b_b, const double *c0, uint64_t seed, int32_t chain, int64_t m, uint32_t mask,
                double *b, double *psi, int32_t *tries);

#ifdef __cplusplus
}
#endif
#endif
