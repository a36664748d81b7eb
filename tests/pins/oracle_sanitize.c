/*
 * oracle_sanitize.c -- a CPU driver that runs every path of the oracle once at
 * the largest design it accepts (L = OR_MAX_L coefficients), so that a build
 * with -fsanitize=address,undefined sees every array access of those paths.
 * It also checks that designs beyond the oracle's bounds are rejected.
 *
 * Inputs are small and deterministic (a linear congruential generator); the
 * numbers themselves are not checked here, only that nothing reads or writes
 * out of bounds and that the calls succeed.  Prints "ok" and exits 0.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t lcg_state = 12345u;
static double lcg_u(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return ((double)(lcg_state >> 11) + 0.5) * 0x1p-53;
}

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

enum { G = 37, N = 16, L = OR_MAX_L, F = 32, H = 24 };

static double *fill(size_t n, double scale)
{
    double *p = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (size_t i = 0; i < n; ++i) p[i] = scale * (2.0 * lcg_u() - 1.0);
    return p;
}

static int run_paths(void)
{
    /* design: the 8 rows of the order-8 Hadamard matrix (column 0 is the
     * intercept), each twice */
    static double X[N * L];
    for (int n = 0; n < N; ++n)
        for (int l = 0; l < L; ++l) X[n * L + l] = (__builtin_popcount((unsigned)((n % 8) & l)) & 1) ? -1.0 : 1.0;
    static int32_t y[G * N];
    for (int i = 0; i < G * N; ++i) y[i] = (int32_t)(lcg_u() * 60.0);
    y[0] = 0;
    y[1] = 100000;
    double h[N], c[L], s[L];
    for (int n = 0; n < N; ++n) h[n] = 0.1 * (2.0 * lcg_u() - 1.0);
    for (int l = 0; l < L; ++l) { c[l] = 10.0; s[l] = 100.0; }
    or_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.G = G; cfg.N = N; cfg.L = L; cfg.y = y; cfg.X = X; cfg.h = h;
    cfg.a = 1.0; cfg.b = 1.0; cfg.d = 1000.0; cfg.c = c; cfg.s = s;
    cfg.seed = 99; cfg.chain = 1; cfg.burnin = 4; cfg.tune_start = 1; cfg.K = 15; cfg.w0 = 1.0;
    cfg.update_mask = OR_UPDATE_ALL; cfg.shrink_cap = 200;

    or_ctx *ctx = NULL;
    CHECK(or_create(&ctx, &cfg) == 0);
    CHECK(or_num_rows(ctx) == 8);
    CHECK(or_init_default(ctx) == 0);
    /* contrast events: two events over three rows */
    const int32_t row_event[3] = { 0, 0, 1 };
    double v[3 * L], b[3];
    for (int i = 0; i < 3 * L; ++i) v[i] = (i % 3) - 1.0;
    b[0] = 0.0; b[1] = -0.5; b[2] = 0.25;
    CHECK(or_set_contrasts(ctx, 2, 3, row_event, v, b) == 0);
    /* plain slice sweeps, through burn-in and past it */
    or_sweep(ctx, 6);
    /* with the shift step, then the exact conjugate draws as well */
    CHECK(or_set_update_mask(ctx, OR_UPDATE_ALL | (1u << OR_KIND_SHIFT)) == 0);
    or_sweep(ctx, 3);
    CHECK(or_set_update_mask(ctx, OR_UPDATE_ALL | (1u << OR_KIND_SHIFT) | (1u << OR_KIND_EXACT)) == 0);
    or_sweep(ctx, 3);
    /* the learned proposal: a random network, a third of the genes in fallback */
    const int O = 2 * L + L * (L - 1) / 2;
    CHECK(or_mlp_coefs(O) == L);
    double *fmean = fill(F, 0.1), *fscale = fill(F, 0.0), *W1 = fill((size_t)F * H, 0.2), *b1 = fill(H, 0.1);
    double *W2 = fill((size_t)H * H, 0.2), *b2 = fill(H, 0.1), *W3 = fill((size_t)H * O, 0.05), *b3 = fill(O, 0.05);
    double *omean = fill(L, 0.0), *oscale = fill(L, 0.0);
    for (int i = 0; i < F; ++i) fscale[i] = 1.0;
    for (int l = 0; l < L; ++l) oscale[l] = 1.0;
    or_mlp net = { F, H, O, fmean, fscale, W1, b1, W2, b2, W3, b3, omean, oscale };
    int32_t fb[G];
    for (int g = 0; g < G; ++g) fb[g] = g % 3 == 0;
    CHECK(or_set_proposal(ctx, &net, fb) == 0);
    CHECK(or_set_update_mask(ctx, OR_UPDATE_ALL) == 0);
    or_sweep(ctx, 3);
    CHECK(or_set_update_mask(ctx, OR_UPDATE_ALL | (1u << OR_KIND_SHIFT)) == 0);
    or_sweep(ctx, 2);
    int32_t acc[G];
    double la[G];
    CHECK(or_get_imh(ctx, acc, la) == 0);
    double *phi = (double *)malloc(sizeof(double) * G * F);
    CHECK(or_features(ctx, F, phi) == 0);
    double *mu = (double *)malloc(sizeof(double) * G * L), *ls = (double *)malloc(sizeof(double) * G * L);
    double *off = (double *)malloc(sizeof(double) * G * (L * (L - 1) / 2));
    CHECK(or_mlp_forward(&net, phi, G, mu, ls, off) == 0);
    double *tgt = fill((size_t)G * L, 1.0), loss = 0.0;
    double *gW1 = fill((size_t)F * H, 0.0), *gb1 = fill(H, 0.0), *gW2 = fill((size_t)H * H, 0.0);
    double *gb2 = fill(H, 0.0), *gW3 = fill((size_t)H * O, 0.0), *gb3 = fill(O, 0.0);
    CHECK(or_mlp_loss_grad(&net, phi, tgt, G, &loss, gW1, gb1, gW2, gb2, gW3, gb3) == 0);
    CHECK(isfinite(loss));
    CHECK(or_set_proposal(ctx, NULL, NULL) == 0);
    /* the three-level driver's prior hooks */
    double tm[L];
    for (int l = 0; l < L; ++l) tm[l] = 0.1 * l;
    CHECK(or_set_top_priors(ctx, 2.0, tm) == 0);
    or_sweep(ctx, 2);
    /* every read-out */
    double *eps = malloc(sizeof(double) * G * N), *weps = malloc(sizeof(double) * G * N),
           *waeps = malloc(sizeof(double) * G * N), *gam = malloc(sizeof(double) * G),
           *wgam = malloc(sizeof(double) * G), *wagam = malloc(sizeof(double) * G),
           *beta = malloc(sizeof(double) * G * L), *wbeta = malloc(sizeof(double) * G * L),
           *wabeta = malloc(sizeof(double) * G * L), hyp[2 + 2 * L], whyp[2 + L], wahyp[2 + L];
    int64_t m = 0;
    CHECK(or_get_state(ctx, eps, gam, beta, hyp, weps, waeps, wgam, wagam, wbeta, wabeta, whyp, wahyp, &m) == 0);
    CHECK(m == 19);
    CHECK(or_set_state(ctx, eps, gam, beta, hyp, weps, waeps, wgam, wagam, wbeta, wabeta, whyp, wahyp, m) == 0);
    double *me = malloc(sizeof(double) * G * N), *se = malloc(sizeof(double) * G * N), mg[G], sg[G];
    double *mb = malloc(sizeof(double) * G * L), *sbq = malloc(sizeof(double) * G * L), mh[2 + 2 * L], sh[2 + 2 * L];
    int64_t cnt = 0;
    CHECK(or_get_moments(ctx, me, se, mg, sg, mb, sbq, mh, sh, &cnt) == 0);
    CHECK(cnt == 15);
    int32_t *ce = malloc(sizeof(int32_t) * 4 * G * N), cg[4 * G], *cb = malloc(sizeof(int32_t) * 4 * G * L),
            ch[4 * (2 + L)];
    double *re = malloc(sizeof(double) * G * N), rg[G], *rb = malloc(sizeof(double) * G * L), rh[2 + L];
    CHECK(or_get_counts(ctx, ce, cg, cb, ch, re, rg, rb, rh) == 0);
    double red[2 + 2 * L];
    CHECK(or_get_reductions(ctx, red) == 0);
    int64_t evc[G * 2], nsw = 0;
    CHECK(or_event_counts(ctx, evc, &nsw) == 0);
    CHECK(nsw == 15);
    or_destroy(ctx);

    /* the top-level draws of the three-level form, K = 5 groups */
    enum { K = 5 };
    double th[K * L], tau[K], a[K], cc[K * L], c0[L], bb = 1.0, psi[L];
    for (int i = 0; i < K * L; ++i) { th[i] = lcg_u(); cc[i] = 1.0 + lcg_u(); }
    for (int k = 0; k < K; ++k) { tau[k] = 0.5 + lcg_u(); a[k] = 1.0 + lcg_u(); }
    for (int l = 0; l < L; ++l) c0[l] = 10.0;
    int32_t tries = 0;
    CHECK(or_top_draw(K, L, th, tau, a, cc, 1.0, 1.0, c0, 7, 0, 3, 3u, &bb, psi, &tries) == 0);
    CHECK(or_top_draw(K, L + 1, th, tau, a, cc, 1.0, 1.0, c0, 7, 0, 3, 3u, &bb, psi, &tries) == -1);

    /* the slice sampler on its textbook targets */
    double x0[64], x1[64], prm[3] = { 3.5, 1.0, 0.35 };
    int32_t counts[4 * 64];
    for (int i = 0; i < 64; ++i) x0[i] = 0.05 + 0.004 * i;
    for (int t = 0; t < 4; ++t) CHECK(or_slice_test(t, prm, x0, x1, 64, 0.3, 15, 5, 2, counts) != -1);

    free(fmean); free(fscale); free(W1); free(b1); free(W2); free(b2); free(W3); free(b3);
    free(omean); free(oscale); free(phi); free(mu); free(ls); free(off); free(tgt);
    free(gW1); free(gb1); free(gW2); free(gb2); free(gW3); free(gb3);
    free(eps); free(weps); free(waeps); free(gam); free(wgam); free(wagam);
    free(beta); free(wbeta); free(wabeta); free(me); free(se); free(mb); free(sbq);
    free(ce); free(cb); free(re); free(rb);
    return 0;
}

/* Designs beyond the work arrays are rejected by or_create. */
static int run_bounds(void)
{
    enum { NB = 70, LB = OR_MAX_L + 1 };
    static double X[NB * LB];
    static int32_t y[2 * NB];
    double h[NB], c[LB], s[LB];
    for (int i = 0; i < NB * LB; ++i) X[i] = (i % LB == 0) ? 1.0 : (double)((i * 7) % 3) - 1.0;
    for (int n = 0; n < NB; ++n) h[n] = 0.0;
    for (int l = 0; l < LB; ++l) { c[l] = 10.0; s[l] = 100.0; }
    or_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.G = 2; cfg.N = 16; cfg.L = LB; cfg.y = y; cfg.X = X; cfg.h = h;
    cfg.a = 1.0; cfg.b = 1.0; cfg.d = 1000.0; cfg.c = c; cfg.s = s;
    cfg.seed = 1; cfg.K = 15; cfg.w0 = 1.0; cfg.update_mask = OR_UPDATE_ALL; cfg.shrink_cap = 200;
    or_ctx *ctx = NULL;
    CHECK(or_create(&ctx, &cfg) == -1 && ctx == NULL);
    /* L = 2 but more distinct rows than OR_MAX_ROWS: row n = (1, n) */
    for (int n = 0; n < NB; ++n) { X[2 * n] = 1.0; X[2 * n + 1] = (double)n; }
    cfg.N = NB; cfg.L = 2;
    CHECK(or_create(&ctx, &cfg) == -1 && ctx == NULL);
    /* at the bound itself it is accepted */
    cfg.N = OR_MAX_ROWS;
    CHECK(or_create(&ctx, &cfg) == 0 && ctx != NULL);
    CHECK(or_num_rows(ctx) == OR_MAX_ROWS);
    or_init_default(ctx);
    or_sweep(ctx, 2);
    or_destroy(ctx);
    return 0;
}

int main(void)
{
    if (run_paths() != 0) return 1;
    if (run_bounds() != 0) return 1;
    printf("ok\n");
    return 0;
}
