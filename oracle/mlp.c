/*
 * mlp.c -- TEST INFRASTRUCTURE ONLY: FP64 reference of the learned beta
 * proposal (plain loops, no blocking).
 *
 * The proposal is an independence Metropolis-Hastings step for beta_g (the
 * block of L coefficients of one gene).  Its base is the Laplace approximation
 * N(bh, H^-1) of the beta_g conditional (oracle.c), and the network corrects it
 * in the whitened coordinates w = U^T (b - bh), H = U U^T: w ~ N(mu, Lc Lc^T)
 * with mean and lower-triangular factor given by a small MLP of per-gene
 * features (a zero network with omean = 0, oscale = 1 leaves the Laplace
 * proposal):
 *
 *   input   x = (phi - fmean) * fscale, clipped to [-8, 8]        [F]
 *   z1 = x W1 + b1,  h1 = gelu(z1)                                [H]
 *   z2 = h1 W2 + b2, h2 = gelu(z2)                                [H]
 *   o  = h2 W3 + b3                                  [O = 2L + L(L-1)/2]
 *   mu_l  = omean_l + oscale_l o_l
 *   Lc_ll = exp(ls_l),  ls_l = log(oscale_l) + o_{L+l}
 *   Lc_lj = oscale_l o_{2L + l(l-1)/2 + j}   (j < l; zero above the diagonal)
 *
 * so Lc = diag(oscale) Ls, with Ls the factor in units of oscale.  The clip
 * keeps the network on the range its training inputs are clipped to.  gelu(z) =
 * z Phi(z) (the erf form).  Weights are row-major with the input index first:
 * z1_j = b1_j + sum_i x_i W1[i][j].
 *
 * Features of gene g (any function of y_g, eps_g, h, theta, sigma^2 -- never
 * of beta_g, so the proposal does not depend on the current value and the
 * step is an exact independence sampler): for each distinct row r of X,
 * Y_r = sum of the counts of the samples with that row and
 * A_r = sum of exp(h_n + eps_gn) over those samples;
 *   phi[r]       = log((Y_r + 1/2) / A_r)   (the row's log-rate estimate)
 *   phi[R + r]   = log(Y_r + 1/2)           (its information)
 *   phi[2R + l]  = theta_l,  phi[2R + L + l] = log sigma_l^2,
 * zero beyond 2R + 2L.
 *
 * Training loss (Gaussian negative log likelihood of a target, the whitened
 * w of a draw of beta_g from its conditional), averaged
 * over the batch: sum_l ls_l + |u|^2 / 2 with Lc u = t - mu (forward
 * substitution).  With zero off-diagonal outputs this is
 * sum_l [ls_l + (t_l - mu_l)^2 exp(-2 ls_l) / 2].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double gelu_d(double z)
{
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}

/* Forward pass of one input row; keeps the pre-activations for backward. */
static void fwd(const or_mlp *m, const double *phi, double *x, double *z1, double *h1,
                double *z2, double *h2, double *o)
{
    const int F = m->F, H = m->H, O = m->O;
    for (int i = 0; i < F; ++i) x[i] = fmin(fmax((phi[i] - m->fmean[i]) * m->fscale[i], -8.0), 8.0);
    for (int j = 0; j < H; ++j) {
        double s = m->b1[j];
        for (int i = 0; i < F; ++i) s += x[i] * m->W1[i * H + j];
        z1[j] = s;
        h1[j] = gelu(s);
    }
    for (int j = 0; j < H; ++j) {
        double s = m->b2[j];
        for (int i = 0; i < H; ++i) s += h1[i] * m->W2[i * H + j];
        z2[j] = s;
        h2[j] = gelu(s);
    }
    for (int j = 0; j < O; ++j) {
        double s = m->b3[j];
        for (int i = 0; i < H; ++i) s += h2[i] * m->W3[i * O + j];
        o[j] = s;
    }
}

int or_mlp_coefs(int O)
{
    for (int L = 1; L <= 16; ++L)
        if (2 * L + L * (L - 1) / 2 == O) return L;
    return -1;
}

int or_mlp_forward(const or_mlp *m, const double *phi, int64_t B, double *mu, double *ls, double *off)
{
    if (!m || !phi || B < 0 || m->F > OR_MLP_MAXW || m->H > OR_MLP_MAXW || m->O > OR_MLP_MAXW) return -1;
    const int L = or_mlp_coefs(m->O), K = L * (L - 1) / 2;
    if (L < 1) return -1;
    double x[OR_MLP_MAXW], z1[OR_MLP_MAXW], h1[OR_MLP_MAXW], z2[OR_MLP_MAXW], h2[OR_MLP_MAXW], o[OR_MLP_MAXW];
    for (int64_t b = 0; b < B; ++b) {
        fwd(m, phi + b * m->F, x, z1, h1, z2, h2, o);
        for (int l = 0; l < L; ++l) {
            if (mu) mu[b * L + l] = m->omean[l] + m->oscale[l] * o[l];
            if (ls) ls[b * L + l] = log(m->oscale[l]) + o[L + l];
        }
        if (off)
            for (int k = 0; k < K; ++k) off[b * K + k] = o[2 * L + k];
    }
    return 0;
}

/* u with Lc u = d: Lc_ll = oscale_l exp(o_{L+l}), Lc_lj = oscale_l o_{2L+l(l-1)/2+j}. */
void or_mlp_solve(const or_mlp *m, int L, const double *o, const double *d, double *u)
{
    for (int l = 0; l < L; ++l) {
        double s = d[l] / m->oscale[l];
        for (int j = 0; j < l; ++j) s -= o[2 * L + l * (l - 1) / 2 + j] * u[j];
        u[l] = s / exp(o[L + l]);
    }
}

/* The raw outputs o of one feature row. */
void or_mlp_outputs(const or_mlp *m, const double *phi, double *o)
{
    double x[OR_MLP_MAXW], z1[OR_MLP_MAXW], h1[OR_MLP_MAXW], z2[OR_MLP_MAXW], h2[OR_MLP_MAXW];
    fwd(m, phi, x, z1, h1, z2, h2, o);
}

int or_mlp_loss_grad(const or_mlp *m, const double *phi, const double *target, int64_t B,
                     double *loss, double *gW1, double *gb1, double *gW2, double *gb2,
                     double *gW3, double *gb3)
{
    if (!m || !phi || !target || B < 1) return -1;
    const int F = m->F, H = m->H, O = m->O, L = or_mlp_coefs(O);
    if (F > OR_MLP_MAXW || H > OR_MLP_MAXW || O > OR_MLP_MAXW || L < 1) return -1;
    if (gW1) memset(gW1, 0, sizeof(double) * (size_t)F * H);
    if (gb1) memset(gb1, 0, sizeof(double) * (size_t)H);
    if (gW2) memset(gW2, 0, sizeof(double) * (size_t)H * H);
    if (gb2) memset(gb2, 0, sizeof(double) * (size_t)H);
    if (gW3) memset(gW3, 0, sizeof(double) * (size_t)H * O);
    if (gb3) memset(gb3, 0, sizeof(double) * (size_t)O);
    double x[OR_MLP_MAXW], z1[OR_MLP_MAXW], h1[OR_MLP_MAXW], z2[OR_MLP_MAXW], h2[OR_MLP_MAXW], o[OR_MLP_MAXW];
    double dO[OR_MLP_MAXW], dZ2[OR_MLP_MAXW], dZ1[OR_MLP_MAXW];
    double d[OR_MLP_MAXW], u[OR_MLP_MAXW], v[OR_MLP_MAXW];
    double total = 0.0;
    const double invB = 1.0 / (double)B;
    for (int64_t b = 0; b < B; ++b) {
        fwd(m, phi + b * F, x, z1, h1, z2, h2, o);
        for (int l = 0; l < L; ++l) d[l] = target[b * L + l] - (m->omean[l] + m->oscale[l] * o[l]);
        or_mlp_solve(m, L, o, d, u);
        /* v = Ls^{-T} u (back substitution on the factor in units of oscale) */
        for (int l = L - 1; l >= 0; --l) {
            double s = u[l];
            for (int i = l + 1; i < L; ++i) s -= o[2 * L + i * (i - 1) / 2 + l] * v[i];
            v[l] = s / exp(o[L + l]);
        }
        for (int l = 0; l < L; ++l) total += log(m->oscale[l]) + o[L + l] + 0.5 * u[l] * u[l];
        /* d/d o: mean -v_l; log-diagonal 1 - v_l u_l Ls_ll; off-diagonal (l, j) -v_l u_j */
        for (int j = 0; j < O; ++j) dO[j] = 0.0;
        for (int l = 0; l < L; ++l) {
            dO[l] = -v[l] * invB;
            dO[L + l] = (1.0 - v[l] * u[l] * exp(o[L + l])) * invB;
            for (int j = 0; j < l; ++j) dO[2 * L + l * (l - 1) / 2 + j] = -v[l] * u[j] * invB;
        }
        for (int j = 0; j < O; ++j) {
            if (gb3) gb3[j] += dO[j];
            if (gW3) for (int i = 0; i < H; ++i) gW3[i * O + j] += h2[i] * dO[j];
        }
        for (int i = 0; i < H; ++i) {
            double s = 0.0;
            for (int j = 0; j < O; ++j) s += m->W3[i * O + j] * dO[j];
            dZ2[i] = s * gelu_d(z2[i]);
        }
        for (int j = 0; j < H; ++j) {
            if (gb2) gb2[j] += dZ2[j];
            if (gW2) for (int i = 0; i < H; ++i) gW2[i * H + j] += h1[i] * dZ2[j];
        }
        for (int i = 0; i < H; ++i) {
            double s = 0.0;
            for (int j = 0; j < H; ++j) s += m->W2[i * H + j] * dZ2[j];
            dZ1[i] = s * gelu_d(z1[i]);
        }
        for (int j = 0; j < H; ++j) {
            if (gb1) gb1[j] += dZ1[j];
            if (gW1) for (int i = 0; i < F; ++i) gW1[i * H + j] += x[i] * dZ1[j];
        }
    }
    if (loss) *loss = total * invB;
    return 0;
}
