/*
 * libfbmc -- fully Bayesian MCMC for the Poisson-lognormal RNA-seq model on
 * AMD Instinct MI355X (gfx950).
 *
 * Landau & Niemi, "A fully Bayesian strategy for high-dimensional hierarchical
 * modeling using massively parallel computing", arXiv 1606.06659.
 *
 * Model (Section 4.1, Fig. 3), for genes g = 1..G and samples n = 1..N:
 *   y_gn | eps_gn, beta_g ~ Poisson(exp(h_n + eps_gn + X_n beta_g))
 *   eps_gn | gamma_g      ~ Normal(0, gamma_g)            (variance)
 *   gamma_g | nu, tau     ~ InvGamma(nu/2, nu tau/2)      (shape, scale)
 *   nu ~ Uniform(0, d),   tau ~ Gamma(a, rate b)
 *   beta_gl | theta_l, sigma_l ~ Normal(theta_l, sigma_l^2)
 *   theta_l ~ Normal(0, c_l^2),  sigma_l ~ Uniform(0, s_l)
 *
 * One sweep (Algorithm 1) draws every eps_gn, gamma_g and beta_gl from its full
 * conditional with the stepping-out slice sampler of Algorithm 2 (Appendix A),
 * in parallel over genes, forms the sufficient sums of gamma and beta by
 * parallel reductions (Section 2.2), draws nu, tau (slice), theta_l (Normal)
 * and sigma_l^2 (slice), and updates the running mean and mean of squares of
 * every parameter on the device (Section 3.1).  All random numbers come from
 * Philox4x32-10 with the counter (gene, kind << 24 | index, sweep,
 * chain << 16 | block) under the 64-bit seed, so every draw is reproducible.
 *
 * Conventions for every function below
 * ------------------------------------
 *  - Host pointers, row-major arrays, caller-owned.  The library copies every
 *    input it keeps and never retains a caller pointer after the call returns.
 *  - Status codes: FB_OK (0) or a negative FB_E* code; nothing is thrown across
 *    the ABI.  fb_last_error() returns a message for the last failure on a
 *    context (fb_last_error(NULL) covers fb_create failures, per thread).
 *  - A context is not thread-safe; calls on one context must not overlap.
 *  - Work is enqueued on the context's HIP stream (fb_options.stream, or a
 *    stream the library creates).  fb_sweep returns once the work is enqueued;
 *    device-side errors surface on a later synchronising call
 *    (fb_sync, fb_get_state, fb_summaries, fb_trace, fb_debug_counts).
 */
#ifndef LIBFBMC_H
#define LIBFBMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FB_OK        0
#define FB_EINVAL   (-1)  /* invalid argument or unsupported shape */
#define FB_ENOMEM   (-2)  /* device or host allocation failed */
#define FB_EDEVICE  (-3)  /* a HIP runtime call failed */
#define FB_ENUMERIC (-4)  /* a draw met a non-finite log density or hit the shrink cap (sticky) */
#define FB_ESTATE   (-5)  /* call not valid in the context's current state */

/* Limits of this build. */
#define FB_MAX_N        64   /* samples per dataset */
#define FB_MAX_L        8    /* model-matrix columns */
#define FB_MAX_ROWS     8    /* distinct rows of X */
#define FB_MAX_COLVALS  4    /* distinct non-zero values in one column of X */

enum fb_precision {
    FB_FP64 = 0,   /* every draw in double precision */
    FB_FP32 = 1    /* eps/gamma/beta log densities in float; reductions, moments,
                      hyperparameters in double */
};

enum fb_kind {     /* Philox counter kinds, also bit positions of update_mask */
    FB_KIND_EPS = 1, FB_KIND_GAMMA = 2, FB_KIND_NU = 3, FB_KIND_TAU = 4,
    FB_KIND_BETA = 5, FB_KIND_THETA = 6, FB_KIND_SIG2 = 7, FB_KIND_IMH = 8,
    FB_KIND_SHIFT = 11, FB_KIND_EXACT = 12
};
/* The steps of Algorithm 1.  The shift step (bit 1 << FB_KIND_SHIFT) is an
 * addition that is off unless asked for: after steps 2 and 5 it moves every
 * gene along the directions that leave eps_gn + X_n beta_g -- and so the
 * likelihood of the model of Section 4.1 -- unchanged,
 *   beta_g -> beta_g + delta,  eps_gn -> eps_gn - X_n delta,
 * with delta drawn exactly from its Gaussian conditional given those sums,
 * gamma_g, theta and sigma^2 (precision X^T X / gamma_g + diag(1 / sigma^2),
 * mean precision^-1 [X^T eps_g / gamma_g - (beta_g - theta) / sigma^2]).
 * Philox counter (g, 11 << 24, m, chain << 16 | j); Box-Muller pairs on words
 * (2p, 2p + 1).  It leaves the posterior invariant and removes the slow
 * exchange between eps_g and beta_g that the one-at-a-time conditionals have
 * when the counts pin their sum.
 *
 * Exact conjugate draws (bit 1 << FB_KIND_EXACT, off unless asked for):
 * Section 4.2 slice-samples the gamma and inverse-gamma full conditionals and
 * names a gamma sampler as the alternative.  With this bit, gamma_g ~
 * IG(nu/2 + N/2, nu tau/2 + S_g/2), tau ~ Gamma(a + G nu/2, rate b + (nu/2)
 * sum 1/gamma) and sigma_l^2 ~ IG((G-1)/2, S_l/2) truncated to (0, s_l^2)
 * are drawn directly (each only when its own bit is set) from Gamma variates
 * by the method of Marsaglia and Tsang (ACM TOMS 26(3), 2000), in FP64 in
 * both precision modes.  Attempt k of a draw reads Philox block (g, 12 << 24
 * | sub, m, chain << 16 | k), sub = 0 for gamma_g, 1 for tau, 2 + l for
 * sigma_l^2: words 0 and 1 give the normal (Box-Muller), word 2 the
 * acceptance uniform, word 3 the U^(1/alpha) factor used when the shape is
 * below 1.  After 64 failed attempts (or a shape <= 0, e.g. sigma^2 with
 * G = 1) the parameter takes its slice step.  fb_debug_counts records an
 * exact draw as (K_L, left, right, candidates) = (-1, 0, 0, attempts). */
#define FB_UPDATE_ALL 0xFEu

/* Prior constants of Section 4.1: tau ~ Gamma(a, rate b), nu ~ U(0, d),
 * theta_l ~ N(0, c[l]^2), sigma_l ~ U(0, s[l]).  The paper uses
 * a = b = 1, d = 1000, c_l = 10, s_l = 100 (fb_default_priors). */
typedef struct {
    double a, b, d;
    const double *c;   /* [L] */
    const double *s;   /* [L] */
} fb_priors;

typedef struct {
    int32_t chains;         /* independent chains per dataset (>= 1); chain k uses counter word chain = k */
    int64_t burnin;         /* M_B: sweeps 1..M_B tune the slice widths; moments use sweeps > M_B */
    int64_t tune_start;     /* M_C < M_B: widths are recomputed only for M_C < m <= M_B */
    int32_t max_steps;      /* K of Algorithm 2: one of 0, 1, 3, 7, 15 */
    double w0;              /* initial slice width of every parameter (> 0) */
    int32_t shrink_cap;     /* maximum shrink candidates per draw (>= 1) */
    int32_t precision;      /* enum fb_precision */
    uint32_t update_mask;   /* bit (1 << kind) enables that Gibbs step; FB_UPDATE_ALL */
    int32_t thin;           /* record a trace point every `thin` sweeps; 0 = no trace */
    int32_t trace_genes;    /* genes per segment whose gamma and beta are traced */
    int32_t trace_after_burnin; /* 1: record only sweeps m > M_B */
    int64_t trace_capacity; /* trace points kept on the device per segment */
    int32_t debug_counts;   /* 1: keep per-draw integer records of the last sweep */
    int32_t jitter;         /* 1: chains > 0 start from seeded jittered values */
    void *stream;           /* hipStream_t to use, or NULL */
    /* Device memory of the context (its arrays, and the temporaries of
     * fb_autotune and fb_features): with both NULL (the default) the library
     * calls hipMalloc and hipFree; otherwise the caller's allocator, e.g.
     * PyTorch's caching allocator: dev_alloc(bytes, alloc_user) returns
     * device memory of the current device, 256-byte aligned, or NULL
     * (FB_ENOMEM); dev_free(ptr, alloc_user) takes back what dev_alloc gave,
     * after the context's stream has finished using it (fb_destroy
     * synchronises first).  The library synchronises the device after each
     * dev_alloc, so a block that a caching allocator hands out while work of
     * its previous user is still queued on another stream is safe to use.
     * Set both or neither (FB_EINVAL).  The functions must stay callable
     * until fb_destroy returns. */
    void *(*dev_alloc)(size_t bytes, void *alloc_user);
    void (*dev_free)(void *ptr, void *alloc_user);
    void *alloc_user;
} fb_options;

/* One dataset of a batch: counts [G][N] (row g = gene), X [N][L], h [N]. */
typedef struct {
    const int32_t *counts;
    int64_t G;
    int32_t N;
    const double *X;
    int32_t L;
    const double *h;
    const fb_priors *priors;  /* NULL = the paper's constants */
    uint64_t seed;
} fb_dataset;

typedef struct fb_ctx fb_ctx;

/* Fill *o with the defaults: 1 chain, M_B = 1000, M_C = 100, K = 15, w0 = 1,
 * shrink_cap = 200, FP64, all steps, no trace, no debug records. */
void fb_default_options(fb_options *o);

/* Create a sampler for one dataset (Section 4.1).
 *   counts: [G][N] int32 >= 0;  X: [N][L] finite;  h: [N] finite offsets;
 *   pri: NULL for the paper's constants;  seed: Philox key;  opt: NULL = defaults.
 * Requires 1 <= L <= N <= FB_MAX_N, L <= FB_MAX_L, at most FB_MAX_ROWS distinct
 * rows in X and FB_MAX_COLVALS distinct non-zero values per column; a, b, d,
 * c_l, s_l > 0.  Starting values: per-gene least squares of log(1 + y) - h on X
 * for beta, eps = 0, gamma from the residual variance, theta and sigma^2 from
 * the spread of the beta, tau = mean gamma, nu = 10 (jittered for chains > 0 if
 * opt->jitter).  The chains of one dataset form its segments 0..C-1.
 * Errors: FB_EINVAL, FB_ENOMEM, FB_EDEVICE; *out is NULL on failure. */
int fb_create(fb_ctx **out, const int32_t *counts, int64_t G, int32_t N, const double *X,
              int32_t L, const double *h, const fb_priors *pri, uint64_t seed,
              const fb_options *opt);

/* Create one sampler over n_datasets datasets (each with opt->chains chains)
 * that advance together: segment k * chains + c is chain c of dataset k. */
int fb_create_batch(fb_ctx **out, const fb_dataset *ds, int32_t n_datasets,
                    const fb_options *opt);

/* Free everything; fb_destroy(NULL) is a no-op. */
void fb_destroy(fb_ctx *c);

/* Enqueue n >= 0 sweeps of Algorithm 1 on every segment (sweep index m advances
 * by n).  Returns FB_ENUMERIC if an earlier sweep raised the numeric flag. */
int fb_sweep(fb_ctx *c, int64_t n);

/* Wait for all enqueued work; returns the sticky error status.  When a slice
 * draw reached the shrink cap (FB_ENUMERIC), fb_last_error names the first
 * such draw: its kind (eps, gamma, beta, hyperparameter), dataset, chain,
 * gene, sweep and index (the sample n for eps; for a hyperparameter 0 for
 * the (nu, tau) draws, 1 + l for (theta_l, sigma_l^2)). */
int fb_sync(fb_ctx *c);

/* Number of segments, and the shape of segment seg. */
int32_t fb_num_segments(const fb_ctx *c);
int fb_segment_dims(const fb_ctx *c, int32_t seg, int64_t *G, int32_t *N, int32_t *L,
                    int32_t *dataset, int32_t *chain);

/* Full state of one segment in row-major host arrays (any pointer may be NULL to
 * skip that block):  eps [G][N], gamma [G], beta [G][L],
 * hyp [2 + 2L] = (nu, tau, theta_1..L, sigma^2_1..L); slice widths w and their
 * tuning sums waux with the same shapes, and for the hyperparameters
 * w_hyp / waux_hyp [2 + L] = (nu, tau, sigma^2_1..L).  m = sweeps completed. */
typedef struct {
    double *eps, *gam, *beta, *hyp;
    double *w_eps, *waux_eps, *w_gam, *waux_gam, *w_beta, *waux_beta, *w_hyp, *waux_hyp;
    int64_t m;
} fb_state;

int fb_get_state(fb_ctx *c, int32_t seg, fb_state *s);
/* Writes every non-NULL block and sets the sweep counter of the whole context
 * to s->m.  Rejects values outside the support (gamma, tau, sigma^2, widths
 * must be > 0, 0 < nu < d, sigma^2_l < s_l^2, everything finite). */
int fb_set_state(fb_ctx *c, int32_t seg, const fb_state *s);

/* Running means and means of squares (FP64) of one segment, same shapes as
 * fb_state; count = number of sweeps averaged (m - M_B once m > M_B).  Clears
 * nothing.  NULL pointers skip a block.
 * Acceptance statistics of the independence-MH beta step (Section 2.1's
 * remark on independence proposals; fb_set_beta_update), per gene [G]:
 * imh_steps = sampling sweeps (m > M_B) in which beta_g took the IMH step,
 * imh_accepts = how many of those steps accepted the proposal; their ratio is
 * the gene's acceptance rate.  Genes on the slice steps (plain sweep, fallback
 * genes) count no steps; the slice draws themselves always move.  The counts
 * restart, as the moments do, with the first sampling sweep after fb_set_state
 * sets m <= M_B; zero before the IMH step is first configured. */
typedef struct {
    double *mean_eps, *msq_eps, *mean_gam, *msq_gam, *mean_beta, *msq_beta;
    double *mean_hyp, *msq_hyp;
    int64_t count;
    int64_t *imh_steps, *imh_accepts;
} fb_summary;

int fb_summaries(fb_ctx *c, int32_t seg, fb_summary *s);

/* Trace (Section 3.1: thinned samples of the hyperparameters and of a few
 * genes).  Each point of segment seg holds 2 + 2L + T (L + 1) floats:
 * hyp (nu, tau, theta, sigma^2), then for each traced gene gamma, beta_1..L.
 * Points are recorded on sweeps m with m % thin == 0 (and m > M_B when
 * trace_after_burnin), into rows 0, 1, ... of a device buffer of
 * trace_capacity points shared in numbering by all segments.
 * fb_trace_genes writes the T traced gene indices (ascending).
 * fb_trace copies the first min(recorded, cap) points of segment seg into buf
 * ([points][2 + 2L + T (L + 1)] floats) and sets *n_out (with buf = NULL it
 * only reports the number recorded); *dropped counts sweeps not recorded
 * because the buffer was full.  fb_trace_reset forgets every recorded point. */
int fb_trace_genes(const fb_ctx *c, int32_t seg, int64_t *genes, int32_t *T);
int fb_trace(fb_ctx *c, int32_t seg, float *buf, int64_t cap, int64_t *n_out,
             int64_t *dropped);
int fb_trace_reset(fb_ctx *c);

/* Per-draw integer records of the last sweep when opt.debug_counts = 1:
 * 4 int32 per slice draw (K_L, left moves, right moves, shrink candidates):
 * eps [G][N][4], gamma [G][4], beta [G][L][4], hyp [2 + L][4] (nu, tau, sigma^2). */
int fb_debug_counts(fb_ctx *c, int32_t seg, int32_t *eps, int32_t *gam, int32_t *beta,
                    int32_t *hyp);

/* The reductions the last hyperparameter step used (FP64):
 * [sum log gamma, sum 1/gamma, then per l: sum beta_l, sum (beta_l - theta_l)^2]. */
int fb_reductions(fb_ctx *c, int32_t seg, double *out);

/* Philox4x32-10 words computed on the device: ctr [n][4], key [n][2], out [n][4]. */
int fb_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n);

/* Time of the last fb_sweep batch measured with HIP events around all its
 * launches (milliseconds), and the number of sweeps in it. */
int fb_last_sweep_time(fb_ctx *c, double *ms, int64_t *sweeps);

/* Sampled kernel timing with HIP events on the context's stream.  A sweep is
 * two to four launches: the eps kernel (Algorithm 1 step 1), the gamma/beta
 * kernel (steps 2 and 5), the shift kernel when that step is on, and the
 * hyperparameter step (steps 3, 4, 6, 7), which either rides in the next
 * sweep's eps kernel (fused, the eps time includes it) or is a kernel of its
 * own (see fb_set_launch).  From now on the launches of every `every`-th sweep
 * are bracketed by events, for at most max_samples sweeps (every = 0 turns it
 * off).  fb_kernel_times waits for the stream, returns the mean duration (ms)
 * of the sampled eps, gamma/beta, separate hyperparameter (0 when fused) and
 * shift (0 when off) launches and the number of samples, and starts a new
 * sample set.  Null output pointers are skipped. */
int fb_profile(fb_ctx *c, int32_t every, int32_t max_samples);
int fb_kernel_times(fb_ctx *c, double *eps_ms, double *gb_ms, double *hyper_ms, double *shift_ms,
                    int64_t *samples);

/* Posterior probabilities of contrast events (Section 3.2).  Event e
 * (0 <= e < n_events <= 8) holds for gene g at a sweep when every row r with
 * row_event[r] == e satisfies sum_l v[r][l] beta_gl > b[r] (v is [n_rows][L],
 * n_events <= n_rows <= 16, every event has a row; L is the context's, so all
 * of its datasets must share it).  From the next sweep on, every post-burn-in
 * sweep adds 1 to count[g][e] when event e holds on that sweep's final beta_g
 * (after the shift step when it is on); the estimate of the probability is
 * count / n_sweeps.  A new call replaces the events and restarts the counts.
 * fb_event_counts fills counts [G][n_events] of segment `seg` (caller-
 * allocated, NULL skips) and n_sweeps, the sweeps counted.  The library copies
 * the arguments.  Errors: FB_EINVAL, FB_ENOMEM, FB_EDEVICE. */
int fb_set_contrasts(fb_ctx *c, int32_t n_events, int32_t n_rows, const int32_t *row_event, const double *v,
                     const double *b);
int fb_event_counts(fb_ctx *c, int32_t seg, int32_t *counts, int64_t *n_sweeps);

/* Three-level form (Section 2.3).  The datasets of a batched context become
 * the groups k of a three-level hierarchy: each keeps its own hyperparameters
 * phi_k = (nu_k, tau_k, theta_k, sigma_k^2), whose priors are tied by a top
 * level psi = (b, psi_1..psi_L) per chain:
 *   tau_k ~ Gamma(a_k, rate b),   theta_kl ~ N(psi_l, c_kl^2),
 *   b ~ Gamma(a_b, rate b_b),     psi_l ~ N(0, c0_l^2)
 * (a_k, c_kl from each dataset's fb_priors; b of fb_priors and the prior mean
 * 0 of theta are replaced by the top level).  Each sweep draws psi(m) from the
 * groups' phi(m - 1) -- given phi the top level is independent of the genes,
 * the paper's (mu, psi) | phi step -- then the genes and phi_k(m) given psi(m)
 * as before.  Both top-level conditionals are conjugate and drawn exactly from
 * reductions over the groups:
 *   b     ~ Gamma(a_b + sum_k a_k, rate b_b + sum_k tau_k)
 *   psi_l ~ N(v sum_k theta_kl / c_kl^2, v),  1/v = 1/c0_l^2 + sum_k 1/c_kl^2
 * Philox counter (0, 13 << 24 | sub, m, chain << 16 | j), key = `seed`: psi_l
 * sub = l, Box-Muller on words 0 and 1 of block 0; b sub = 128, a Gamma
 * variate as in the exact conjugate draws (attempt j in block j; b keeps its
 * value if all 64 attempts fail).  `mask` bit 0 draws b, bit 1 the psi_l
 * (3: both; others hold them fixed).  Sums run over the datasets in order.
 *
 * fb_set_top_level(c, p) turns the top level on (p != NULL) or off (NULL); on,
 * it starts at b = the first dataset's prior rate and psi = 0 for every chain
 * and needs every dataset to have the same L.  It must be called before burn-in
 * ends (the running moments of b and psi start at M_B).  fb_get_top copies the
 * chain's b, psi [L], the running means and means of squares [1 + L] (b, then
 * psi) and the attempts of the last b draw (any pointer may be NULL);
 * fb_set_top replaces b and psi.  Errors: FB_EINVAL (bad arguments, no top
 * level, different L, after burn-in), FB_ENOMEM, FB_EDEVICE. */
typedef struct {
    double a_b, b_b;       /* b ~ Gamma(a_b, rate b_b) */
    const double *c0;      /* [L]: psi_l ~ N(0, c0[l]^2) */
    uint64_t seed;         /* Philox key of the top-level draws */
    uint32_t mask;         /* bit 0: draw b, bit 1: draw psi */
} fb_top_priors;
int fb_set_top_level(fb_ctx *c, const fb_top_priors *p);
int fb_get_top(fb_ctx *c, int32_t chain, double *b, double *psi, double *mean, double *msq, int32_t *tries);
int fb_set_top(fb_ctx *c, int32_t chain, double b, const double *psi);

/* Graph replay of the sweep (HIP graphs).  With sweeps > 0, fb_sweep(n) runs
 * n / sweeps chunks (integer division) of `sweeps` sweeps each as one replay of
 * a captured HIP graph of the chunk's launches, and the remaining sweeps with
 * direct launches.  Before each replay the chunk's per-sweep arguments (sweep
 * index, trace rows, training-pair rows, ...) are copied from pinned host
 * memory to a device array that the captured kernels read, so one capture
 * serves every chunk; the chunk is captured again only when the launch shape,
 * the buffers or the set of kernels changes (e.g. fb_set_launch, the learned
 * step).  The draws are those of direct launches, bit for bit.  While
 * fb_profile samples, sweeps launch directly.  sweeps = 0 turns replay off.
 * Limits: 0 <= sweeps <= 4096.  The graph records no memset nodes.
 * Errors: FB_EINVAL, FB_ENOMEM, FB_EDEVICE.  fb_get_graph returns the current
 * setting (0 when off or for NULL). */
int fb_set_graph(fb_ctx *c, int32_t sweeps);
int32_t fb_get_graph(const fb_ctx *c);

/* Launch shape of a sweep; no choice changes any draw (the draws are functions
 * of their counters only).
 *   samples_per_wave  eps draws per lane, in sample order (1 .. max N): a
 *                     wavefront covers 64 genes x this many samples
 *   fuse_hyper        1: the hyperparameter step of sweep m runs in the first
 *                     workgroups of sweep m + 1's eps kernel (no eps conditional
 *                     involves a hyperparameter); 0: a kernel of its own
 * Defaults: 1 and 1.  FB_EINVAL outside these values. */
int fb_set_launch(fb_ctx *c, int32_t samples_per_wave, int32_t fuse_hyper);
/* With the shift step on, the slice sweep runs the gamma, beta and shift draws
 * of a tile in one kernel (fused = 1, the default: a tile's shift overlaps
 * other tiles' beta draws) or the shift as a kernel of its own after the
 * gamma/beta kernel (0).  The learned step always uses the separate kernel.
 * No choice changes any draw.  Errors: FB_EINVAL. */
int fb_set_shift_fusion(fb_ctx *c, int32_t fused);
/* Lanes per gene in the beta draws of the slice sweep (with the shift step
 * when it runs inside the gamma/beta kernel): 1 (one lane per gene) or 2 (a
 * pair of lanes: both step-out
 * directions at once and shrink candidates two at a time -- fewer dependent
 * trips per gene where few tiles share the chip, more work per gene where
 * many do).  fb_autotune tries both.  No choice changes any draw.
 * fb_get_beta_lanes returns the setting (0 for NULL).  Errors: FB_EINVAL. */
int fb_set_beta_lanes(fb_ctx *c, int32_t lanes);
int32_t fb_get_beta_lanes(const fb_ctx *c);
/* Workgroups of the hyperparameter step (Algorithm 1 steps 3, 4, 6 and 7),
 * fused into the next eps launch or as its own kernel: on = 1 (the default)
 * runs 1 + L workgroups per segment, one per chain of draws (nu then tau;
 * theta_l then sigma_l^2), each reducing only the two partial sums it needs,
 * so the chains run at once; on = 0 runs the whole step on one workgroup per
 * segment.  The sums are added in the same order either way, so no choice
 * changes any draw.  fb_autotune leaves the setting as it is (the split was
 * faster or level at every measured shape).  fb_get_hyper_split returns the
 * setting (0 for NULL).  Errors: FB_EINVAL. */
int fb_set_hyper_split(fb_ctx *c, int32_t on);
int32_t fb_get_hyper_split(const fb_ctx *c);
int fb_get_launch(const fb_ctx *c, int32_t *samples_per_wave, int32_t *fuse_hyper);
/* Single-launch sweep (on = 1): the slice sweep with one lane per gene for
 * beta and no shift step runs as one kernel per sweep instead of two.  One
 * workgroup per 64-gene tile draws the tile's eps_gn (Algorithm 1 step 1) on
 * four wavefronts, keeps the new values in LDS, and after a barrier draws
 * gamma_g (step 2) and beta_g (step 5) from them; the previous sweep's
 * hyperparameter step (steps 3, 4, 6, 7) runs in the launch's first
 * workgroups while the tiles draw eps, and the gamma and beta draws wait for
 * it through a per-segment flag in device memory (a bounded wait: should it
 * ever time out, the sticky status becomes FB_EDEVICE).  The draws are those
 * of the two-kernel sweep, bit for bit; samples_per_wave does not apply (a
 * wavefront takes ceil(N / 4) samples).  Other sweeps (shift step, two beta
 * lanes, learned or Laplace step) keep their kernels.  fb_autotune tries it.
 * Default 0.  fb_get_tile_sweep returns the setting (0 for NULL).
 * With it on, fb_kernel_times reports the whole launch as the eps time and
 * 0 for the gamma/beta kernel.  Errors: FB_EINVAL. */
int fb_set_tile_sweep(fb_ctx *c, int32_t on);
int32_t fb_get_tile_sweep(const fb_ctx *c);

/* Autotuner: times trial_sweeps sweeps (after 2 warm-up sweeps) for every
 * samples_per_wave in {1, 2, 4, 8} (up to max N), with and without fusion,
 * starting each trial from a device snapshot of the state, then restores the
 * snapshot and keeps the fastest shape.  The chain continues exactly as if no trial had run (traces
 * and training pairs are not written by the trials; the time reported by
 * fb_last_sweep_time is the last trial's).  Outputs (each may be NULL): the
 * chosen shape, its time per sweep (ms), and table[10], the time per sweep of shape
 * k = 2 log2(samples_per_wave) + fuse_hyper (k < 8, two-kernel sweep, current
 * beta lanes), then the single-launch sweep (fb_set_tile_sweep) with
 * fuse_hyper 1 (k = 8) and 0 (k = 9), tried for the plain slice sweep; -1 if
 * not tried.  If a two-kernel shape wins, with the slice steps for beta (and the shift step,
 * if on, inside the gamma/beta kernel) it then times the other number of beta
 * lanes (fb_set_beta_lanes) at the chosen shape and keeps the faster;
 * ms_per_sweep is the time of the final choice.  The single-launch setting
 * is left at the choice (fb_get_tile_sweep).
 * Needs device memory for one copy of the state. */
int fb_autotune(fb_ctx *c, int32_t trial_sweeps, int32_t *samples_per_wave, int32_t *fuse_hyper,
                double *ms_per_sweep, double *table);

/* ------------------------------------------------------------------------
 * Learned beta proposal (independence Metropolis-Hastings for the block beta_g)
 *
 * A network maps 32 features of gene g -- for each distinct row r of X,
 * log((Y_r + 1/2) / A_r) and log(Y_r + 1/2) with Y_r the row's count sum and
 * A_r = sum over the row's samples of exp(h_n + eps_gn); then theta_l and
 * log sigma_l^2; zero-padded -- to a correction of the Laplace approximation
 * N(bh, H^-1) of the beta_g conditional.  bh and H = U U^T come from the same
 * sufficient statistics (a weighted least-squares start, two Newton steps, the
 * negative Hessian at the last iterate); in the whitened coordinates
 * w = U^T (b - bh) the network gives w ~ N(mu, Lc Lc^T), so
 * beta* = bh + U^-T (mu + Lc z).  The features never involve beta_g, so one
 * step with exact acceptance probability leaves the beta_g full conditional
 * invariant.  Network: x = (phi - fmean) * fscale, each element clipped to
 * [-8, 8] (the range the training inputs are clipped to); h1 = gelu(x W1 + b1);
 * h2 = gelu(h1 W2 + b2); o = h2 W3 + b3 (O = 2L + L(L-1)/2 outputs used);
 *   mu_l = omean_l + oscale_l o_l,
 *   Lc_ll = exp(ls_l), ls_l = log(oscale_l) + o_{L+l},
 *   Lc_lj = oscale_l o_{2L + l(l-1)/2 + j} for j < l
 * (gelu in the erf form; a zero network with omean = 0, oscale = 1 leaves the
 * Laplace proposal).  Products run on the matrix cores with BF16 operands and
 * FP32 accumulation; parameters are kept in FP32.
 * ---------------------------------------------------------------------- */
enum fb_beta_update { FB_BETA_SLICE = 0, FB_BETA_LEARNED = 1, FB_BETA_LAPLACE = 2 };

/* Host arrays of the network's parameters (FP32, row-major, input index first). */
typedef struct {
    float *fmean, *fscale;   /* [32] input standardisation */
    float *W1, *b1;          /* [32][128], [128] */
    float *W2, *b2;          /* [128][128], [128] */
    float *W3, *b3;          /* [128][64], [64]; outputs >= 2L + L(L-1)/2 are unused */
    float *omean, *oscale;   /* [8]; the first L are used */
} fb_mlp;

typedef struct {
    int32_t epochs;           /* passes over pairs_per_epoch sampled pairs */
    int32_t pairs_per_epoch;  /* pairs drawn (with replacement) per epoch */
    int32_t minibatch;        /* Adam step size in pairs, a multiple of 32 */
    double lr;                /* Adam learning rate */
    uint64_t seed;            /* initial weights and minibatch sampling */
} fb_train_opts;

/* epochs 200, 10240 pairs per epoch, minibatch 1024, lr 1e-3, seed 1. */
void fb_default_train_opts(fb_train_opts *o);

/* Run `sweeps` sweeps with slice draws for beta and, on every sweep whose index
 * is a multiple of `every`, store (features, whitened new beta_g) of every gene
 * of every segment as training pairs (earlier pairs are discarded). */
int fb_proposal_collect(fb_ctx *c, int64_t sweeps, int32_t every);
/* Train the network on the stored pairs with the project's own device kernels:
 * input standardisation from the pairs' feature means and sds, the output map
 * at the identity (omean 0, oscale 1: the targets are already whitened by the
 * Laplace approximation), seeded initial weights for the hidden layers and a
 * zero output layer (so the untrained network is the Laplace proposal), Adam
 * on the mean Gaussian negative log likelihood of the whitened beta given the
 * features.
 * epoch_loss (may be NULL) receives the mean training loss of each epoch. */
int fb_proposal_train(fb_ctx *c, const fb_train_opts *o, double *epoch_loss);
/* Run `sweeps` sweeps in which every gene of every segment takes the IMH
 * step, then set the fallback mask: genes whose acceptance rate was below
 * min_accept keep the slice steps from now on.  Adaptive: call it during
 * burn-in only.  With FB_BETA_LAPLACE set it calibrates the Laplace-only
 * proposal (no network needed), otherwise the network's. */
int fb_proposal_calibrate(fb_ctx *c, int64_t sweeps, double min_accept);
/* FB_BETA_SLICE, FB_BETA_LEARNED (needs a trained or loaded network), or
 * FB_BETA_LAPLACE: the same independence-MH step with the per-gene Laplace
 * approximation alone as the proposal (the network's correction set to the
 * identity; no network kernel runs) -- the ablation that shows what the
 * network adds.  Fallback genes keep the slice steps in either IMH mode. */
int fb_set_beta_update(fb_ctx *c, int32_t mode);
/* Copy the network's parameters out, or load new ones (both host arrays). */
int fb_proposal_get(fb_ctx *c, fb_mlp *out);
int fb_proposal_set(fb_ctx *c, const fb_mlp *in);
/* Per-gene fallback mask of a segment (1 = slice), read or written. */
int fb_fallback(fb_ctx *c, int32_t seg, int32_t *get, const int32_t *set);
/* Last sweep's beta step per gene: 1 IMH accepted, 0 rejected, -1 slice. */
int fb_imh_last(fb_ctx *c, int32_t seg, int32_t *last);
/* Features of every gene of segment seg computed on the device from its
 * current state ([G][32]). */
int fb_features(fb_ctx *c, int32_t seg, float *phi);

/* Device kernels of the network on host data (tests): one matrix-core product
 * of A [32][16] and B [16][32] into C [32][32]; the network's outputs for raw
 * features phi [B][32] (mu, ls: [B][L]; off: [B][L(L-1)/2], the factor's
 * strict lower triangle in units of oscale, row-major; off may be NULL); and
 * the mean loss sum_l ls_l + |u|^2 / 2 (Lc u = target - mu) and its gradients
 * for targets [B][L] (B a multiple of 32; gradients of fmean, fscale, omean,
 * oscale are zero). */
int fb_mfma_probe(const float *A, const float *B, float *C);
int fb_mlp_forward(const fb_mlp *w, int32_t L, const float *phi, int64_t B, float *mu, float *ls,
                   float *off);
int fb_mlp_loss_grad(const fb_mlp *w, int32_t L, const float *phi, const float *target, int64_t B,
                     float *loss, fb_mlp *grad);

/* Allocation-free loss and gradients, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight training or serving loops,
 * harnesses that forbid hipMalloc.  The result is that of fb_mlp_loss_grad,
 * here on device buffers the caller owns:
 *   master  [FB_MLP_PARAMS] floats, 16-byte aligned, the fb_mlp blocks one
 *           after another in the order fmean[32], fscale[32], W1[32][128],
 *           b1[128], W2[128][128], b2[128], W3[128][64], b3[64], omean[8],
 *           oscale[8];
 *   phi     [B][32] raw features;  target [B][L] whitened targets;
 *   loss    one float, the mean loss;  grad [FB_MLP_PARAMS], same layout
 *           (zero for fmean, fscale, omean, oscale).
 * 32 <= B <= FB_NOALLOC_MAX_ROWS, B a multiple of 32; 1 <= L <= FB_MAX_L.
 * Intermediate results (standardised inputs, activations, backward
 * temporaries, per-row losses) live in a static device array of
 * FB_NOALLOC_MAX_ROWS x 1057 floats (8.3 MiB), which each GPU the library runs
 * on holds until the process ends; no call allocates or frees memory.  The
 * work is enqueued on `stream` (a hipStream_t; NULL = the null stream) of the
 * current device and the call returns without waiting; outputs are valid once
 * the stream has reached that point.  Every call on one GPU shares that GPU's
 * array, so calls that may overlap on one GPU (other streams, other threads)
 * race; calls in order on one stream do not.  The first call on each device
 * looks up the array's device address (do it once outside graph capture).
 * Errors: FB_EINVAL (null pointer, master not 16-byte aligned, L or B out of
 * range, B above FB_NOALLOC_MAX_ROWS), FB_EDEVICE (a HIP call failed);
 * message in fb_last_error(NULL). */
#define FB_MLP_PARAMS        29072
#define FB_NOALLOC_MAX_ROWS  2048
int fb_mlp_loss_grad_noalloc(const float *master, int32_t L, const float *phi, const float *target, int64_t B,
                             float *loss, float *grad, void *stream);

const char *fb_last_error(const fb_ctx *c);
const char *fb_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* LIBFBMC_H */
