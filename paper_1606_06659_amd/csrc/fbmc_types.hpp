// fbmc_types.hpp -- device-visible tables of libfbmc, shared by host and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fbmc {

constexpr int kMaxN = 64;      // samples per dataset
constexpr int kMaxL = 8;       // model-matrix columns
constexpr int kMaxRows = 8;    // distinct rows of X
constexpr int kMaxVals = 4;    // distinct non-zero values per column
constexpr int kTile = 64;      // genes per wavefront tile
constexpr int kMaxParts = 2 + 2 * kMaxL;
constexpr int kHypFlags = 1 + kMaxL;
constexpr int kColChunks = 128;          // row ranges of the pairs' column moments (launch_col_moments)     // chains of hyperparameter draws: (nu, tau), (theta_l, sigma_l^2)
constexpr int kKindShift = 11;  // Philox kind and update_mask bit of the shift step
constexpr int kKindExact = 12;  // update_mask bit of the exact conjugate draws (gamma, tau, sigma^2)
constexpr int kKindTop = 13;    // Philox kind of the top-level draws (three-level form)
constexpr int kMaxEv = 8;       // contrast events per context
constexpr int kMaxCtr = 16;     // contrast rows (inequalities) over all events

// Top level of the three-level form (Section 2.3), one per chain: the groups
// (datasets) of the chain have tau_k ~ Gamma(a_k, rate b) and theta_kl ~
// N(psi_l, c_kl^2), with b ~ Gamma(a_b, rate b_b) and psi_l ~ N(0, c0_l^2).
struct TopState {
    double b;
    double psi[kMaxL];
    double2 mom[1 + kMaxL];       // b, psi[L]: running mean and mean of squares after burn-in
    int32_t tries;                // attempts of the last b draw (0: none succeeded, b kept)
    int32_t pad;
};

struct TopPriors {
    double a_b, b_b;
    double c0[kMaxL];
    uint32_t key0, key1;          // Philox key of the top-level draws
    int32_t L;
    uint32_t mask;                // bit 0: draw b, bit 1: draw psi
};

// Per-segment (dataset x chain) description.  Lives in device memory and is
// read with wavefront-uniform loads.  Arrays of state are gene-contiguous
// (structure of arrays): element (k, g) of a [K][Gp] array sits at k*Gp + g.
struct SegInfo {
    int64_t G;          // genes
    int64_t Gp;         // padded to a multiple of kTile
    int64_t ntiles;     // Gp / kTile
    int32_t N, L, R;    // samples, columns, distinct rows of X
    int32_t chain;
    uint32_t key0, key1;          // Philox key = the dataset seed
    int32_t dataset;
    int32_t trace_T;              // traced genes
    int32_t trace_stride;         // floats per trace point
    int32_t pad0;
    // design, in the kernel's working precision-independent form
    double X[kMaxN * kMaxL];      // [N][L]
    double h[kMaxN];
    double eh[kMaxN];             // exp(h_n)
    int32_t row_of[kMaxN];        // distinct-row index of sample n
    double Xrow[kMaxRows * kMaxL];// [R][L] distinct rows
    int32_t xidx[kMaxRows * kMaxL];// [R][L]: index of X_rl among the column's non-zero values, -1 if 0
    int32_t nv[kMaxL];            // distinct non-zero values of column l
    int32_t pm[kMaxL];            // 1: those values are exactly {v, -v} (v first)
    double vals[kMaxL * kMaxVals];// [L][kMaxVals]
    double XtX[kMaxL * kMaxL];    // [L][L] sum_n X_n^T X_n (shift step)
    // prior constants (Section 4.1)
    double a, b, d;
    double c[kMaxL], s[kMaxL];
    // contrast events (Section 3.2): event e holds when every row r with
    // crow_event[r] == e has sum_l cv[r][l] beta_gl > cb[r]; ev_count[e][g]
    // counts the sweeps m > max(M_B, ev_from) where it held for gene g
    int32_t n_ev, n_crow;
    int64_t ev_from;
    int32_t crow_event[kMaxCtr];
    double cv[kMaxCtr * kMaxL];   // [n_crow][kMaxL]
    double cb[kMaxCtr];
    int32_t *ev_count;            // [kMaxEv][Gp]
    // device pointers
    const int32_t *y;             // [N][Gp]
    void *eps, *w_eps, *wa_eps;   // [N][Gp] (float or double)
    void *gam, *w_gam, *wa_gam;   // [Gp]
    void *beta, *w_beta, *wa_beta;// [L][Gp]
    double2 *mom_eps;             // [N][Gp]  (mean, mean of squares)
    double2 *mom_gam;             // [Gp]
    double2 *mom_beta;            // [L][Gp]
    double *partials;             // [kMaxParts][pstride] (part-major): tiles, then fallback groups
    int64_t pstride;              // columns of the partials array: 2 ntiles
    const int32_t *fb_genes;      // learned step: genes that keep the slice steps, ascending
    int32_t nfbw;                 // learned step: fallback groups (<= 64 genes each) of this segment
    int32_t pad1;
    int32_t *trace_slot;          // [Gp] slot of traced genes, -1 otherwise
    float *trace;                 // [capacity][trace_stride]
    int4 *dbg_eps, *dbg_gam, *dbg_beta;  // per-draw records [N][Gp], [Gp], [L][Gp]
    struct HyperState *hyp;
    // split sweep (eps/gamma, then beta) used by the learned proposal
    void *Ar;                     // [R][Gp] sum over row r of exp(h_n + eps_gn), this sweep
    void *YR;                     // [R][Gp] sum over row r of y_gn (constant)
    float *mlp_out;               // [2L + L(L-1)/2][Gp] the proposal network's outputs, this sweep
    int32_t *fallback;            // [Gp] 1 = slice step for beta_g
    int32_t *imh_count;           // [Gp] accepted IMH steps while counting
    int32_t *imh_last;            // [Gp] last sweep: 1 accepted, 0 rejected, -1 slice
    int2 *imh_stat;               // [Gp] over the sweeps m > M_B: (IMH steps taken, accepted)
    float *pairs;                 // training pairs [capacity][kPairStride]: features, beta
    const TopState *top;          // three-level form: the chain's top level (b, psi), else null
    // single-launch sweep: per chain of hyperparameter draws c (0: nu, tau;
    // 1 + l: theta_l, sigma_l^2), the sweep index whose values of that chain
    // the segment's HyperState holds, published by the hyperparameter step
    // that runs in the first workgroups of that launch ([kHypFlags])
    int64_t *hyp_flag;
};

constexpr int kPairStride = 32 + kMaxL;   // 32 raw features then L targets

// FP64 hyperparameter state of one segment.
struct HyperState {
    double nu, tau;
    double theta[kMaxL], sig2[kMaxL];
    double w_nu, wa_nu, w_tau, wa_tau;
    double w_sig2[kMaxL], wa_sig2[kMaxL];
    double2 mom[2 + 2 * kMaxL];   // nu, tau, theta[L], sig2[L]
    double red[kMaxParts];        // reductions used by the last hyper step
    int4 dbg[2 + kMaxL];          // records of nu, tau, sig2[L]
};

// Arguments of one sweep that change from sweep to sweep.
struct SweepArgs {
    int64_t m;            // sweep index (1-based)
    int64_t burnin;       // M_B
    int64_t tune_start;   // M_C
    double inv_k;         // 1 / (m - M_B) once m > M_B: weight of the running moments
    int32_t K;            // step-out budget
    int32_t cap;          // shrink cap
    uint32_t mask;        // update mask
    int32_t trace_point;  // trace row to write this sweep, or -1
    int32_t dbg;          // write per-draw records
    int32_t learned;      // beta by independence MH where the fallback mask is 0
    int32_t count_imh;    // add accepted IMH steps to imh_count
    int32_t laplace;      // the IMH proposal is the Laplace base alone (no network outputs)
    int64_t pair_base;    // collect (features, beta) pairs at row pair_base + g, or -1
    // graph replay: when dev is set, the kernel takes its arguments from
    // dev[idx] (written before each replay) and ignores the fields above
    const SweepArgs *dev;
    int64_t idx;
};

// The arguments a kernel runs with: its own copy, or the one in device memory.
// Written as a copy and a branch on purpose: the conditional-operator form
// (a.dev ? a.dev[a.idx] : a), which selects between the kernel-argument copy
// and the device-memory copy by address, gave wrong independence-MH
// decisions in the FP64 learned gamma/beta kernel with this toolchain (the
// FP64 parity tests against the oracle catch it); this form matches.
__device__ inline SweepArgs resolve_args(const SweepArgs &a)
{
    SweepArgs r = a;
    if (a.dev != nullptr) r = a.dev[a.idx];
    return r;
}

}  // namespace fbmc
