// fbmc_kernels.hip -- the sweep kernels of libfbmc for gfx950.
//
// One sweep of Algorithm 1 is two launches on the context's stream:
//
//  eps_sweep<T>      step 1: one lane per (gene, sample); a wavefront draws
//                    eps_gn for a 64-gene tile and a run of samples.  Its first
//                    workgroups (1 + L per segment, one per chain of draws:
//                    nu then tau, theta_l then sigma_l^2 -- hyper_chain -- or
//                    one per segment, hyper_block) run the previous sweep's
//                    hyperparameter step: no eps conditional involves a
//                    hyperparameter.
//  gb_sweep<T, mode, kML>
//                    steps 2 and 5: one 128-thread workgroup per tile,
//                    wavefront 0 draws gamma_g and wavefront 1 beta_g1..beta_gL
//                    (slice steps, or one independence-MH step for the block
//                    with the learned or Laplace proposal), then the running
//                    moments and the tile's FP64 partial sums of log gamma,
//                    1/gamma, beta_l - theta_l and its square.
//
// Variants of the second launch: gb_pair_sweep (two lanes per gene for the
// beta draws), gb_shift_sweep (the shift step after a barrier in the same
// workgroup), shift_sweep (the shift step as a kernel of its own), and before
// it mlp_sweep (the proposal network) in the learned form.  hyper_sweep runs the
// hyperparameter step alone after the last sweep of a call, and top_sweep the
// top level of the three-level form.  Running steps 1, 2 and 5 before 3, 4, 6
// and 7 is the same Markov chain as the printed order: eps and beta do not
// depend on nu or tau, nu and tau not on beta, gamma not on theta or sigma^2,
// and with counter-based random numbers no draw changes either.
//
// Full conditionals (Section 4.1; the gene-level ones are evaluated as
// differences from the current value x0, which keeps float arithmetic away from
// cancellation between large terms):
//   eps:   log f(x) - log f(x0) = y d - mu0 expm1(d) - d (x0 + d/2) / gamma,
//          d = x - x0, mu0 = exp(h_n + x0 + X_n beta_g)
//   gamma: InvGamma(nu/2 + N/2, nu tau/2 + S_g/2), S_g = sum_n eps_gn^2
//   beta:  log f(x) - log f(x0) = Y_l d - sum_k G_k expm1(v_k d) - d (x0 - theta_l + d/2) / sigma_l^2
//          where Y_l = sum_n y_gn X_nl and G_k sums exp(h_n + eps_gn + X_n beta_g)
//          over the samples whose X_nl equals the k-th distinct non-zero value v_k
//          of column l (exact regrouping of the sum over n).
#include <type_traits>

#include "fbmc_device.hpp"
#include "fbmc_mlp.hpp"
#include "fbmc_types.hpp"


namespace fbmc {

// ---------------------------------------------------------------------------
// Log-density functors for slice_draw
// ---------------------------------------------------------------------------
template <typename T>
struct EpsF {
    T y, mu0, x0, inv_gam;
    __device__ T base(T) const { return (T)0; }
    __device__ T operator()(T x) {
        const T d = x - x0;
        return y * d - mu0 * dexpm1(d) - d * (x0 + (T)0.5 * d) * inv_gam;
    }
};

template <typename T>
struct GamF {
    T alpha1, scale, x0;
    __device__ T base(T) const { return (T)0; }
    __device__ T operator()(T x) {
        if (!(x > (T)0)) return neg_inf<T>();
        const T d = x - x0;
        return -alpha1 * dlog1p(d / x0) + scale * d / (x * x0);
    }
};

// kForm fixes the column's form at compile time so the slice loop carries no
// branch on it: 0 reads nv and pm at run time, 1 one non-zero value, -1 the
// +-v form (float); the arithmetic is the same in every form.
template <typename T, int kForm = 0>
struct BetaF {
    T Y, x0, dth, inv_s2;
    T Gk[kMaxVals], vk[kMaxVals];
    T em1[kMaxVals];   // expm1(v_k d) at the last evaluated point
    int nv;
    bool pm;           // the column's non-zero values are exactly v and -v
    __device__ T base(T) const { return (T)0; }
    __device__ T operator()(T x) {
        const T d = x - x0;
        T s = Y * d - d * (dth + (T)0.5 * d) * inv_s2;
        if constexpr (kForm == 1) {
            em1[0] = dexpm1(vk[0] * d);
            s -= Gk[0] * em1[0];
        } else if (std::is_same<T, float>::value && (kForm == -1 || (kForm == 0 && pm))) {
            // expm1(-v d) = -e / (1 + e) with e = expm1(v d): one exponential
            // for a +-v column (both rounding errors are a few ulp)
            const T e = dexpm1(vk[0] * d);
            em1[0] = e;
            em1[1] = -e * (T)__builtin_amdgcn_rcpf((float)((T)1 + e));
            s -= Gk[0] * em1[0];
            s -= Gk[1] * em1[1];
        } else {
#pragma unroll
            for (int k = 0; k < kMaxVals; ++k) {
                if (k < nv) {
                    em1[k] = dexpm1(vk[k] * d);
                    s -= Gk[k] * em1[k];
                }
            }
        }
        return s;
    }
};

// FP64 hyperparameter conditionals, evaluated in the plain (uncentred) form.
struct NuF {
    double G, tau, sum_log, sum_inv, d;
    __device__ double val(double x) const {
        if (!(x > 0.0) || !(x < d)) return -__builtin_inf();
        return -G * ::lgamma(0.5 * x) + 0.5 * G * x * ::log(0.5 * x * tau)
               - 0.5 * x * (sum_log + tau * sum_inv);
    }
    __device__ double base(double x0) const { return val(x0); }
    __device__ double operator()(double x) { return val(x); }
};

struct TauF {
    double shape_m1, rate;
    __device__ double val(double x) const {
        if (!(x > 0.0)) return -__builtin_inf();
        return shape_m1 * ::log(x) - rate * x;
    }
    __device__ double base(double x0) const { return val(x0); }
    __device__ double operator()(double x) { return val(x); }
};

struct Sig2F {
    double halfGp1, S, upper;
    __device__ double val(double x) const {
        if (!(x > 0.0) || !(x < upper)) return -__builtin_inf();
        return -halfGp1 * ::log(x) - S / (2.0 * x);
    }
    __device__ double base(double x0) const { return val(x0); }
    __device__ double operator()(double x) { return val(x); }
};

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// N wavefront sums at once, each with the same butterfly as wave_sum (so the
// same bits): per step all N exchanges are issued before any add waits for
// them, instead of N dependent chains one after another.
template <int N>
__device__ inline void wave_sum_n(double (&v)[N])
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double t[N];
#pragma unroll
        for (int k = 0; k < N; ++k) t[k] = __shfl_xor(v[k], off, 64);
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += t[k];
    }
}

// Orders the LDS accesses of one wavefront: the writes of every lane before
// the reads that follow.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// L of a segment in code compiled for at most kML coefficients.  The launcher
// picks kML < kMaxL only when every segment has L <= kML; the bound lets the
// compiler drop the array elements and loop steps beyond kML.
template <int kML>
__device__ inline int seg_L(const SegInfo &S) { return kML >= kMaxL ? S.L : (S.L < kML ? S.L : kML); }

// err[0]: flag bits (2: a slice draw reached the shrink cap, 4: a wait for
// the hyperparameter step timed out); err[1..7]: the first capped draw --
// claimed, kind, dataset, chain, gene (-1 for a hyperparameter), sweep, index
// within the kind (sample n, or -1).
constexpr int kErrWords = 8;

__device__ inline void raise_flag(int *err, int bit)
{
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void report_cap(int *err, int kind, const SegInfo &S, int64_t g, int64_t m, int sub)
{
    raise_flag(err, 2);
    if (atomicCAS(&err[1], 0, 1) == 0) {
        err[2] = kind;
        err[3] = S.dataset;
        err[4] = S.chain;
        err[5] = (int)g;
        err[6] = (int)m;
        err[7] = sub;
    }
}

// ---------------------------------------------------------------------------
// Beta-step building blocks (one lane per gene)
// ---------------------------------------------------------------------------
// C_r = A_r exp(X_r beta_g): the sum over the samples of distinct row r of
// exp(h_n + eps_gn + X_n beta_g).
template <typename T, int kML = kMaxL>
__device__ inline void row_sums_at_beta(const SegInfo &S, const T (&A)[kMaxRows], const T (&beta)[kMaxL],
                                        T (&C)[kMaxRows])
{
    const int L = seg_L<kML>(S), R = S.R;
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
        T xr = (T)0;
#pragma unroll
        for (int l = 0; l < kMaxL; ++l)
            if (l < L) xr += (T)S.Xrow[r * kMaxL + l] * beta[l];
        C[r] = (r < R) ? A[r] * dexp(xr) : (T)0;
    }
}

// Features of the learned proposal (any function of y_g, eps_g, h, theta,
// sigma^2, never of beta_g): per distinct row r, log((Y_r + 1/2) / A_r) and
// log(Y_r + 1/2); then theta_l and log sigma_l^2; zero up to 32.
template <typename T, int kML = kMaxL>
__device__ inline void gene_features(const SegInfo &S, const T (&A)[kMaxRows], const T (&YR)[kMaxRows],
                                     const double (&th)[kMaxL], const double (&s2)[kMaxL], float (&phi)[32])
{
    const int L = seg_L<kML>(S), R = S.R;
#pragma unroll
    for (int k = 0; k < 32; ++k) phi[k] = 0.0f;
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
        if (r < R) {
            const float y = (float)YR[r] + 0.5f;
            const float lr = ::logf(y / (float)A[r]);
            const float ly = ::logf(y);
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                if (k == r) phi[k] = lr;
                if (k == R + r) phi[k] = ly;
            }
        }
    }
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        if (l < L) {
            const float t = (float)th[l], ls2 = ::logf((float)s2[l]);
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                if (k == 2 * R + l) phi[k] = t;
                if (k == 2 * R + L + l) phi[k] = ls2;
            }
        }
    }
}

// One slice draw of a beta coefficient with the column's form fixed (kForm of
// BetaF); em1 at the accepted point is handed back in f.
template <int kForm, bool kPair, typename T>
__device__ inline T beta_draw_as(BetaF<T> &f, T b0, T w, uint32_t k0, uint32_t k1, uint4 ctr, int K, int cap,
                                 DrawRec &rec)
{
    BetaF<T, kForm> h;
    h.Y = f.Y;
    h.x0 = f.x0;
    h.dth = f.dth;
    h.inv_s2 = f.inv_s2;
    h.nv = f.nv;
    h.pm = f.pm;
#pragma unroll
    for (int k = 0; k < kMaxVals; ++k) {
        h.Gk[k] = f.Gk[k];
        h.vk[k] = f.vk[k];
        h.em1[k] = f.em1[k];
    }
    T b1;
    if constexpr (kPair) b1 = slice_draw_pair<T>(h, b0, w, k0, k1, ctr, K, cap, rec);
    else b1 = slice_draw<T>(h, b0, w, k0, k1, ctr, K, cap, rec);
#pragma unroll
    for (int k = 0; k < kMaxVals; ++k) f.em1[k] = h.em1[k];
    return b1;
}

// Algorithm 1 step 5 by slice draws: beta_g1..beta_gL in order, each moving
// the row sums C_r to the new coefficient; only `lead` lanes store.  kPair:
// two lanes per gene draw together (slice_draw_pair); the factor
// exp(X_rl (b1 - b0)) is then recomputed at the accepted point, the same
// expression on the same operands as the evaluation that accepted it.
template <typename T, int kML = kMaxL, bool kPair = false>
__device__ inline void beta_slice_draws(const SegInfo &S, const SweepArgs &a, int64_t g, int64_t Gp, bool lead,
                                        T (&beta)[kMaxL], T (&wb)[kMaxL], T (&wab)[kMaxL],
                                        const double (&th)[kMaxL], const double (&s2)[kMaxL],
                                        T (&C)[kMaxRows], const T (&YR)[kMaxRows], bool tuning, int &bad)
{
    const int L = seg_L<kML>(S), R = S.R;
    const uint32_t mm = (uint32_t)a.m;
    T *__restrict__ betap = (T *)S.beta;
    // Y_l = sum_r X_rl Y_r for every l up front: static offsets, so the design
    // table's loads issue together instead of one dependent load per row and
    // coefficient inside the loop (the same sums in the same order)
    T Yl[kMaxL];
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        Yl[j] = (T)0;
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            const T t = (T)S.Xrow[r * kMaxL + j] * YR[r];
            Yl[j] = (j < L && r < R) ? Yl[j] + t : Yl[j];
        }
    }
    for (int l = 0; l < L; ++l) {
        const int64_t idx = (int64_t)l * Gp + g;
        T b0 = (T)0, w = (T)1, wa = (T)0, Y = (T)0;
        double thl = 0.0, s2l = 1.0;
#pragma unroll
        for (int j = 0; j < kMaxL; ++j)
            if (j == l) { b0 = beta[j]; w = wb[j]; wa = wab[j]; thl = th[j]; s2l = s2[j]; Y = Yl[j]; }
        BetaF<T> f;
        f.Y = Y;
        f.nv = S.nv[l];
        f.pm = S.pm[l] != 0;
#pragma unroll
        for (int k = 0; k < kMaxVals; ++k) {
            f.Gk[k] = (T)0;
            f.vk[k] = (T)S.vals[l * kMaxVals + k];
            f.em1[k] = (T)0;
        }
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            const int k = S.xidx[r * kMaxL + l];
#pragma unroll
            for (int kk = 0; kk < kMaxVals; ++kk)
                if (r < R && k == kk) f.Gk[kk] += C[r];
        }
        f.x0 = b0;
        f.dth = (T)((double)b0 - thl);
        f.inv_s2 = (T)(1.0 / s2l);
        DrawRec rec;
        const uint4 ctr = draw_counter((uint32_t)g, 5, (uint32_t)l, mm, (uint32_t)S.chain, 0);
        T b1;
        if constexpr (std::is_same<T, float>::value) {
            // the column's form is uniform over the wavefront: pick the loop once
            if (f.pm) b1 = beta_draw_as<-1, kPair>(f, b0, w, S.key0, S.key1, ctr, a.K, a.cap, rec);
            else if (f.nv == 1) b1 = beta_draw_as<1, kPair>(f, b0, w, S.key0, S.key1, ctr, a.K, a.cap, rec);
            else b1 = beta_draw_as<0, kPair>(f, b0, w, S.key0, S.key1, ctr, a.K, a.cap, rec);
        } else {
            b1 = beta_draw_as<0, kPair>(f, b0, w, S.key0, S.key1, ctr, a.K, a.cap, rec);
        }
        if (tuning) {
            tune_width<T>(w, wa, b0, b1, a.m, a.burnin, a.tune_start);
            if (lead) {
                ((T *)S.w_beta)[idx] = w;
                ((T *)S.wa_beta)[idx] = wa;
            }
        }
        if (lead) betap[idx] = b1;
        bad |= rec.bad;
        if (a.dbg && lead) S.dbg_beta[idx] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
        // C_r *= exp(X_rl (b1 - b0)), from expm1 at the accepted point
        T fac[kMaxVals];
#pragma unroll
        for (int k = 0; k < kMaxVals; ++k) {
            if constexpr (kPair) fac[k] = (rec.bad || k >= f.nv) ? (T)1 : (T)1 + dexpm1(f.vk[k] * (b1 - b0));
            else fac[k] = rec.bad ? (T)1 : (T)1 + f.em1[k];
        }
        if constexpr (kPair && std::is_same<T, float>::value) {
            // a +-v column: the second factor by the evaluation's own route
            if (f.pm && !rec.bad) {
                const T e = dexpm1(f.vk[0] * (b1 - b0));
                fac[1] = (T)1 + -e * (T)__builtin_amdgcn_rcpf((float)((T)1 + e));
            }
        }
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            const int k = S.xidx[r * kMaxL + l];
#pragma unroll
            for (int kk = 0; kk < kMaxVals; ++kk)
                if (r < R && k == kk) C[r] *= fac[kk];
        }
#pragma unroll
        for (int j = 0; j < kMaxL; ++j)
            if (j == l) beta[j] = b1;
    }
}

// ---------------------------------------------------------------------------
// Laplace approximation of the beta_g conditional given eps_g (the base of the
// learned proposal).  Symmetric and triangular L x L matrices are stored
// packed by rows of their lower triangle: element (i, j), j <= i, at tri(i, j).
// ---------------------------------------------------------------------------
constexpr int kTri = kMaxL * (kMaxL + 1) / 2;
constexpr int kMaxOff = kMaxL * (kMaxL - 1) / 2;   // strict lower triangle
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ inline float dsqrt(float x) { return ::sqrtf(x); }
__device__ inline double dsqrt(double x) { return ::sqrt(x); }

// In place: H (symmetric positive definite) -> U, lower, with H = U U^T; dinv
// receives 1 / U_jj, which the solves multiply by.
template <typename T>
__device__ inline void chol_packed(T (&H)[kTri], int L, T (&dinv)[kMaxL])
{
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        dinv[j] = (T)1;
        if (j < L) {
            T d = H[tri(j, j)];
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                if (k < j) d -= H[tri(j, k)] * H[tri(j, k)];
            const T ujj = dsqrt(d);
            const T inv = (T)1 / ujj;
            H[tri(j, j)] = ujj;
            dinv[j] = inv;
#pragma unroll
            for (int i = 0; i < kMaxL; ++i) {
                if (i > j && i < L) {
                    T sum = H[tri(i, j)];
#pragma unroll
                    for (int k = 0; k < kMaxL; ++k)
                        if (k < j) sum -= H[tri(i, k)] * H[tri(j, k)];
                    H[tri(i, j)] = sum * inv;
                }
            }
        }
    }
}

// x with U U^T x = b (forward, then back substitution).
template <typename T>
__device__ inline void chol_solve_packed(const T (&U)[kTri], const T (&dinv)[kMaxL], int L, const T (&b)[kMaxL],
                                         T (&x)[kMaxL])
{
    T t[kMaxL];
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
        t[i] = (T)0;
        if (i < L) {
            T sum = b[i];
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                if (k < i) sum -= U[tri(i, k)] * t[k];
            t[i] = sum * dinv[i];
        }
    }
#pragma unroll
    for (int i = kMaxL - 1; i >= 0; --i) {
        x[i] = (T)0;
        if (i < L) {
            T sum = t[i];
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                if (k > i && k < L) sum -= U[tri(k, i)] * x[k];
            x[i] = sum * dinv[i];
        }
    }
}

// With Y_r and A_r the row sums (counts; exp(h_n + eps_gn)) over the samples of
// distinct row r (x_r) of X, the conditional is
//   log pi(b) = sum_r [Y_r x_r.b - A_r exp(x_r.b)] - sum_l (b_l - theta_l)^2 / (2 sigma_l^2).
// Start: the weighted least-squares fit of log((Y_r + 1/2) / A_r) on x_r with
// weights Y_r + 1/2 and the prior; then two Newton steps
//   b += H^-1 [sum_r (Y_r - c_r) x_r - (b - theta) / sigma^2],
//   H = sum_r c_r x_r x_r^T + diag(1 / sigma^2),  c_r = A_r exp(x_r.b).
// Returns the last iterate bh, the lower Cholesky factor U of H at bh and
// 1 / diag(U).  thT, is2: theta and 1 / sigma^2 in the working precision.
template <typename T, int kML = kMaxL>
__device__ inline void laplace_base(const SegInfo &S, const T (&A)[kMaxRows], const T (&Y)[kMaxRows],
                                    const T (&thT)[kMaxL], const T (&is2)[kMaxL], T (&bh)[kMaxL], T (&U)[kTri],
                                    T (&dinv)[kMaxL])
{
    const int L = seg_L<kML>(S), R = S.R;
    T rhs[kMaxL];
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
        rhs[i] = i < L ? thT[i] * is2[i] : (T)0;
#pragma unroll
        for (int j = 0; j <= i; ++j) U[tri(i, j)] = (i == j && i < L) ? is2[i] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
        if (r < R) {
            const T w = Y[r] + (T)0.5, z = dlog(w / A[r]);
#pragma unroll
            for (int i = 0; i < kMaxL; ++i) {
                if (i < L) {
                    const T xi = (T)S.Xrow[r * kMaxL + i];
                    rhs[i] += w * z * xi;
#pragma unroll
                    for (int j = 0; j <= i; ++j) U[tri(i, j)] += w * xi * (T)S.Xrow[r * kMaxL + j];
                }
            }
        }
    }
    chol_packed<T>(U, L, dinv);
    chol_solve_packed<T>(U, dinv, L, rhs, bh);
#pragma unroll 1
    for (int it = 0; it <= 2; ++it) {
        T cr[kMaxRows];
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            T xb = (T)0;
#pragma unroll
            for (int l = 0; l < kMaxL; ++l)
                if (l < L) xb += (T)S.Xrow[r * kMaxL + l] * bh[l];
            cr[r] = r < R ? A[r] * dexp(xb) : (T)0;
        }
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) {
            rhs[i] = i < L ? (thT[i] - bh[i]) * is2[i] : (T)0;
#pragma unroll
            for (int j = 0; j <= i; ++j) U[tri(i, j)] = (i == j && i < L) ? is2[i] : (T)0;
        }
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            if (r < R) {
#pragma unroll
                for (int i = 0; i < kMaxL; ++i) {
                    if (i < L) {
                        const T xi = (T)S.Xrow[r * kMaxL + i];
                        rhs[i] += (Y[r] - cr[r]) * xi;
#pragma unroll
                        for (int j = 0; j <= i; ++j) U[tri(i, j)] += cr[r] * xi * (T)S.Xrow[r * kMaxL + j];
                    }
                }
            }
        }
        chol_packed<T>(U, L, dinv);
        if (it == 2) break;
        T step[kMaxL];
        chol_solve_packed<T>(U, dinv, L, rhs, step);
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) bh[l] += step[l];
    }
}

// Algorithm 1 step 5 by one independence Metropolis-Hastings step for the
// block beta_g.  The proposal is the Laplace approximation N(bh, H^-1),
// H = U U^T (laplace_base), corrected by the network in the whitened
// coordinates w = U^T (b - bh): w ~ N(mu_w, Lw Lw^T) with mu_w,l = omean_l +
// oscale_l o_l, Lw = diag(oscale) Ls, Ls_ll = exp(o_{L+l}), Ls_lj =
// o_{2L + l(l-1)/2 + j}.  So beta* = bh + U^-T (mu_w + Lw z), and up to a
// constant log q(x) = -sum_l ls_l - |u|^2 / 2 with Lw u = U^T (x - bh) - mu_w.
// Random words: counter (g, 8 << 24, m, chain << 16 | j); word 0 is the
// acceptance uniform, words (1 + 2p, 2 + 2p) the Box-Muller pair p.
// log alpha = [log pi(beta*) - log pi(beta)] + [log q(beta) - log q(beta*)],
// the conditional's difference formed from the row sums:
//   sum_r [Y_r X_r d - C_r expm1(X_r d)] - sum_l d_l (beta_l - theta_l + d_l / 2) / sigma_l^2.
// Returns 1 if accepted.
template <typename T, int kML = kMaxL>
__device__ inline int beta_imh_draw(const SegInfo &S, const SweepArgs &a, int64_t g, int64_t Gp,
                                    T (&beta)[kMaxL], const T (&thT)[kMaxL], const T (&is2)[kMaxL],
                                    const T (&C)[kMaxRows], const T (&YR)[kMaxRows], const T (&bh)[kMaxL],
                                    const T (&U)[kTri], const T (&dinv)[kMaxL], const MlpDev *__restrict__ net,
                                    const float (&om)[kMaxL],
                                    const float (&ol)[kMaxL], const float (&oo)[kMaxOff])
{
    const int L = seg_L<kML>(S), R = S.R;
    const uint32_t mm = (uint32_t)a.m;
    const uint4 ctr = draw_counter((uint32_t)g, 8, 0, mm, (uint32_t)S.chain, 0);
    uint4 b0 = philox4x32_10(ctr, S.key0, S.key1);
    uint4 b1 = philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, ctr.w | 1u), S.key0, S.key1);
    uint4 b2 = philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, ctr.w | 2u), S.key0, S.key1);
    const uint32_t wv[12] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w, b2.x, b2.y, b2.z, b2.w};
    T z[kMaxL];
#pragma unroll
    for (int p = 0; p < kMaxL / 2; ++p) {
        const T ua = u01<T>(wv[1 + 2 * p]), ub = u01<T>(wv[2 + 2 * p]);
        if constexpr (sizeof(T) == sizeof(float)) {
            const float rho = ::sqrtf(-2.0f * ::logf(ua));
            float sn, cs;
            ::sincosf(6.28318530717958648f * ub, &sn, &cs);
            z[2 * p] = rho * cs;
            z[2 * p + 1] = rho * sn;
        } else {
            const double rho = ::sqrt(-2.0 * ::log((double)ua));
            const double ang = 6.283185307179586 * (double)ub;
            z[2 * p] = (T)(rho * ::cos(ang));
            z[2 * p + 1] = (T)(rho * ::sin(ang));
        }
    }
    // w = mu_w + Lw z, then beta* = bh + v with U^T v = w (back substitution)
    T mw[kMaxL], dg[kMaxL], idg[kMaxL], ios[kMaxL], w[kMaxL], bs[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        mw[l] = (T)0; dg[l] = (T)1; idg[l] = (T)1; ios[l] = (T)1; w[l] = (T)0;
        if (l < L) {
            const T osl = (T)net->oscale[l];
            mw[l] = (T)net->omean[l] + osl * (T)om[l];
            dg[l] = dexp((T)ol[l]);
            idg[l] = dexp(-(T)ol[l]);
            ios[l] = (T)(1.0f / net->oscale[l]);
            T sz = dg[l] * z[l];
#pragma unroll
            for (int j = 0; j < kMaxL; ++j)
                if (j < l) sz += (T)oo[l * (l - 1) / 2 + j] * z[j];
            w[l] = mw[l] + osl * sz;
        }
    }
#pragma unroll
    for (int i = kMaxL - 1; i >= 0; --i) {
        bs[i] = beta[i];
        if (i < L) {
            T sum = w[i];
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                if (k > i && k < L) sum -= U[tri(k, i)] * (bs[k] - bh[k]);
            bs[i] = bh[i] + sum * dinv[i];
        }
    }
    // log q at beta* and at beta: u with Lw u = U^T (x - bh) - mu_w
    T dq = (T)0;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        T dd[kMaxL], u[kMaxL];
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) {
            dd[i] = (T)0;
            if (i < L) {
                T sum = (T)0;
#pragma unroll
                for (int k = 0; k < kMaxL; ++k)
                    if (k >= i && k < L) sum += U[tri(k, i)] * ((pass == 0 ? bs[k] : beta[k]) - bh[k]);
                dd[i] = sum - mw[i];
            }
        }
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) {
            u[l] = (T)0;
            if (l < L) {
                T sum = dd[l] * ios[l];
#pragma unroll
                for (int j = 0; j < kMaxL; ++j)
                    if (j < l) sum -= (T)oo[l * (l - 1) / 2 + j] * u[j];
                u[l] = sum * idg[l];
                dq += (pass == 0 ? (T)0.5 : (T)-0.5) * u[l] * u[l];
            }
        }
    }
    T d[kMaxL];
    T dpi = (T)0;
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        d[l] = (T)0;
        if (l < L) {
            d[l] = bs[l] - beta[l];
            dpi -= d[l] * ((beta[l] - thT[l]) + (T)0.5 * d[l]) * is2[l];
        }
    }
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
        if (r < R) {
            T xd = (T)0;
#pragma unroll
            for (int l = 0; l < kMaxL; ++l)
                if (l < L) xd += (T)S.Xrow[r * kMaxL + l] * d[l];
            dpi += YR[r] * xd - C[r] * dexpm1(xd);
        }
    }
    const T la = dpi + dq;
    const bool acc = dlog(u01<T>(wv[0])) < la;
    if (acc) {
#pragma unroll
        for (int l = 0; l < kMaxL; ++l)
            if (l < L) {
                beta[l] = bs[l];
                ((T *)S.beta)[(int64_t)l * Gp + g] = bs[l];
            }
    }
    return acc ? 1 : 0;
}

// Whitened coordinates w = U^T (b - bh) of the Laplace approximation: the
// training targets of the proposal network.
template <typename T>
__device__ inline void whiten(int L, const T (&U)[kTri], const T (&bh)[kMaxL], const T (&b)[kMaxL], T (&w)[kMaxL])
{
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
        w[i] = (T)0;
        if (i < L) {
            T sum = (T)0;
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                if (k >= i && k < L) sum += U[tri(k, i)] * (b[k] - bh[k]);
            w[i] = sum;
        }
    }
}

// After the beta step: moments, trace, and the tile partials of
// (beta_l - theta_l) and its square (all lanes of the wavefront call).
template <typename T, int kML = kMaxL>
__device__ inline void beta_finish(const SegInfo &S, const SweepArgs &a, int64_t g, int64_t Gp, bool active,
                                   const T (&beta)[kMaxL], double2 (&mob)[kMaxL], const double (&th)[kMaxL],
                                   int tile, int lane, int tslot, float *trow, bool sampling)
{
    const int L = seg_L<kML>(S);
    constexpr int kB = kML < kMaxL ? kML : kMaxL;
    double sv[2 * kB];
#pragma unroll
    for (int l = 0; l < kB; ++l) {
        sv[2 * l] = 0.0;
        sv[2 * l + 1] = 0.0;
        if (l < L) {
            const T b1 = beta[l];
            if (active && sampling) {
                double2 mo = mob[l];
                welford(mo, (double)b1, a.inv_k);
                S.mom_beta[(int64_t)l * Gp + g] = mo;
            }
            if (tslot >= 0) trow[(int64_t)tslot * (L + 1) + 1 + l] = (float)b1;
            const double dv = active ? (double)b1 - th[l] : 0.0;
            sv[2 * l] = dv;
            sv[2 * l + 1] = dv * dv;
        }
    }
    // contrast events (Section 3.2) on the end-of-sweep beta: bit e of `fail`
    // is set when a row of event e does not hold
    if (S.n_ev > 0 && active && sampling && a.m > S.ev_from) {
        uint32_t fail = 0;
        for (int r = 0; r < S.n_crow; ++r) {
            double sum = 0.0;
#pragma unroll
            for (int l = 0; l < kB; ++l)
                if (l < L) sum += S.cv[r * kMaxL + l] * (double)beta[l];
            if (!(sum > S.cb[r])) fail |= 1u << S.crow_event[r];
        }
        for (int e = 0; e < S.n_ev; ++e)
            if (!((fail >> e) & 1u)) S.ev_count[(int64_t)e * Gp + g] += 1;
    }
    wave_sum_n(sv);
    if (lane == 0) {
#pragma unroll
        for (int l = 0; l < kB; ++l)
            if (l < L) {
                S.partials[(int64_t)(2 + 2 * l) * S.pstride + tile] = sv[2 * l];
                S.partials[(int64_t)(3 + 2 * l) * S.pstride + tile] = sv[2 * l + 1];
            }
    }
}

// ---------------------------------------------------------------------------
// Step 1: eps draws, one lane per (gene, sample)
// ---------------------------------------------------------------------------
// A work item is (segment, tile, n0, n1): one wavefront draws eps_gn for the
// 64 genes of the tile and the samples n0 <= n < n1, one sample after the
// other.  The eps conditional involves only y_gn, h_n, X_n beta_g and gamma_g,
// so every (gene, sample) draw is independent of the others in the sweep.
// se, sx (the single-launch sweep): LDS arrays [N][kTile] that receive the new
// eps_gn and exp(h_n + eps_gn) for the tile's gamma and beta draws.
template <typename T>
__device__ inline void eps_wave(const SegInfo &S, int tile, int n0, int n1, const SweepArgs &a, int *err,
                                T *se = nullptr, T *sx = nullptr)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t Gp = S.Gp;
    const int64_t g = (int64_t)tile * kTile + lane;
    if (g >= S.G) return;                 // no cross-lane operations follow
    const int L = S.L;
    const uint32_t mm = (uint32_t)a.m, chain = (uint32_t)S.chain;
    const uint32_t k0 = S.key0, k1 = S.key1;
    const bool tuning = a.m <= a.burnin;
    // with the shift step on, eps moments are taken after it (shift_sweep)
    const bool sampling = a.m > a.burnin && !((a.mask >> kKindShift) & 1u);
    const bool upd = (a.mask >> 1) & 1u;
    const int32_t *__restrict__ yp = S.y;
    T *__restrict__ eps = (T *)S.eps;
    T *__restrict__ w_eps = (T *)S.w_eps;
    T *__restrict__ wa_eps = (T *)S.wa_eps;
    double2 *__restrict__ mom = S.mom_eps;
    const T *__restrict__ betap = (const T *)S.beta;
    T beta[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) beta[l] = l < L ? betap[(int64_t)l * Gp + g] : (T)0;
    const T inv_gam = (T)1 / ((const T *)S.gam)[g];
    int bad = 0, bad_n = -1;
    // software pipeline: the next sample's inputs are requested before the
    // current draw, so their latency hides behind its slice loop
    int y_nx = 0;
    T e_nx = (T)0, w_nx = (T)1, wa_nx = (T)0;
    double2 mo_nx = make_double2(0.0, 0.0);
    auto fetch = [&](int n) {
        const int64_t idx = (int64_t)n * Gp + g;
        y_nx = yp[idx];
        e_nx = eps[idx];
        if (upd) w_nx = w_eps[idx];
        if (upd && tuning) wa_nx = wa_eps[idx];
        if (sampling) mo_nx = mom[idx];
    };
    if (n0 < n1) fetch(n0);
    for (int n = n0; n < n1; ++n) {
        const int64_t idx = (int64_t)n * Gp + g;
        const int yv = y_nx;
        const T e0 = e_nx;
        T w = w_nx, wa = wa_nx;
        double2 mo = mo_nx;
        if (n + 1 < n1) fetch(n + 1);
        T xb = (T)0;
#pragma unroll
        for (int l = 0; l < kMaxL; ++l)
            if (l < L) xb += (T)S.X[n * kMaxL + l] * beta[l];
        T e1 = e0;
        if (upd) {
            EpsF<T> f{(T)yv, dexp((T)S.h[n] + e0 + xb), e0, inv_gam};
            DrawRec rec;
            e1 = slice_draw<T>(f, e0, w, k0, k1, draw_counter((uint32_t)g, 1, (uint32_t)n, mm, chain, 0), a.K,
                               a.cap, rec);
            eps[idx] = e1;
            if (tuning) {
                tune_width<T>(w, wa, e0, e1, a.m, a.burnin, a.tune_start);
                w_eps[idx] = w;
                wa_eps[idx] = wa;
            }
            if (rec.bad) {
                bad = 1;
                bad_n = n;
            }
            if (a.dbg) S.dbg_eps[idx] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
        }
        if (sampling) {
            welford(mo, (double)e1, a.inv_k);
            mom[idx] = mo;
        }
        if (se) {
            se[n * kTile + lane] = e1;
            sx[n * kTile + lane] = dexp((T)S.h[n] + e1);
        }
    }
    if (bad) report_cap(err, 1, S, g, a.m, bad_n);
}

// ---------------------------------------------------------------------------
// Steps 2 and 5 after the eps draws: gamma_g and beta_g on two wavefronts
// ---------------------------------------------------------------------------
// Given eps_g, gamma_g depends on nu and tau only and beta_g on theta and
// sigma^2 only, so the two draws of a gene are independent and run on
// separate wavefronts of the tile's workgroup.

// Step 2 (wavefront 0): S_g = sum_n eps_gn^2, one gamma draw, moments, trace
// and the tile partials of log gamma and 1 / gamma.
// se: the tile's new eps in LDS ([N][kTile], single-launch sweep), else null
template <typename T, int kML = kMaxL>
__device__ inline void gamma_wave(const SegInfo &S, int tile, const SweepArgs &a, int *err, const T *se = nullptr)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t Gp = S.Gp;
    const int64_t g = (int64_t)tile * kTile + lane;
    const bool active = g < S.G;
    const int N = S.N, L = seg_L<kML>(S);
    const bool tuning = a.m <= a.burnin, sampling = a.m > a.burnin;
    const T *__restrict__ eps = (const T *)S.eps;
    T *__restrict__ gamp = (T *)S.gam;
    double lg = 0.0, ig = 0.0;
    int bad = 0;
    if (active) {
        T S2 = (T)0;
#pragma unroll 8
        for (int n = 0; n < N; ++n) {
            const T e = se ? se[n * kTile + lane] : eps[(int64_t)n * Gp + g];
            S2 += e * e;
        }
        T gam = gamp[g];
        if ((a.mask >> 2) & 1u) {
            const HyperState &H = *S.hyp;
            const double nu = H.nu, tau = H.tau;
            T wg = ((T *)S.w_gam)[g];
            T wag = tuning ? ((T *)S.wa_gam)[g] : (T)0;
            const double alpha1 = 0.5 * nu + 0.5 * N + 1.0;
            const double scale = 0.5 * nu * tau + 0.5 * (double)S2;
            int tries = 0;
            if ((a.mask >> kKindExact) & 1u) {
                // exact draw: gamma_g = (nu tau/2 + S_g/2) / X, X ~ Gamma(nu/2 + N/2)
                double v = 0.0;
                tries = exact_gamma_draw(kKindExact, 0.5 * nu + 0.5 * N, scale, true, __builtin_inf(), S.key0, S.key1,
                                         (uint32_t)g, 0, (uint32_t)a.m, (uint32_t)S.chain, v);
                if (tries > 0) {
                    gam = (T)v;
                    gamp[g] = gam;
                    if (a.dbg) S.dbg_gam[g] = make_int4(-1, 0, 0, tries);
                }
            }
            if (tries == 0) {
                GamF<T> f{(T)alpha1, (T)scale, gam};
                DrawRec rec;
                const T g1 = slice_draw<T>(f, gam, wg, S.key0, S.key1,
                                           draw_counter((uint32_t)g, 2, 0, (uint32_t)a.m, (uint32_t)S.chain, 0),
                                           a.K, a.cap, rec);
                if (tuning) {
                    tune_width<T>(wg, wag, gam, g1, a.m, a.burnin, a.tune_start);
                    ((T *)S.w_gam)[g] = wg;
                    ((T *)S.wa_gam)[g] = wag;
                }
                gam = g1;
                gamp[g] = g1;
                bad |= rec.bad;
                if (a.dbg) S.dbg_gam[g] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
            }
        }
        if (sampling) {
            double2 mog = S.mom_gam[g];
            welford(mog, (double)gam, a.inv_k);
            S.mom_gam[g] = mog;
        }
        lg = ::log((double)gam);
        ig = 1.0 / (double)gam;
        if (a.trace_point >= 0) {
            const int tslot = S.trace_slot[g];
            if (tslot >= 0)
                S.trace[(int64_t)a.trace_point * S.trace_stride + 2 + 2 * L + (int64_t)tslot * (L + 1)] = (float)gam;
        }
    }
    double sv[2] = {lg, ig};
    wave_sum_n(sv);
    if (lane == 0) {
        S.partials[tile] = sv[0];
        S.partials[S.pstride + tile] = sv[1];
    }
    if (bad) report_cap(err, 2, S, g, a.m, -1);
}


// Step 5 for the genes of one wavefront: the row sums A_r = sum over the
// samples of row r of exp(h_n + eps_gn), then beta_g1..beta_gL by slice draws,
// or, with the learned proposal, one independence MH step for the block.
// Then the moments, trace, training pairs and the wavefront's partials of
// (beta_l - theta_l) and its square in column `col`.
//   lane gene g, `active`: the lane holds a gene
//   kMode 0: slice steps (Algorithm 1)
//   kMode 1 (learned kernel, any sweep: training pairs, slice or MH steps) and
//   kMode 2 (the MH step only, no training pairs: the code the learned sweeps
//   run), fallback_group = false: a tile's wavefront; with a.learned the genes
//   flagged for fallback are left to their fallback group
//   fallback_group = true: up to 64 flagged genes, slice steps only
//   sx: exp(h_n + eps_gn) of the tile's genes in LDS ([N][kTile], single-launch
//   sweep, a tile's own wavefront), else null
template <typename T, int kMode, int kML = kMaxL>
__device__ inline void beta_genes(const SegInfo &S, int64_t g, bool active, int64_t col, bool fallback_group,
                                  const SweepArgs &a, const MlpDev *__restrict__ net, int *err,
                                  const T *sx = nullptr)
{
    constexpr bool kLearned = kMode != 0;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t Gp = S.Gp;
    const int N = S.N, L = seg_L<kML>(S), R = S.R;
    const bool tuning = a.m <= a.burnin, sampling = a.m > a.burnin;
    const bool upd_beta = (a.mask >> 5) & 1u;
    // with the learned step, a tile's wavefront leaves flagged genes alone
    bool mine = active;
    if constexpr (kLearned)
        if (!fallback_group && a.learned && active && S.fallback[g] != 0) mine = false;
    const HyperState &H = *S.hyp;
    double th[kMaxL], s2[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        th[l] = l < L ? H.theta[l] : 0.0;
        s2[l] = l < L ? H.sig2[l] : 1.0;
    }
    T beta[kMaxL], wb[kMaxL], wab[kMaxL];
    double2 mob[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        const bool on = l < L && mine;
        const int64_t idx = (int64_t)l * Gp + g;
        beta[l] = on ? ((const T *)S.beta)[idx] : (T)0;
        wb[l] = (on && upd_beta) ? ((const T *)S.w_beta)[idx] : (T)1;
        wab[l] = (on && upd_beta && tuning) ? ((const T *)S.wa_beta)[idx] : (T)0;
        mob[l] = (on && sampling) ? S.mom_beta[idx] : make_double2(0.0, 0.0);
    }
    T A[kMaxRows], YR[kMaxRows];
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
        A[r] = (T)0;
        YR[r] = (r < R && mine) ? ((const T *)S.YR)[(int64_t)r * Gp + g] : (T)0;
    }
    if (mine) {
        const T *__restrict__ eps = (const T *)S.eps;
#pragma unroll 8
        for (int n = 0; n < N; ++n) {
            const T ehe = sx ? sx[n * kTile + lane] : dexp((T)S.h[n] + eps[(int64_t)n * Gp + g]);
            const int rr = S.row_of[n];
#pragma unroll
            for (int r = 0; r < kMaxRows; ++r)
                if (r == rr) A[r] += ehe;
        }
    }
    const int tslot = (a.trace_point >= 0 && mine) ? S.trace_slot[g] : -1;
    float *trow = a.trace_point >= 0 ? S.trace + (int64_t)a.trace_point * S.trace_stride + 2 + 2 * L : nullptr;
    T C[kMaxRows];
    row_sums_at_beta<T, kML>(S, A, beta, C);
    int bad = 0;
    if constexpr (kLearned) {
        if (fallback_group) {
            if (mine && upd_beta) {
                beta_slice_draws<T, kML>(S, a, g, Gp, true, beta, wb, wab, th, s2, C, YR, tuning, bad);
                S.imh_last[g] = -1;
            }
        } else {
            // training pairs: the features the beta step saw, then the new beta
            float *pair = (kMode == 1 && a.pair_base >= 0 && mine) ? S.pairs + (a.pair_base + g) * kPairStride
                                                                   : nullptr;
            if (pair) {
                float phi[32];
                gene_features<T, kML>(S, A, YR, th, s2, phi);
#pragma unroll
                for (int k = 0; k < 32; ++k) pair[k] = phi[k];
            }
            // the network's outputs for this gene (mlp_sweep ran before this kernel)
            float om[kMaxL], ol[kMaxL], oo[kMaxOff];
            const bool use_net = a.learned && mine && upd_beta && !a.laplace;
            const int nof = L * (L - 1) / 2;
#pragma unroll
            for (int l = 0; l < kMaxL; ++l) {
                om[l] = (use_net && l < L) ? S.mlp_out[(int64_t)l * Gp + g] : 0.0f;
                ol[l] = (use_net && l < L) ? S.mlp_out[(int64_t)(L + l) * Gp + g] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < kMaxOff; ++k)
                oo[k] = (use_net && k < nof) ? S.mlp_out[(int64_t)(2 * L + k) * Gp + g] : 0.0f;
            T thT[kMaxL], is2[kMaxL];
#pragma unroll
            for (int l = 0; l < kMaxL; ++l) {
                thT[l] = (T)th[l];
                is2[l] = (T)(1.0 / s2[l]);
            }
            T bh[kMaxL], U[kTri], dinv[kMaxL];
            if (a.learned || pair) laplace_base<T, kML>(S, A, YR, thT, is2, bh, U, dinv);
            if (mine && upd_beta) {
                if (kMode == 2 || a.learned) {
                    const int acc =
                        beta_imh_draw<T, kML>(S, a, g, Gp, beta, thT, is2, C, YR, bh, U, dinv, net, om, ol, oo);
                    S.imh_last[g] = acc;
                    if (a.count_imh) S.imh_count[g] += acc;
                    if (a.m > a.burnin) {        // acceptance statistics of the sampling sweeps
                        int2 st = S.imh_stat[g];
                        st.x += 1;
                        st.y += acc;
                        S.imh_stat[g] = st;
                    }
                } else {
                    beta_slice_draws<T, kML>(S, a, g, Gp, true, beta, wb, wab, th, s2, C, YR, tuning, bad);
                    S.imh_last[g] = -1;
                }
            }
            if (pair) {          // the target: beta after the step, whitened
                T wt[kMaxL];
                whiten<T>(L, U, bh, beta, wt);
#pragma unroll
                for (int l = 0; l < kMaxL; ++l)
                    if (l < L) pair[32 + l] = (float)wt[l];
            }
        }
    } else {
        if (mine && upd_beta) beta_slice_draws<T, kML>(S, a, g, Gp, true, beta, wb, wab, th, s2, C, YR, tuning, bad);
    }
    // with the shift step on, the moments, trace and partials of beta are
    // taken after it (shift_sweep)
    if (!((a.mask >> kKindShift) & 1u))
        beta_finish<T, kML>(S, a, g, Gp, mine, beta, mob, th, col, lane, tslot, trow, sampling);
    if (bad) report_cap(err, 5, S, g, a.m, -1);
}

// Steps 2 and 5: one workgroup per tile (wavefront 0 gamma, wavefront 1
// beta); with the learned step, `nfb` further workgroups each draw beta by
// slice steps for a group of up to 64 genes flagged for fallback
// (fb_items: segment, first list entry, count, partial column).
template <typename T, int kMode, int kML>
__global__ __launch_bounds__(128) void gb_sweep(const SegInfo *__restrict__ segs, const int2 *__restrict__ tiles,
                                                int ntiles, const int4 *__restrict__ fb_items, int nfb, SweepArgs a0,
                                                const MlpDev *__restrict__ net, int *err)
{
    const SweepArgs a = resolve_args(a0);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int tix = (int)blockIdx.x;
    if (tix < ntiles) {
        const int2 tt = tiles[tix];
        const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
        const int tile = __builtin_amdgcn_readfirstlane(tt.y);
        const SegInfo &S = segs[sidx];
        if (wave == 0) {
            gamma_wave<T, kML>(S, tile, a, err);
        } else {
            // the beta wavefront is the workgroup's longer chain: it gets the
            // SIMD's issue slots first (paper design G = 50,000: 34.0 -> 33.5 us;
            // with the shift step, gb_shift_sweep, no gain, so not there)
            __builtin_amdgcn_s_setprio(3);
            const int64_t g = (int64_t)tile * kTile + lane;
            beta_genes<T, kMode, kML>(S, g, g < S.G, tile, false, a, net, err);
        }
        return;
    }
    if constexpr (kMode != 0) {
        if (tix - ntiles >= nfb || wave != 0) return;
        const int4 it = fb_items[tix - ntiles];
        const int sidx = __builtin_amdgcn_readfirstlane(it.x);
        const SegInfo &S = segs[sidx];
        const bool active = lane < it.z;
        const int64_t g = active ? S.fb_genes[it.y + lane] : 0;
        const int64_t col = it.w;
        beta_genes<T, kMode, kML>(S, g, active, col, true, a, net, err);
        if (lane == 0) {      // no gamma in a fallback column
            S.partials[col] = 0.0;
            S.partials[S.pstride + col] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// The shift step (an addition to Algorithm 1; update_mask bit kKindShift),
// after steps 2 and 5 and before the hyperparameter steps.  In the model of
// Section 4.1 the counts of gene g depend on eps_g and beta_g only through
// eps_gn + X_n beta_g, so beta_g -> beta_g + delta, eps_gn -> eps_gn - X_n delta
// keeps the likelihood and has unit Jacobian; given those sums, gamma_g, theta
// and sigma^2, delta is Gaussian with precision P = X^T X / gamma_g +
// diag(1 / sigma^2) and mean P^-1 c, c = X^T eps_g / gamma_g - (beta_g - theta)
// / sigma^2.  It is drawn exactly: delta = P^-1 c + U^-T z, P = U U^T, z from
// Box-Muller pairs on words (2p, 2p + 1) of counter (g, 11 << 24, m,
// chain << 16 | j).  The eps moments, and the beta moments, trace and tile
// partials, are taken here, after the step.  One lane per gene, one wavefront
// per tile, four tiles per workgroup.
// ---------------------------------------------------------------------------
constexpr int kShiftChunk = 16;    // samples whose eps and moments a lane holds at once

template <typename T, int kML>
__device__ inline void shift_genes(const SegInfo &S, int tile, const SweepArgs &a)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t Gp = S.Gp;
    const int64_t g = (int64_t)tile * kTile + lane;
    const bool active = g < S.G;
    const int N = S.N, L = seg_L<kML>(S);
    const bool sampling = a.m > a.burnin;
    const HyperState &H = *S.hyp;
    double th[kMaxL], s2[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        th[l] = l < L ? H.theta[l] : 0.0;
        s2[l] = l < L ? H.sig2[l] : 1.0;
    }
    T *__restrict__ eps = (T *)S.eps;
    T *__restrict__ betap = (T *)S.beta;
    double2 *__restrict__ mom = S.mom_eps;
    // every load of the first chunk is issued before any arithmetic: the
    // kernel is one lane per gene, so its time is memory round trips
    T beta[kMaxL], d[kMaxL], e[kShiftChunk];
    double2 mob[kMaxL], mo[kShiftChunk];
    const T gam = active ? ((const T *)S.gam)[g] : (T)1;
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        const bool on = l < L && active;
        beta[l] = on ? betap[(int64_t)l * Gp + g] : (T)0;
        mob[l] = (on && sampling) ? S.mom_beta[(int64_t)l * Gp + g] : make_double2(0.0, 0.0);
        d[l] = (T)0;
    }
#pragma unroll
    for (int k = 0; k < kShiftChunk; ++k) {
        const bool on = active && k < N;
        e[k] = on ? eps[(int64_t)k * Gp + g] : (T)0;
        mo[k] = (on && sampling) ? mom[(int64_t)k * Gp + g] : make_double2(0.0, 0.0);
    }
    if (active) {
        const T ig = (T)1 / gam;
        T xe[kMaxL];
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) xe[l] = (T)0;
#pragma unroll
        for (int k = 0; k < kShiftChunk; ++k)
            if (k < N) {
#pragma unroll
                for (int l = 0; l < kMaxL; ++l)
                    if (l < L) xe[l] += (T)S.X[k * kMaxL + l] * e[k];
            }
        for (int c0 = kShiftChunk; c0 < N; c0 += kShiftChunk) {     // N > 16: further chunks
            T ec[kShiftChunk];
#pragma unroll
            for (int k = 0; k < kShiftChunk; ++k) ec[k] = c0 + k < N ? eps[(int64_t)(c0 + k) * Gp + g] : (T)0;
#pragma unroll
            for (int k = 0; k < kShiftChunk; ++k)
                if (c0 + k < N) {
#pragma unroll
                    for (int l = 0; l < kMaxL; ++l)
                        if (l < L) xe[l] += (T)S.X[(c0 + k) * kMaxL + l] * ec[k];
                }
        }
        T U[kTri], dinv[kMaxL], cv[kMaxL], mean[kMaxL];
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) {
            const T is2 = (T)(1.0 / s2[i]);
            cv[i] = i < L ? xe[i] * ig - (beta[i] - (T)th[i]) * is2 : (T)0;
#pragma unroll
            for (int j = 0; j <= i; ++j)
                U[tri(i, j)] = (i < L) ? (T)S.XtX[i * kMaxL + j] * ig + (i == j ? is2 : (T)0) : (T)0;
        }
        chol_packed<T>(U, L, dinv);
        chol_solve_packed<T>(U, dinv, L, cv, mean);
        const uint4 ctr = draw_counter((uint32_t)g, kKindShift, 0, (uint32_t)a.m, (uint32_t)S.chain, 0);
        const uint4 b0 = philox4x32_10(ctr, S.key0, S.key1);
        const uint4 b1 = philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, ctr.w | 1u), S.key0, S.key1);
        const uint32_t wv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
        T z[kMaxL];
#pragma unroll
        for (int p = 0; p < kMaxL / 2; ++p) {
            const T ua = u01<T>(wv[2 * p]), ub = u01<T>(wv[2 * p + 1]);
            if constexpr (sizeof(T) == sizeof(float)) {
                const float rho = ::sqrtf(-2.0f * ::logf(ua));
                float sn, cs;
                ::sincosf(6.28318530717958648f * ub, &sn, &cs);
                z[2 * p] = rho * cs;
                z[2 * p + 1] = rho * sn;
            } else {
                const double rho = ::sqrt(-2.0 * ::log((double)ua));
                const double ang = 6.283185307179586 * (double)ub;
                z[2 * p] = (T)(rho * ::cos(ang));
                z[2 * p + 1] = (T)(rho * ::sin(ang));
            }
        }
        // v = U^-T z (back substitution), delta = mean + v
        T v[kMaxL];
#pragma unroll
        for (int i = kMaxL - 1; i >= 0; --i) {
            v[i] = (T)0;
            if (i < L) {
                T sum = z[i];
#pragma unroll
                for (int k = 0; k < kMaxL; ++k)
                    if (k > i && k < L) sum -= U[tri(k, i)] * v[k];
                v[i] = sum * dinv[i];
            }
        }
#pragma unroll
        for (int l = 0; l < kMaxL; ++l)
            if (l < L) {
                d[l] = mean[l] + v[l];
                beta[l] += d[l];
                betap[(int64_t)l * Gp + g] = beta[l];
            }
        for (int c0 = 0; c0 < N; c0 += kShiftChunk) {
            if (c0 > 0) {
#pragma unroll
                for (int k = 0; k < kShiftChunk; ++k) {
                    const bool on = c0 + k < N;
                    e[k] = on ? eps[(int64_t)(c0 + k) * Gp + g] : (T)0;
                    mo[k] = (on && sampling) ? mom[(int64_t)(c0 + k) * Gp + g] : make_double2(0.0, 0.0);
                }
            }
#pragma unroll
            for (int k = 0; k < kShiftChunk; ++k) {
                const int n = c0 + k;
                if (n < N) {
                    const int64_t idx = (int64_t)n * Gp + g;
                    T xd = (T)0;
#pragma unroll
                    for (int l = 0; l < kMaxL; ++l)
                        if (l < L) xd += (T)S.X[n * kMaxL + l] * d[l];
                    const T en = e[k] - xd;
                    eps[idx] = en;
                    if (sampling) {
                        double2 m2 = mo[k];
                        welford(m2, (double)en, a.inv_k);
                        mom[idx] = m2;
                    }
                }
            }
        }
    }
    const int tslot = (a.trace_point >= 0 && active) ? S.trace_slot[g] : -1;
    float *trow = a.trace_point >= 0 ? S.trace + (int64_t)a.trace_point * S.trace_stride + 2 + 2 * L : nullptr;
    beta_finish<T, kML>(S, a, g, Gp, active, beta, mob, th, tile, lane, tslot, trow, sampling);
}

template <typename T, int kML>
__global__ __launch_bounds__(256) void shift_sweep(const SegInfo *__restrict__ segs, const int2 *__restrict__ tiles,
                                                   int ntiles, SweepArgs a0)
{
    const SweepArgs a = resolve_args(a0);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int tix = (int)blockIdx.x * 4 + wave;
    if (tix >= ntiles) return;            // the whole wavefront leaves
    const int2 tt = tiles[tix];
    const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
    const int tile = __builtin_amdgcn_readfirstlane(tt.y);
    shift_genes<T, kML>(segs[sidx], tile, a);
}

// Steps 2 and 5 and the shift step in one launch (the shift step on, with the
// slice steps (kMode 0) or with the independence-MH beta step when no gene
// falls back to the slice steps (kMode 2)): per tile, gamma on wavefront 0 and
// beta on wavefront 1 as in gb_sweep, a workgroup barrier (the tile's new
// gamma_g and beta_g are then written and visible to the workgroup), then
// wavefront 1 shifts the tile.  A tile's shift overlaps other tiles' beta
// draws instead of waiting for a launch of its own; the arithmetic is that of
// shift_sweep.  A kernel of its own so that the shift code's registers do not
// lower the occupancy of gb_sweep.
template <typename T, int kMode, int kML>
__global__ __launch_bounds__(128) void gb_shift_sweep(const SegInfo *__restrict__ segs,
                                                      const int2 *__restrict__ tiles, int ntiles, SweepArgs a0,
                                                      const MlpDev *__restrict__ net, int *err)
{
    static_assert(kMode == 0 || kMode == 2, "the fused shift needs every beta of the tile drawn in the tile");
    const SweepArgs a = resolve_args(a0);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int tix = (int)blockIdx.x;
    if (tix >= ntiles) return;            // the whole workgroup leaves
    const int2 tt = tiles[tix];
    const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
    const int tile = __builtin_amdgcn_readfirstlane(tt.y);
    const SegInfo &S = segs[sidx];
    if (wave == 0) {
        gamma_wave<T, kML>(S, tile, a, err);
    } else {
        const int64_t g = (int64_t)tile * kTile + lane;
        beta_genes<T, kMode, kML>(S, g, g < S.G, tile, false, a, net, err);
    }
    __syncthreads();
    if (wave == 1) shift_genes<T, kML>(S, tile, a);
}

// Steps 2 and 5 of the slice sweep with two lanes per gene for beta (no shift
// step): wavefront 0 draws gamma for the tile's 64 genes, wavefronts 1 and 2
// draw beta for 32 genes each, lanes 2j and 2j + 1 of a wavefront together
// for one gene (slice_draw_pair: both step-out directions at once, shrink
// candidates two at a time).  At a few tiles per SIMD the beta wavefront is a
// chain of dependent slice trips, and the pair takes about 30% fewer of them.
// The new beta goes through LDS to wavefront 0, which (with the moments
// prefetched while the draws ran) takes the moments, trace, events and tile
// partials with beta_finish, in the order of gb_sweep: the chains are the same
// bit for bit.  kShift: the shift step on -- wavefront 1 then shifts the tile
// after the barrier (shift_genes, which takes the moments, trace, events and
// partials), as in gb_shift_sweep.
template <typename T, int kML, bool kShift = false>
__global__ __launch_bounds__(192) void gb_pair_sweep(const SegInfo *__restrict__ segs,
                                                     const int2 *__restrict__ tiles, int ntiles, SweepArgs a0,
                                                     int *err)
{
    __shared__ double sbeta[kMaxL][kTile];
    const SweepArgs a = resolve_args(a0);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int tix = (int)blockIdx.x;
    if (tix >= ntiles) return;            // the whole workgroup leaves
    const int2 tt = tiles[tix];
    const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
    const int tile = __builtin_amdgcn_readfirstlane(tt.y);
    const SegInfo &S = segs[sidx];
    const int64_t Gp = S.Gp;
    const int L = seg_L<kML>(S);
    const bool sampling = a.m > a.burnin;
    double2 mob[kMaxL];
    double th[kMaxL];
    int tslot = -1;
    float *trow = nullptr;
    if (wave == 0) {
        gamma_wave<T, kML>(S, tile, a, err);
        // prefetch what beta_finish needs while the beta wavefronts draw
        const int64_t g = (int64_t)tile * kTile + lane;
        const bool active = g < S.G;
        const HyperState &H = *S.hyp;
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) {
            th[l] = l < L ? H.theta[l] : 0.0;
            mob[l] = (l < L && active && sampling) ? S.mom_beta[(int64_t)l * Gp + g] : make_double2(0.0, 0.0);
        }
        tslot = (a.trace_point >= 0 && active) ? S.trace_slot[g] : -1;
        trow = a.trace_point >= 0 ? S.trace + (int64_t)a.trace_point * S.trace_stride + 2 + 2 * L : nullptr;
    } else {
        const int j = 32 * (wave - 1) + (lane >> 1);
        const int64_t g = (int64_t)tile * kTile + j;
        const bool active = g < S.G;
        const bool lead = (lane & 1) == 0;
        const bool tuning = a.m <= a.burnin;
        const bool upd_beta = (a.mask >> 5) & 1u;
        const int N = S.N, R = S.R;
        const HyperState &H = *S.hyp;
        double thd[kMaxL], s2[kMaxL];
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) {
            thd[l] = l < L ? H.theta[l] : 0.0;
            s2[l] = l < L ? H.sig2[l] : 1.0;
        }
        T beta[kMaxL], wb[kMaxL], wab[kMaxL];
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) {
            const bool on = l < L && active;
            const int64_t idx = (int64_t)l * Gp + g;
            beta[l] = on ? ((const T *)S.beta)[idx] : (T)0;
            wb[l] = (on && upd_beta) ? ((const T *)S.w_beta)[idx] : (T)1;
            wab[l] = (on && upd_beta && tuning) ? ((const T *)S.wa_beta)[idx] : (T)0;
        }
        T A[kMaxRows], YR[kMaxRows];
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            A[r] = (T)0;
            YR[r] = (r < R && active) ? ((const T *)S.YR)[(int64_t)r * Gp + g] : (T)0;
        }
        if (active) {
            const T *__restrict__ eps = (const T *)S.eps;
#pragma unroll 8
            for (int n = 0; n < N; ++n) {
                const T ehe = dexp((T)S.h[n] + eps[(int64_t)n * Gp + g]);
                const int rr = S.row_of[n];
#pragma unroll
                for (int r = 0; r < kMaxRows; ++r)
                    if (r == rr) A[r] += ehe;
            }
        }
        T C[kMaxRows];
        row_sums_at_beta<T, kML>(S, A, beta, C);
        int bad = 0;
        // both lanes of a pair hold the same gene, so they enter together
        if (active && upd_beta)
            beta_slice_draws<T, kML, true>(S, a, g, Gp, lead, beta, wb, wab, thd, s2, C, YR, tuning, bad);
        if (lead) {
#pragma unroll
            for (int l = 0; l < kMaxL; ++l) sbeta[l][j] = (double)beta[l];
        }
        if (bad) report_cap(err, 5, S, g, a.m, -1);
    }
    __syncthreads();
    if constexpr (kShift) {
        if (wave == 1) shift_genes<T, kML>(S, tile, a);
        return;
    }
    if (wave == 0 && !((a.mask >> kKindShift) & 1u)) {
        const int64_t g = (int64_t)tile * kTile + lane;
        T beta[kMaxL];
#pragma unroll
        for (int l = 0; l < kMaxL; ++l) beta[l] = (T)sbeta[l][lane];
        beta_finish<T, kML>(S, a, g, Gp, g < S.G, beta, mob, th, tile, lane, tslot, trow, sampling);
    }
}

// ---------------------------------------------------------------------------
// Proposal network inference: one wavefront per block of 32 genes.  The
// layers run transposed, out^T = W^T in^T, on v_mfma_f32_32x32x16_bf16 with
// the packed weights (from LDS) as the A operand and the activations as the B
// operand.  Only the standardised features pass through LDS (one row per
// gene); after that the activations stay in registers: the accumulator tile of
// one layer, after bias, GELU and BF16 rounding, is register for register the
// B fragments of the next layer (hidden units numbered in wt_unit order).
// ---------------------------------------------------------------------------

// GELU(v) = v Phi(v) for inference, branch-free: with x = |v| / sqrt(2),
// q = erfc(x) from Abramowitz & Stegun 7.1.26 (q = t (a1 + t (a2 + ...)) e^(-x^2),
// t = 1 / (1 + p x), |error| <= 1.5e-7), Phi(v) = 1 - q / 2 for v >= 0 and
// q / 2 for v < 0 (no cancellation).  The activations are rounded to BF16
// right after, whose relative step (2^-8) is far above that error.
__device__ inline float gelu_f(float v)
{
    const float x = ::fabsf(v) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
    const float poly =
        t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
    const float q = poly * __expf(-x * x);
    return v >= 0.0f ? v * (1.0f - 0.5f * q) : v * (0.5f * q);
}

// Bias, GELU and BF16 rounding of one 32 x 32 output tile `ot`: register r of
// lane 32 h + i holds unit 32 ot + 8 (r / 4) + 4 h + r % 4, which is element
// r % 8 of the next layer's B fragment for k-step 2 ot + r / 8 (units in
// wt_unit order).
constexpr int kFrStride = kMlpF + 1;   // LDS feature-row stride (floats), odd against bank conflicts
// Standardised features (and, in training, whitened targets) are clipped to
// [-kPairClip, kPairClip], in training and in inference alike, so the network
// is never evaluated on inputs outside the range it was trained on.
constexpr float kPairClip = kMlpClip;
__device__ inline float clip_feature(float v) { return fminf(fmaxf(v, -kPairClip), kPairClip); }

// The network's parameters as a workgroup keeps them in LDS: the packed
// weights, then the feature standardisation and the biases (every per-lane
// read in the layers is an LDS read).
struct MlpLds {
    bf16x8 W[kWtFrags * 64];
    float fmean[kMlpF], fscale[kMlpF];
    float b1[kMlpH], b2[kMlpH], b3[kMlpO];
};

// The biases of one output tile, units 32 ot + 8 q + 4 h + t as float4 q.
__device__ inline void tile_bias(const float *bias, int ot, int h, float4 (&bb)[4])
{
    const float *bp = bias + 32 * ot + 4 * h;
#pragma unroll
    for (int q = 0; q < 4; ++q) bb[q] = *reinterpret_cast<const float4 *>(bp + 8 * q);
}

// Eight floats rounded to one BF16 fragment, built as a whole (element-wise
// insertion makes the compiler shuffle 64-bit registers around each element).
__device__ inline bf16x8 pack_bf16x8(const float (&v)[8])
{
    return bf16x8{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3],
                  (__bf16)v[4], (__bf16)v[5], (__bf16)v[6], (__bf16)v[7]};
}

__device__ inline void tile_to_next(const floatx16 &acc, const float *bias, int ot, int h, bf16x8 (&nx)[8])
{
    float4 bb[4];
    tile_bias(bias, ot, h, bb);
    float gv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float4 &b4 = bb[r >> 2];
        const float bv = (r & 3) == 0 ? b4.x : (r & 3) == 1 ? b4.y : (r & 3) == 2 ? b4.z : b4.w;
        gv[r] = gelu_f(acc[r] + bv);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        float v8[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v8[j] = gv[8 * q + j];
        nx[2 * ot + q] = pack_bf16x8(v8);
    }
}

// The network on 32 feature rows per wavefront, in the transposed form
// out^T = W^T in^T: v_mfma_f32_32x32x16_bf16 with A = packed weights (in LDS)
// and B = activations, so that each layer's accumulators become the next
// layer's B fragments in registers (tile_to_next).  `row` is the raw feature
// row of row i = lane % 32 (in LDS); lane 32 h + i takes features
// 16 ks + 8 h .. + 7 of it, standardised, as the layer-1 B fragment of k-step
// ks.  store(u, i, v) receives output u < O of row i (0..31) from lane
// 32 h + i for the units 8 q + 4 h + t it holds.
template <typename Store>
__device__ inline void mlp_block_x(const bf16x8 (&x1)[2], const MlpLds &P, int O, Store &&store)
{
    const bf16x8 *Wl = P.W;
    const int lane = (int)(threadIdx.x & 63);
    const int h = lane >> 5;
    bf16x8 h1[8], h2[8];
    const int nct3 = (O + 31) >> 5;
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        floatx16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wl[(2 * ot + ks) * 64 + lane], x1[ks], acc, 0, 0, 0);
        tile_to_next(acc, P.b1, ot, h, h1);
    }
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        // one output tile's weight fragments in flight at a time
        __builtin_amdgcn_sched_barrier(0);
        floatx16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wl[(8 + 8 * ot + ks) * 64 + lane], h1[ks], acc, 0, 0, 0);
        tile_to_next(acc, P.b2, ot, h, h2);
    }
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
        __builtin_amdgcn_sched_barrier(0);
        if (ot < nct3) {
            floatx16 acc = {};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wl[(40 + 8 * ot + ks) * 64 + lane], h2[ks], acc, 0, 0,
                                                              0);
            float4 bb[4];
            tile_bias(P.b3, ot, h, bb);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int u = 32 * ot + 8 * (r >> 2) + 4 * h + (r & 3);
                const float4 &b4 = bb[r >> 2];
                const float bv = (r & 3) == 0 ? b4.x : (r & 3) == 1 ? b4.y : (r & 3) == 2 ? b4.z : b4.w;
                if (u < O) store(u, lane & 31, acc[r] + bv);
            }
        }
    }
}

// The same from a raw feature row in LDS: standardised and rounded to BF16
// here (the layer-1 B fragments of lane 32 h + i).
template <typename Store>
__device__ inline void mlp_block(const float *row, bool active, const MlpLds &P, int O, Store &&store)
{
    const int h = (int)(threadIdx.x & 63) >> 5;
    bf16x8 x1[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        float v8[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 16 * ks + 8 * h + j;
            v8[j] = active ? clip_feature((row[k] - P.fmean[k]) * P.fscale[k]) : 0.0f;
        }
        x1[ks] = pack_bf16x8(v8);
    }
    mlp_block_x(x1, P, O, store);
}

// Copy of the network's parameters into the workgroup's LDS (all threads call).
__device__ inline void load_weights(MlpLds &P, const MlpDev *__restrict__ net)
{
    const bf16x8 *src = reinterpret_cast<const bf16x8 *>(net->Wt);
    for (int t = (int)threadIdx.x; t < kWtFrags * 64; t += (int)blockDim.x) P.W[t] = src[t];
    for (int t = (int)threadIdx.x; t < kMlpF; t += (int)blockDim.x) {
        P.fmean[t] = net->fmean[t];
        P.fscale[t] = net->fscale[t];
    }
    for (int t = (int)threadIdx.x; t < kMlpH; t += (int)blockDim.x) {
        P.b1[t] = net->b1[t];
        P.b2[t] = net->b2[t];
    }
    for (int t = (int)threadIdx.x; t < kMlpO; t += (int)blockDim.x) P.b3[t] = net->b3[t];
    __syncthreads();
}

// The proposal network of every gene in the sweep, after the eps draws and
// before the gamma/beta kernel: features from this sweep's eps (row sums A_r,
// Y_r) and the current theta, sigma^2, then the network; output u of gene g
// goes to mlp_out[u][g].  512 threads: eight wavefronts share the weights in
// LDS, each taking 32-gene blocks (half tiles) in turn.
constexpr int kFrStrideB = kMlpF + 8;   // BF16 feature-row stride: 80 B, 16-B aligned fragments

template <typename T, int kWaves>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8))) void mlp_sweep(
    const SegInfo *__restrict__ segs, const int2 *__restrict__ tiles, int ntiles, const MlpDev *__restrict__ net)
{
    __shared__ MlpLds P;
    // standardised feature rows of each wavefront's 32 genes, in BF16 (the
    // precision the first layer multiplies them in): written by lanes 0..31 at
    // positions that depend on the segment's R and L, read back as fragments.
    // BF16 rows keep a workgroup's LDS under half a CU's, so two workgroups
    // share a CU.
    __shared__ __align__(16) __bf16 frb[kWaves][32 * kFrStrideB];
    load_weights(P, net);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    __bf16 *rowb = &frb[wave][(lane & 31) * kFrStrideB];
    for (int bi = (int)blockIdx.x * kWaves + wave; bi < 2 * ntiles; bi += (int)gridDim.x * kWaves) {
        const int2 tt = tiles[bi >> 1];
        const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
        const int tile = __builtin_amdgcn_readfirstlane(tt.y);
        const SegInfo &S = segs[sidx];
        const int64_t Gp = S.Gp, g0 = (int64_t)tile * kTile + 32 * (bi & 1);
        const int64_t g = g0 + (lane & 31);
        const bool active = g < S.G;
        const int N = S.N, L = S.L, R = S.R;
        T A[kMaxRows], YR[kMaxRows];
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) {
            A[r] = (T)0;
            YR[r] = (r < R && active) ? ((const T *)S.YR)[(int64_t)r * Gp + g] : (T)0;
        }
        if (active) {
            const T *__restrict__ eps = (const T *)S.eps;
#pragma unroll 8
            for (int n = 0; n < N; ++n) {
                const T ehe = dexp((T)S.h[n] + eps[(int64_t)n * Gp + g]);
                const int rr = S.row_of[n];
#pragma unroll
                for (int r = 0; r < kMaxRows; ++r)
                    if (r == rr) A[r] += ehe;
            }
        }
        // the features of gene_features: log((Y_r + 1/2) / A_r), log(Y_r + 1/2),
        // theta_l, log sigma_l^2, zero to 32
        wave_lds_sync();                  // earlier readers of the rows are done
        if (lane < 32) {
            // feature k standardised as (phi_k - fmean_k) fscale_k, then BF16
            auto put = [&](int k, float v) { rowb[k] = (__bf16)clip_feature((v - P.fmean[k]) * P.fscale[k]); };
#pragma unroll
            for (int k = 0; k < kMlpF; ++k) put(k, 0.0f);
#pragma unroll
            for (int r = 0; r < kMaxRows; ++r)
                if (r < R) {
                    const float y = (float)YR[r] + 0.5f;
                    put(r, ::logf(y / (float)A[r]));
                    put(R + r, ::logf(y));
                }
#pragma unroll
            for (int l = 0; l < kMaxL; ++l)
                if (l < L) {
                    put(2 * R + l, (float)S.hyp->theta[l]);
                    put(2 * R + L + l, ::logf((float)S.hyp->sig2[l]));
                }
        }
        wave_lds_sync();
        bf16x8 x1[2];
        const bf16x8 *frag = reinterpret_cast<const bf16x8 *>(rowb);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) x1[ks] = active ? frag[2 * ks + (lane >> 5)] : bf16x8{};
        float *__restrict__ out = S.mlp_out;
        const int64_t G = S.G;
        mlp_block_x(x1, P, mlp_outputs(L), [&](int u, int rw, float v) {
            if (g0 + rw < G) out[(int64_t)u * Gp + g0 + rw] = v;
        });
    }
}

// The network on raw feature rows phi [B][32] (tests): mu, ls [B][L] and the
// factor's strict lower triangle off [B][L(L-1)/2] (units of oscale), through
// the same block routine as the sweep.
__global__ __launch_bounds__(512) void mlp_infer_raw(const float *__restrict__ phi, int64_t B, int L,
                                                     const MlpDev *__restrict__ net, float *mu_out, float *ls_out,
                                                     float *off_out)
{
    __shared__ MlpLds P;
    __shared__ float fr[8][32 * kFrStride];
    load_weights(P, net);
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t b0 = ((int64_t)blockIdx.x * 8 + wave) * 32;
    if (b0 >= B) return;                  // whole wavefront; no workgroup barrier follows
    const int64_t b = b0 + (lane & 31);
    const bool active = b < B;
    float *rowp = &fr[wave][(lane & 31) * kFrStride];
    if (lane < 32) {
#pragma unroll
        for (int k = 0; k < kMlpF; ++k) rowp[k] = active ? phi[b * kMlpF + k] : 0.0f;
    }
    wave_lds_sync();
    const int K = L * (L - 1) / 2;
    mlp_block(rowp, active, P, mlp_outputs(L), [&](int u, int row, float v) {
        const int64_t bb = b0 + row;
        if (bb >= B) return;
        if (u < L) mu_out[bb * L + u] = net->omean[u] + net->oscale[u] * v;
        else if (u < 2 * L) ls_out[bb * L + u - L] = ::logf(net->oscale[u - L]) + v;
        else off_out[bb * K + u - 2 * L] = v;
    });
}

// Features of every gene from the current state (tests): A_r and Y_r summed
// from eps and y, theta and sigma^2 from the hyperparameter state.
template <typename T>
__global__ void features_kernel(const SegInfo *__restrict__ seg, float *__restrict__ out)
{
    const SegInfo &S = *seg;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= S.G) return;
    const int N = S.N, L = S.L, R = S.R;
    T A[kMaxRows], YR[kMaxRows];
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) { A[r] = (T)0; YR[r] = (T)0; }
    for (int n = 0; n < N; ++n) {
        const int64_t idx = (int64_t)n * S.Gp + g;
        const T e = dexp((T)S.h[n] + ((const T *)S.eps)[idx]);
        const T y = (T)S.y[idx];
        const int rr = S.row_of[n];
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r)
            if (r == rr) { A[r] += e; YR[r] += y; }
    }
    double th[kMaxL], s2[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) {
        th[l] = l < L ? S.hyp->theta[l] : 0.0;
        s2[l] = l < L ? S.hyp->sig2[l] : 1.0;
    }
    float phi[32];
    gene_features<T>(S, A, YR, th, s2, phi);
    for (int k = 0; k < 32; ++k) out[g * 32 + k] = phi[k];
    (void)R;
}

// Minibatch gather: row i takes pair (Philox word of (i, step, epoch)) mod P,
// standardises its features and copies its targets, both clipped to
// [-kPairClip, kPairClip]: a gene whose Laplace approximation is far off (two
// Newton steps from a poor start) gives whitened draws in the tens, whose
// squared residuals would dominate the loss; the proposal stays exact under
// the MH correction whatever the network learns from them.
__global__ void gather_pairs(const float *__restrict__ pairs, int64_t P, int L, const float *__restrict__ master,
                             float *X, float *Tg, int B, uint32_t epoch, uint32_t step, uint32_t k0, uint32_t k1)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= B) return;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)i, step, epoch, 0xB0u), k0, k1);
    const int64_t p = (int64_t)(((uint64_t)r.x << 32 | r.y) % (uint64_t)P);
    const float *row = pairs + p * kPairStride;
    for (int k = 0; k < kMlpF; ++k) {
        const float v = (row[k] - master[kOffFmean + k]) * master[kOffFscale + k];
        X[(int64_t)i * kMlpF + k] = clip_feature(v);
    }
    for (int l = 0; l < L; ++l) Tg[(int64_t)i * L + l] = clip_feature(row[32 + l]);
}

// Column sums and sums of squares (FP64) of a row-major [rows][cols] float
// array, in two passes: block (c, k) sums column c over the k-th of kColChunks
// row ranges (thread t: rows t, t + 256, ... of the range in order, then a
// fixed-order tree) into part[(c kColChunks + k) 2 + {0, 1}]; col_moments_sum
// adds the chunks of a column in order.  The blocks of a row range share its
// cache lines.
__global__ __launch_bounds__(256) void col_moments(const float *__restrict__ M, int64_t rows, int cols, double *part)
{
    const int c = (int)blockIdx.x, k = (int)blockIdx.y;
    const int64_t r0 = rows * k / kColChunks, r1 = rows * (k + 1) / kColChunks;
    double s = 0.0, q = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const double v = M[r * cols + c];
        s += v;
        q += v * v;
    }
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = q;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * ((int64_t)c * kColChunks + k)] = sh[0][0];
        part[2 * ((int64_t)c * kColChunks + k) + 1] = sh[1][0];
    }
}

__global__ void col_moments_sum(const double *__restrict__ part, int cols, double *out)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= cols) return;
    double s = 0.0, q = 0.0;
    for (int k = 0; k < kColChunks; ++k) {
        s += part[2 * ((int64_t)c * kColChunks + k)];
        q += part[2 * ((int64_t)c * kColChunks + k) + 1];
    }
    out[2 * c] = s;
    out[2 * c + 1] = q;
}

hipError_t launch_mlp_infer_raw(const float *phi, int64_t B, int L, const MlpDev *net, float *mu, float *ls,
                                float *off, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_infer_raw, dim3((unsigned)((B + 255) / 256)), dim3(512), 0, st, phi, B, L, net, mu, ls,
                       off);
    return hipGetLastError();
}

hipError_t launch_mlp_sweep(int precision, const SegInfo *segs, const int2 *tiles, int ntiles, const MlpDev *net,
                            hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    // eight wavefronts per workgroup share one copy of the weights (four per
    // workgroup, which would spread small launches over more CUs, measured
    // slower at G = 50,000: 53.2 against 50.6 us for network and MH step)
    const int nwg = (2 * ntiles + 7) / 8;
    const dim3 grid((unsigned)(nwg < 512 ? nwg : 512)), block(512);
    if (precision == 1)
        hipLaunchKernelGGL((mlp_sweep<float, 8>), grid, block, 0, st, segs, tiles, ntiles, net);
    else
        hipLaunchKernelGGL((mlp_sweep<double, 8>), grid, block, 0, st, segs, tiles, ntiles, net);
    return hipGetLastError();
}

hipError_t launch_features(int precision, const SegInfo *seg, int64_t G, float *out, hipStream_t st)
{
    const unsigned blocks = (unsigned)((G + 255) / 256);
    if (precision == 0) hipLaunchKernelGGL((features_kernel<double>), dim3(blocks), dim3(256), 0, st, seg, out);
    else hipLaunchKernelGGL((features_kernel<float>), dim3(blocks), dim3(256), 0, st, seg, out);
    return hipGetLastError();
}

hipError_t launch_gather_pairs(const float *pairs, int64_t P, int L, const float *master, float *X, float *Tg,
                               int B, uint32_t epoch, uint32_t step, uint32_t k0, uint32_t k1, hipStream_t st)
{
    hipLaunchKernelGGL(gather_pairs, dim3((B + 255) / 256), dim3(256), 0, st, pairs, P, L, master, X, Tg, B,
                       epoch, step, k0, k1);
    return hipGetLastError();
}

// work: 2 cols kColChunks doubles
hipError_t launch_col_moments(const float *M, int64_t rows, int cols, double *work, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(col_moments, dim3(cols, kColChunks), dim3(256), 0, st, M, rows, cols, work);
    hipLaunchKernelGGL(col_moments_sum, dim3((cols + 63) / 64), dim3(64), 0, st, work, cols, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hyperparameter step: one 256-thread workgroup per segment
// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of the tile partials, then the draws on separate
// wavefronts: (nu, then tau) on wavefront 0, (theta_l, then sigma_l^2) on
// wavefront 1 + (l mod 3).  The pairs are conditionally independent of one
// another (nu and tau involve only gamma; theta_l and sigma_l^2 only column l
// of beta), so with counter-based random numbers their order does not matter.
constexpr int kHyperThreads = 256;
constexpr int kHyperWaves = kHyperThreads / 64;

// nu, then tau (Algorithm 1 steps 3 and 4) on one wavefront: every lane
// computes the draws, lane 0 stores.  r0 = sum log gamma_g, r1 = sum 1/gamma_g.
// Hi holds the state before the step and Ho receives the new values of these
// two parameters (their widths, moments, reductions and records); the two may
// be the same object.  Returns whether a draw reached the shrink cap.
__device__ inline bool draw_nu_tau(const SegInfo &S, const SweepArgs &a, const HyperState &Hi, HyperState &Ho,
                                   double r0, double r1, double *wd)
{
    const double G = (double)S.G;
    const uint32_t k0 = S.key0, k1 = S.key1;
    const uint32_t mm = (uint32_t)a.m;
    const uint32_t chain = (uint32_t)S.chain;
    const bool exact = (a.mask >> kKindExact) & 1u;
    const bool w0 = (threadIdx.x & 63) == 0;
    bool bad = false;
    DrawRec rec;
    double nu = Hi.nu, tau = Hi.tau;
    if ((a.mask >> 3) & 1u) {
        NuF f{G, tau, r0, r1, S.d};
        double w = Hi.w_nu, wa = Hi.wa_nu;
        const double x1 = slice_draw_wave(f, nu, w, k0, k1, draw_counter(0, 3, 0, mm, chain, 0), a.K, a.cap, rec, wd);
        tune_width<double>(w, wa, nu, x1, a.m, a.burnin, a.tune_start);
        nu = x1;
        if (w0) { Ho.nu = x1; Ho.w_nu = w; Ho.wa_nu = wa; }
        bad |= rec.bad;
        if (a.dbg && w0) Ho.dbg[0] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
    }
    if ((a.mask >> 4) & 1u) {
        // rate of tau's Gamma prior: b, or the top level's b in the three-level form
        const double rate_b = S.top != nullptr ? S.top->b : S.b;
        TauF f{S.a + 0.5 * G * nu - 1.0, rate_b + 0.5 * nu * r1};
        int tries = 0;
        if (exact) {
            // exact draw, the same on every lane: tau = X / rate, X ~ Gamma(a + G nu / 2)
            double v = 0.0;
            tries = exact_gamma_draw(kKindExact, f.shape_m1 + 1.0, f.rate, false, __builtin_inf(), k0, k1, 0, 1, mm,
                                     chain, v);
            if (tries > 0) {
                tau = v;
                if (w0) Ho.tau = v;
                if (a.dbg && w0) Ho.dbg[1] = make_int4(-1, 0, 0, tries);
            }
        }
        if (tries == 0) {
            double w = Hi.w_tau, wa = Hi.wa_tau;
            const double x1 = slice_draw_wave(f, tau, w, k0, k1, draw_counter(0, 4, 0, mm, chain, 0), a.K, a.cap,
                                              rec, wd);
            tune_width<double>(w, wa, tau, x1, a.m, a.burnin, a.tune_start);
            tau = x1;
            if (w0) { Ho.tau = x1; Ho.w_tau = w; Ho.wa_tau = wa; }
            bad |= rec.bad;
            if (a.dbg && w0) Ho.dbg[1] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
        }
    }
    if (w0) {
        Ho.red[0] = r0;
        Ho.red[1] = r1;
        if (a.m > a.burnin) {
            double2 m0 = Hi.mom[0], m1 = Hi.mom[1];
            welford(m0, nu, a.inv_k);
            welford(m1, tau, a.inv_k);
            Ho.mom[0] = m0;
            Ho.mom[1] = m1;
        }
        if (a.trace_point >= 0) {
            float *trow = S.trace + (int64_t)a.trace_point * S.trace_stride;
            trow[0] = (float)nu;
            trow[1] = (float)tau;
        }
    }
    return bad;
}

// theta_l, then sigma_l^2 (Algorithm 1 steps 6 and 7) on one wavefront, as
// draw_nu_tau.  d1, d2 are the sums of (beta_gl - s) and (beta_gl - s)^2 with
// the shift s = theta_l before this step.
__device__ inline bool draw_theta_sig2(const SegInfo &S, const SweepArgs &a, const HyperState &Hi, HyperState &Ho,
                                       int l, double d1, double d2, double *wd)
{
    const int L = S.L;
    const double G = (double)S.G;
    const uint32_t k0 = S.key0, k1 = S.key1;
    const uint32_t mm = (uint32_t)a.m;
    const uint32_t chain = (uint32_t)S.chain;
    const bool exact = (a.mask >> kKindExact) & 1u;
    const bool w0 = (threadIdx.x & 63) == 0;
    bool bad = false;
    DrawRec rec;
    const double s = Hi.theta[l];
    const double sb = d1 + G * s;
    const double sig2 = Hi.sig2[l];
    double th = s;
    if ((a.mask >> 6) & 1u) {
        const double cl = S.c[l];
        const double prec = G / sig2 + 1.0 / (cl * cl);
        // prior N(0, c_l^2), or N(psi_l, c_l^2) under a top level
        const double mean = S.top != nullptr ? (sb / sig2 + S.top->psi[l] / (cl * cl)) / prec : (sb / sig2) / prec;
        const uint4 r = philox4x32_10(draw_counter(0, 6, (uint32_t)l, mm, chain, 0), k0, k1);
        const double zn = ::sqrt(-2.0 * ::log(u01<double>(r.x))) * ::cos(6.283185307179586 * u01<double>(r.y));
        th = mean + zn / ::sqrt(prec);
    }
    const double dt = th - s;
    const double Ssq = d2 - 2.0 * dt * d1 + G * dt * dt;
    double s2new = sig2;
    double w = Hi.w_sig2[l], wa = Hi.wa_sig2[l];
    if ((a.mask >> 7) & 1u) {
        const double sl = S.s[l];
        int tries = 0;
        if (exact) {
            // exact draw: sigma^2 = (S/2) / X, X ~ Gamma((G - 1)/2), kept below s_l^2
            tries = exact_gamma_draw(kKindExact, 0.5 * (G - 1.0), 0.5 * Ssq, true, sl * sl, k0, k1, 0, 2u + (uint32_t)l,
                                     mm, chain, s2new);
            if (tries > 0 && a.dbg && w0) Ho.dbg[2 + l] = make_int4(-1, 0, 0, tries);
        }
        if (tries == 0) {
            Sig2F f{0.5 * (G + 1.0), Ssq, sl * sl};
            s2new = slice_draw_wave(f, sig2, w, k0, k1, draw_counter(0, 7, (uint32_t)l, mm, chain, 0), a.K, a.cap, rec,
                                    wd);
            tune_width<double>(w, wa, sig2, s2new, a.m, a.burnin, a.tune_start);
            bad |= rec.bad;
            if (a.dbg && w0) Ho.dbg[2 + l] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
        }
    }
    if (w0) {
        Ho.theta[l] = th;
        Ho.sig2[l] = s2new;
        Ho.w_sig2[l] = w;
        Ho.wa_sig2[l] = wa;
        Ho.red[2 + 2 * l] = sb;
        Ho.red[3 + 2 * l] = Ssq;
        if (a.m > a.burnin) {
            double2 mt = Hi.mom[2 + l], ms = Hi.mom[2 + L + l];
            welford(mt, th, a.inv_k);
            welford(ms, s2new, a.inv_k);
            Ho.mom[2 + l] = mt;
            Ho.mom[2 + L + l] = ms;
        }
        if (a.trace_point >= 0) {
            float *trow = S.trace + (int64_t)a.trace_point * S.trace_stride;
            trow[2 + l] = (float)th;
            trow[2 + L + l] = (float)s2new;
        }
    }
    return bad;
}

// Partial columns the reductions add: the tiles, then (learned step) the
// fallback groups, which hold beta partials of their own unless the shift step
// takes every gene's partials in its tile column.
__device__ inline int64_t partial_columns(const SegInfo &S, const SweepArgs &a)
{
    return S.ntiles + ((a.learned && !((a.mask >> kKindShift) & 1u)) ? S.nfbw : 0);
}

// The whole hyperparameter step of one segment on one 256-thread workgroup:
// the reductions, then (nu, then tau) on wavefront 0 and (theta_l, then
// sigma_l^2) on wavefront 1 + (l mod 3).  publish > 0 (the single-launch
// sweep) sets the segment's flags of chains 0..L to `publish`, the index of
// the sweep whose gene draws read the new values, once they are written.
__device__ inline void hyper_block(const SegInfo &S, const SweepArgs &a, int *err, int64_t publish = 0)
{
    const int L = S.L;
    const int nparts = 2 + 2 * L;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    __shared__ double part[kHyperWaves][kMaxParts];
    __shared__ double red[kMaxParts];
    __shared__ double words[kHyperWaves][20];
    // The hyperparameter state is staged in LDS: the draws are short serial
    // chains, and LDS keeps each dependent access at LDS latency.
    __shared__ HyperState H;
    constexpr int kWords = (int)(sizeof(HyperState) / sizeof(double));
    static_assert(sizeof(HyperState) % sizeof(double) == 0, "HyperState must be whole doubles");
    double *hs = reinterpret_cast<double *>(&H);
    const double *hg = reinterpret_cast<const double *>(S.hyp);
    for (int i = tid; i < kWords; i += kHyperThreads) hs[i] = hg[i];

    // thread t sums columns t, t + 256, ... in order; a butterfly inside each
    // wavefront; the wavefronts in order (hyper_chain adds in the same order).
    const int64_t nt = partial_columns(S, a);
    for (int j0 = 0; j0 < nparts; j0 += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
        for (int64_t t = tid; t < nt; t += kHyperThreads) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = j0 + q < nparts ? S.partials[(int64_t)(j0 + q) * S.pstride + t] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += v[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double r = wave_sum(acc[q]);
            if (lane == 0 && j0 + q < nparts) part[wave][j0 + q] = r;
        }
    }
    __syncthreads();
    if (tid < nparts) {
        double s = 0.0;
        for (int w = 0; w < kHyperWaves; ++w) s += part[w][tid];
        red[tid] = s;
    }
    __syncthreads();

    double *wd = &words[wave][0];
    if (wave == 0) {
        if (draw_nu_tau(S, a, H, H, red[0], red[1], wd) && lane == 0) report_cap(err, 3, S, -1, a.m, 0);
    } else {
        for (int l = wave - 1; l < L; l += kHyperWaves - 1)
            if (draw_theta_sig2(S, a, H, H, l, red[2 + 2 * l], red[3 + 2 * l], wd) && lane == 0)
                report_cap(err, 3, S, -1, a.m, 1 + l);
    }
    __syncthreads();
    double *hw = reinterpret_cast<double *>(S.hyp);
    for (int i = tid; i < kWords; i += kHyperThreads) hw[i] = hs[i];
    if (publish > 0) {
        // every wavefront's stores visible device-wide, then the flag
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid <= L) __hip_atomic_store(&S.hyp_flag[tid], publish, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One chain of the hyperparameter step on its own 256-thread workgroup:
// c = 0 draws nu then tau, c = 1 + l draws theta_l then sigma_l^2 (c > L: no
// work).  The chains are conditionally independent of one another, so 1 + L
// workgroups per segment run them at once, each reducing only the two partial
// sums it needs; its loads of all columns of a thread are issued together.
// The sums are added in hyper_block's order, so the draws are the same bits.
// The workgroup stages the state in LDS and writes back only its chain's
// fields to the segment's HyperState.  publish > 0 (the single-launch sweep)
// then sets the chain's flag to `publish`.
__device__ inline void hyper_chain(const SegInfo &S, const SweepArgs &a, int *err, int c, int64_t publish = 0)
{
    if (c > S.L) return;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    __shared__ double part[kHyperWaves][2];
    __shared__ double words[20];
    __shared__ HyperState H;
    constexpr int kWords = (int)(sizeof(HyperState) / sizeof(double));
    double *hs = reinterpret_cast<double *>(&H);
    const double *hg = reinterpret_cast<const double *>(S.hyp);
    for (int i = tid; i < kWords; i += kHyperThreads) hs[i] = hg[i];

    const int64_t nt = partial_columns(S, a);
    const double *p0 = S.partials + (int64_t)(2 * c) * S.pstride;
    const double *p1 = p0 + S.pstride;
    constexpr int kCols = 4;     // columns per thread per round trip
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t t0 = tid; t0 < nt; t0 += kCols * kHyperThreads) {
        double v0[kCols], v1[kCols];
#pragma unroll
        for (int q = 0; q < kCols; ++q) {
            const int64_t t = t0 + (int64_t)q * kHyperThreads;
            v0[q] = t < nt ? p0[t] : 0.0;
            v1[q] = t < nt ? p1[t] : 0.0;
        }
        // adding 0.0 past the last column leaves the sum's bits unchanged (it
        // starts at +0.0, so it is never -0.0)
#pragma unroll
        for (int q = 0; q < kCols; ++q) {
            acc0 += v0[q];
            acc1 += v1[q];
        }
    }
    const double w0s = wave_sum(acc0), w1s = wave_sum(acc1);
    if (lane == 0) {
        part[wave][0] = w0s;
        part[wave][1] = w1s;
    }
    __syncthreads();
    if (wave != 0) return;
    double r0 = 0.0, r1 = 0.0;
    for (int w = 0; w < kHyperWaves; ++w) {
        r0 += part[w][0];
        r1 += part[w][1];
    }
    HyperState &Ho = *S.hyp;
    const bool bad = c == 0 ? draw_nu_tau(S, a, H, Ho, r0, r1, words)
                            : draw_theta_sig2(S, a, H, Ho, c - 1, r0, r1, words);
    if (bad && lane == 0) report_cap(err, 3, S, -1, a.m, c);
    if (publish > 0) {
        // lane 0's stores of the new values visible device-wide, then the flag
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(&S.hyp_flag[c], publish, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Top level of the three-level form (Section 2.3): one workgroup per chain
// ---------------------------------------------------------------------------
// Given the groups' hyperparameters phi the top level is independent of the
// genes, so psi(m) is drawn from phi(m - 1) after the gene kernels of sweep m
// and before its hyperparameter step, which reads it:
//   b     ~ Gamma(a_b + sum_k a_k, rate b_b + sum_k tau_k)             (bit 0)
//   psi_l ~ N(v sum_k theta_kl / c_kl^2, v), 1/v = 1/c0_l^2 + sum_k 1/c_kl^2 (bit 1)
// The groups of chain c are the segments k * chains + c, summed over k in
// order.  Philox (0, kKindTop << 24 | sub, m, chain << 16 | j): psi_l sub = l,
// Box-Muller on block 0; b sub = 128, a Gamma variate (exact_gamma_draw); when
// no attempt succeeds b keeps its value.  Lane i stages group k0 + i's terms
// a_k, tau_k, 1/c_kl^2 and theta_kl/c_kl^2 in LDS (loads and FP64 divisions
// of 64 groups at a time in parallel); then lane l < L adds up psi_l's sums in
// group order and draws psi_l, and lane kMaxL does the same for b.
__global__ __launch_bounds__(64) void top_sweep(const SegInfo *__restrict__ segs, int nseg, int chains,
                                                 TopState *__restrict__ top, TopPriors P, SweepArgs a0)
{
    __shared__ double va[64], vt[64], vq[64][kMaxL], vp[64][kMaxL];
    const SweepArgs a = resolve_args(a0);
    const int chain = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    const int L = P.L;
    const int K = (nseg - chain + chains - 1) / chains;    // groups of this chain: segments k * chains + chain
    const bool psi_lane = lane < L, b_lane = lane == kMaxL;
    double c0l = 1.0;
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) c0l = l == lane ? P.c0[l] : c0l;
    // psi lanes: precision and weighted sum of psi_lane; b lane: sum a_k, sum tau_k
    double s1 = psi_lane ? 1.0 / (c0l * c0l) : 0.0, s2 = 0.0;
    for (int k0 = 0; k0 < K; k0 += 64) {
        const int k = k0 + lane;
        if (k < K) {
            const SegInfo &S = segs[(int64_t)k * chains + chain];
            const HyperState *H = S.hyp;
            va[lane] = S.a;
            vt[lane] = H->tau;
#pragma unroll
            for (int l = 0; l < kMaxL; ++l) {
                if (l < L) {
                    const double ckl = S.c[l];
                    vp[lane][l] = 1.0 / (ckl * ckl);
                    vq[lane][l] = H->theta[l] / (ckl * ckl);
                }
            }
        }
        __syncthreads();
        const int n = K - k0 < 64 ? K - k0 : 64;
        if (psi_lane) {
            for (int i = 0; i < n; ++i) {
                s1 += vp[i][lane];
                s2 += vq[i][lane];
            }
        } else if (b_lane) {
            for (int i = 0; i < n; ++i) {
                s1 += va[i];
                s2 += vt[i];
            }
        }
        __syncthreads();
    }
    TopState &T = top[chain];
    const uint32_t mm = (uint32_t)a.m;
    const bool sampling = a.m > a.burnin;
    if (psi_lane) {
        double psi = T.psi[lane];
        if (P.mask & 2u) {
            const uint4 r = philox4x32_10(draw_counter(0, kKindTop, (uint32_t)lane, mm, (uint32_t)chain, 0),
                                          P.key0, P.key1);
            const double zn = ::sqrt(-2.0 * ::log(u01<double>(r.x))) * ::cos(6.283185307179586 * u01<double>(r.y));
            psi = s2 / s1 + zn / ::sqrt(s1);
            T.psi[lane] = psi;
        }
        if (sampling) welford(T.mom[1 + lane], psi, a.inv_k);
    } else if (b_lane) {
        double b = T.b;
        if (P.mask & 1u) {
            double v = 0.0;
            const int t = exact_gamma_draw(kKindTop, P.a_b + s1, P.b_b + s2, false, __builtin_inf(), P.key0, P.key1,
                                           0, 128u, mm, (uint32_t)chain, v);
            if (t > 0) b = v;
            T.b = b;
            T.tries = t;
        }
        if (sampling) welford(T.mom[0], b, a.inv_k);
    }
}

hipError_t launch_top(const SegInfo *segs, int nseg, int chains, TopState *top, const TopPriors &P,
                      const SweepArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(top_sweep, dim3(chains), dim3(64), 0, st, segs, nseg, chains, top, P, a);
    return hipGetLastError();
}

// The hyperparameter step as a kernel of its own: hsplit workgroups per
// segment, one per chain of draws (hyper_chain), or with hsplit = 1 one per
// segment (hyper_block).
__global__ __launch_bounds__(kHyperThreads) void hyper_sweep(const SegInfo *__restrict__ segs, SweepArgs a0, int hsplit,
                                                             int *err)
{
    const int b = (int)blockIdx.x;
    if (hsplit == 1) hyper_block(segs[b], resolve_args(a0), err);
    else hyper_chain(segs[b / hsplit], resolve_args(a0), err, b % hsplit);
}

// Step 1 of sweep a.m over the work items; when nhyp > 0 the first nhyp
// workgroups run the hyperparameter step of the previous sweep ha.m alongside
// (hsplit per segment as in hyper_sweep), since no eps conditional involves a
// hyperparameter.
// The register budget is set for the eps wavefronts (7 per SIMD); the FP64
// hyperparameter code, which runs on one workgroup per segment, spills.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 8))) void eps_sweep(
    const SegInfo *__restrict__ segs, const int4 *__restrict__ items, int nitems, SweepArgs a0, int nhyp,
    int hsplit, SweepArgs ha, int *err)
{
    if ((int)blockIdx.x < nhyp) {
        const int b = (int)blockIdx.x;
        if (hsplit == 1) hyper_block(segs[b], resolve_args(ha), err);
        else hyper_chain(segs[b / hsplit], resolve_args(ha), err, b % hsplit);
        return;
    }
    const SweepArgs a = resolve_args(a0);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int it = ((int)blockIdx.x - nhyp) * 4 + wave;
    if (it >= nitems) return;
    const int4 w = items[it];
    const int sidx = __builtin_amdgcn_readfirstlane(w.x);
    const int tile = __builtin_amdgcn_readfirstlane(w.y);
    const int n0 = __builtin_amdgcn_readfirstlane(w.z);
    const int n1 = __builtin_amdgcn_readfirstlane(w.w);
    eps_wave<T>(segs[sidx], tile, n0, n1, a, err);
}

// ---------------------------------------------------------------------------
// Single-launch sweep (slice steps, one lane per gene for beta): one
// 256-thread workgroup per tile.  Its four wavefronts draw the tile's eps
// (wavefront w takes samples w s .. w s + s - 1, s = ceil(N / 4)), keeping the
// new eps_gn and exp(h_n + eps_gn) in LDS; after a workgroup barrier
// wavefront 0 draws gamma_g and wavefront 1 beta_g from them, the same
// operations in the same order as eps_sweep followed by gb_sweep, so the
// chain is the same bit for bit.  A tile's gamma and beta draws need the
// previous sweep's hyperparameters; its eps draws do not, so the step runs
// in the launch's first workgroups (per segment one per chain of draws, or
// one) while the tiles draw eps, and publishes the sweep index on the
// segment's flag of each chain; after the barrier wavefront 0 waits (bounded)
// for the flag of (nu, tau) and wavefront 1 for those of (theta_l, sigma_l^2).
// The hyperparameter workgroups have the lowest indices and wait for nothing,
// so they are dispatched and finish whatever the other workgroups do.
// ---------------------------------------------------------------------------
constexpr int64_t kHyperSpins = 1 << 22;   // polls before a wait is abandoned (flag bit 4)

// Waits until the flags of chains c0..c1 hold at least m.  Polls are relaxed
// device-scope loads (no cache invalidation per poll); one acquire fence after
// the flags are seen orders the hyperparameter reads after them.
__device__ inline void wait_hyper(const SegInfo &S, int64_t m, int c0, int c1, int *err)
{
    int64_t spins = 0;
    for (int c = c0; c <= c1; ++c) {
        while (__hip_atomic_load(&S.hyp_flag[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < m) {
            if (++spins > kHyperSpins) {
                if ((threadIdx.x & 63) == 0) raise_flag(err, 4);
                c = c1;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename T, int kML>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void sweep_tile(const SegInfo *__restrict__ segs, const int2 *__restrict__ tiles,
                                                  int ntiles, SweepArgs a0, int nhyp, int hsplit, SweepArgs ha,
                                                  int *err)
{
    const SweepArgs a = resolve_args(a0);
    if ((int)blockIdx.x < nhyp) {
        const int b = (int)blockIdx.x;
        if (hsplit == 1) hyper_block(segs[b], resolve_args(ha), err, a.m);
        else hyper_chain(segs[b / hsplit], resolve_args(ha), err, b % hsplit, a.m);
        return;
    }
    const int tix = (int)blockIdx.x - nhyp;
    if (tix >= ntiles) return;     // the whole workgroup
    extern __shared__ __align__(16) unsigned char tile_lds[];
    const int2 tt = tiles[tix];
    const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
    const int tile = __builtin_amdgcn_readfirstlane(tt.y);
    const SegInfo &S = segs[sidx];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int N = S.N;
    T *se = reinterpret_cast<T *>(tile_lds);
    T *sx = se + N * kTile;
    const int s = (N + 3) / 4;
    const int n0 = wave * s < N ? wave * s : N;
    const int n1 = n0 + s < N ? n0 + s : N;
    eps_wave<T>(S, tile, n0, n1, a, err, se, sx);
    __syncthreads();
    if (wave >= 2) return;
    if (nhyp > 0) {
        if (wave == 0) wait_hyper(S, a.m, 0, 0, err);
        else wait_hyper(S, a.m, 1, S.L, err);
    }
    const int64_t g = (int64_t)tile * kTile + lane;
    if (wave == 0) gamma_wave<T, kML>(S, tile, a, err, se);
    else beta_genes<T, 0, kML>(S, g, g < S.G, tile, false, a, nullptr, err, sx);
}

__global__ void philox_kernel(const uint4 *ctr, const uint2 *key, uint4 *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], key[i].x, key[i].y);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_eps(int precision, const SegInfo *segs, const int4 *items, int nitems, const SweepArgs &a,
                      int nhyp_seg, int hsplit, const SweepArgs &ha, int *err, hipStream_t st)
{
    const int nhyp = nhyp_seg * hsplit;
    const int blocks = nhyp + (nitems + 3) / 4;
    if (blocks == 0) return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL((eps_sweep<double>), dim3(blocks), dim3(256), 0, st, segs, items, nitems, a, nhyp, hsplit,
                           ha, err);
    else
        hipLaunchKernelGGL((eps_sweep<float>), dim3(blocks), dim3(256), 0, st, segs, items, nitems, a, nhyp, hsplit,
                           ha, err);
    return hipGetLastError();
}

// maxN: the largest N over the segments (LDS: new eps and exp(h + eps) of a tile)
hipError_t launch_tile(int precision, int maxL, int maxN, const SegInfo *segs, const int2 *tiles, int ntiles,
                       const SweepArgs &a, int nhyp_seg, int hsplit, const SweepArgs &ha, int *err, hipStream_t st)
{
    const int nhyp = nhyp_seg * hsplit;
    const int blocks = nhyp + ntiles;
    if (blocks == 0) return hipSuccess;
    const dim3 grid((unsigned)blocks), block(256);
    if (precision == 0) {
        const size_t lds = 2 * (size_t)maxN * kTile * sizeof(double);
        if (maxL <= 5)
            hipLaunchKernelGGL((sweep_tile<double, 5>), grid, block, lds, st, segs, tiles, ntiles, a, nhyp, hsplit, ha,
                               err);
        else
            hipLaunchKernelGGL((sweep_tile<double, kMaxL>), grid, block, lds, st, segs, tiles, ntiles, a, nhyp, hsplit, ha,
                               err);
    } else {
        const size_t lds = 2 * (size_t)maxN * kTile * sizeof(float);
        if (maxL <= 5)
            hipLaunchKernelGGL((sweep_tile<float, 5>), grid, block, lds, st, segs, tiles, ntiles, a, nhyp, hsplit, ha,
                               err);
        else
            hipLaunchKernelGGL((sweep_tile<float, kMaxL>), grid, block, lds, st, segs, tiles, ntiles, a, nhyp, hsplit, ha,
                               err);
    }
    return hipGetLastError();
}

// mode: 0 slice steps, 1 learned kernel (any sweep), 2 learned MH step only;
// kML: the smallest compiled bound (5 or kMaxL) on every segment's L.
template <int kMode, int kML>
static void launch_gb_k(int precision, const SegInfo *segs, const int2 *tiles, int ntiles, const int4 *fb_items,
                        int nfb, const SweepArgs &a, const MlpDev *net, int *err, hipStream_t st)
{
    const dim3 block(128), grid(ntiles + nfb);
    if (precision == 0)
        hipLaunchKernelGGL((gb_sweep<double, kMode, kML>), grid, block, 0, st, segs, tiles, ntiles, fb_items, nfb, a,
                           net, err);
    else
        hipLaunchKernelGGL((gb_sweep<float, kMode, kML>), grid, block, 0, st, segs, tiles, ntiles, fb_items, nfb, a,
                           net, err);
}

template <int kMode>
static void launch_gb_m(int precision, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                        const int4 *fb_items, int nfb, const SweepArgs &a, const MlpDev *net, int *err,
                        hipStream_t st)
{
    if (maxL <= 5) launch_gb_k<kMode, 5>(precision, segs, tiles, ntiles, fb_items, nfb, a, net, err, st);
    else launch_gb_k<kMode, kMaxL>(precision, segs, tiles, ntiles, fb_items, nfb, a, net, err, st);
}

hipError_t launch_gb(int precision, int mode, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                     const int4 *fb_items, int nfb, const SweepArgs &a, const MlpDev *net, int *err, hipStream_t st)
{
    if (ntiles == 0) return hipSuccess;
    if (mode == 0) launch_gb_m<0>(precision, maxL, segs, tiles, ntiles, fb_items, 0, a, net, err, st);
    else if (mode == 1) launch_gb_m<1>(precision, maxL, segs, tiles, ntiles, fb_items, nfb, a, net, err, st);
    else launch_gb_m<2>(precision, maxL, segs, tiles, ntiles, fb_items, nfb, a, net, err, st);
    return hipGetLastError();
}

template <int kMode>
static void launch_gb_shift_m(int precision, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                              const SweepArgs &a, const MlpDev *net, int *err, hipStream_t st)
{
    const dim3 grid((unsigned)ntiles), block(128);
    if (precision == 1) {
        if (maxL <= 5)
            hipLaunchKernelGGL((gb_shift_sweep<float, kMode, 5>), grid, block, 0, st, segs, tiles, ntiles, a, net, err);
        else
            hipLaunchKernelGGL((gb_shift_sweep<float, kMode, kMaxL>), grid, block, 0, st, segs, tiles, ntiles, a, net,
                               err);
    } else {
        if (maxL <= 5)
            hipLaunchKernelGGL((gb_shift_sweep<double, kMode, 5>), grid, block, 0, st, segs, tiles, ntiles, a, net,
                               err);
        else
            hipLaunchKernelGGL((gb_shift_sweep<double, kMode, kMaxL>), grid, block, 0, st, segs, tiles, ntiles, a,
                               net, err);
    }
}

template <bool kShift>
static void launch_gb_pair_s(int precision, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                             const SweepArgs &a, int *err, hipStream_t st)
{
    const dim3 grid((unsigned)ntiles), block(192);
    if (precision == 1) {
        if (maxL <= 5)
            hipLaunchKernelGGL((gb_pair_sweep<float, 5, kShift>), grid, block, 0, st, segs, tiles, ntiles, a, err);
        else
            hipLaunchKernelGGL((gb_pair_sweep<float, kMaxL, kShift>), grid, block, 0, st, segs, tiles, ntiles, a,
                               err);
    } else {
        if (maxL <= 5)
            hipLaunchKernelGGL((gb_pair_sweep<double, 5, kShift>), grid, block, 0, st, segs, tiles, ntiles, a, err);
        else
            hipLaunchKernelGGL((gb_pair_sweep<double, kMaxL, kShift>), grid, block, 0, st, segs, tiles, ntiles, a,
                               err);
    }
}

hipError_t launch_gb_pair(int precision, int maxL, bool shift, const SegInfo *segs, const int2 *tiles, int ntiles,
                          const SweepArgs &a, int *err, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (shift) launch_gb_pair_s<true>(precision, maxL, segs, tiles, ntiles, a, err, st);
    else launch_gb_pair_s<false>(precision, maxL, segs, tiles, ntiles, a, err, st);
    return hipGetLastError();
}

// mode 0: slice steps; 2: the MH-only learned kernel (no fallback groups)
hipError_t launch_gb_shift(int precision, int mode, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                           const SweepArgs &a, const MlpDev *net, int *err, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (mode == 0) launch_gb_shift_m<0>(precision, maxL, segs, tiles, ntiles, a, net, err, st);
    else if (mode == 2) launch_gb_shift_m<2>(precision, maxL, segs, tiles, ntiles, a, net, err, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_shift(int precision, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                        const SweepArgs &a, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ntiles + 3) / 4)), block(256);
    if (precision == 1) {
        if (maxL <= 5) hipLaunchKernelGGL((shift_sweep<float, 5>), grid, block, 0, st, segs, tiles, ntiles, a);
        else hipLaunchKernelGGL((shift_sweep<float, kMaxL>), grid, block, 0, st, segs, tiles, ntiles, a);
    } else {
        if (maxL <= 5) hipLaunchKernelGGL((shift_sweep<double, 5>), grid, block, 0, st, segs, tiles, ntiles, a);
        else hipLaunchKernelGGL((shift_sweep<double, kMaxL>), grid, block, 0, st, segs, tiles, ntiles, a);
    }
    return hipGetLastError();
}

hipError_t launch_hyper(const SegInfo *segs, int nseg, int hsplit, const SweepArgs &a, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(hyper_sweep, dim3(nseg * hsplit), dim3(kHyperThreads), 0, st, segs, a, hsplit, err);
    return hipGetLastError();
}

hipError_t launch_philox(const uint4 *ctr, const uint2 *key, uint4 *out, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ctr, key, out, n);
    return hipGetLastError();
}

}  // namespace fbmc
