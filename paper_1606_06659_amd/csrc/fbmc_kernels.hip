// fbmc_kernels.hip -- the sweep kernels of libfbmc for gfx950.
//
// One sweep of Algorithm 1 is two launches:
//
//  gene_sweep<T>   one lane per gene, one wavefront per 64-gene tile.  Per gene it
//                  draws eps_g1..eps_gN (step 1), gamma_g (step 2) and
//                  beta_g1..beta_gL in order (step 5), updates the running
//                  moments, and leaves per-tile FP64 partial sums for the
//                  reductions of steps 3, 4, 6 and 7.  Running steps 1, 2 and 5
//                  back to back is the same Markov chain as the printed order:
//                  eps and beta do not depend on nu or tau, and nu, tau do not
//                  depend on beta, so swapping step 5 ahead of steps 3-4 changes
//                  no conditional and, with counter-based random numbers, no draw.
//  hyper_sweep     one workgroup per segment: fixed-order reduction of the tile
//                  partials, then nu and tau (slice), theta_l (Normal) and
//                  sigma_l^2 (slice) in FP64, hyperparameter moments and trace.
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
#include "fbmc_device.hpp"
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

template <typename T>
struct BetaF {
    T Y, x0, dth, inv_s2;
    T Gk[kMaxVals], vk[kMaxVals];
    T em1[kMaxVals];   // expm1(v_k d) at the last evaluated point
    int nv;
    __device__ T base(T) const { return (T)0; }
    __device__ T operator()(T x) {
        const T d = x - x0;
        T s = Y * d - d * (dth + (T)0.5 * d) * inv_s2;
#pragma unroll
        for (int k = 0; k < kMaxVals; ++k) {
            if (k < nv) {
                em1[k] = dexpm1(vk[k] * d);
                s -= Gk[k] * em1[k];
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

__device__ inline void raise_flag(int *err, int bit)
{
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Gene kernel
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void gene_sweep(const SegInfo *__restrict__ segs,
                                                  const int2 *__restrict__ tiles, int ntiles,
                                                  SweepArgs a, int *err)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int tix = (int)blockIdx.x * 4 + wave;
    if (tix >= ntiles) return;
    const int2 tt = tiles[tix];
    const int sidx = __builtin_amdgcn_readfirstlane(tt.x);
    const int tile = __builtin_amdgcn_readfirstlane(tt.y);
    const SegInfo &S = segs[sidx];
    const HyperState &H = *S.hyp;
    const int64_t Gp = S.Gp;
    const int64_t g = (int64_t)tile * kTile + lane;
    const bool active = g < S.G;
    const int N = S.N, L = S.L, R = S.R;
    const uint32_t mm = (uint32_t)a.m;
    const uint32_t chain = (uint32_t)S.chain;
    const bool tuning = a.m <= a.burnin;
    const bool sampling = a.m > a.burnin;
    const double kmom = (double)(a.m - a.burnin);
    const bool dbg = a.dbg != 0;
    const bool tracing = a.trace_point >= 0;
    const int tslot = (tracing && active) ? S.trace_slot[g] : -1;
    float *trow = tracing ? S.trace + (int64_t)a.trace_point * S.trace_stride + 2 + 2 * L : nullptr;

    T *eps = (T *)S.eps;
    T *w_eps = (T *)S.w_eps;
    T *wa_eps = (T *)S.wa_eps;
    T *gamp = (T *)S.gam;
    T *betap = (T *)S.beta;
    T *w_beta = (T *)S.w_beta;
    T *wa_beta = (T *)S.wa_beta;

    // current beta_g and gamma_g
    T beta[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) beta[l] = (l < L && active) ? betap[(int64_t)l * Gp + g] : (T)0;
    T gam = active ? gamp[g] : (T)1;

    T A[kMaxRows], YR[kMaxRows];
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) { A[r] = (T)0; YR[r] = (T)0; }
    T S2 = (T)0;
    int bad = 0;

    // ---- Algorithm 1 step 1: eps_gn, n = 1..N ----
    const bool upd_eps = (a.mask >> 1) & 1u;
    const T inv_gam = (T)1 / gam;
    if (active) {
        for (int n = 0; n < N; ++n) {
            const int64_t idx = (int64_t)n * Gp + g;
            const int yv = S.y[idx];
            const T e0 = eps[idx];
            T xb = (T)0;
#pragma unroll
            for (int l = 0; l < kMaxL; ++l)
                if (l < L) xb += (T)S.X[n * kMaxL + l] * beta[l];
            const T hn = (T)S.h[n];
            T e1 = e0;
            if (upd_eps) {
                T w = w_eps[idx];
                EpsF<T> f{(T)yv, dexp(hn + e0 + xb), e0, inv_gam};
                DrawRec rec;
                e1 = slice_draw<T>(f, e0, w, S.key0, S.key1, draw_counter((uint32_t)g, 1, (uint32_t)n, mm, chain, 0),
                                   a.K, a.cap, rec);
                eps[idx] = e1;
                if (tuning) {
                    T wa = wa_eps[idx];
                    tune_width<T>(w, wa, e0, e1, a.m, a.burnin, a.tune_start);
                    w_eps[idx] = w;
                    wa_eps[idx] = wa;
                }
                bad |= rec.bad;
                if (dbg) S.dbg_eps[idx] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
            }
            if (sampling) {
                double2 mo = S.mom_eps[idx];
                welford(mo, (double)e1, kmom);
                S.mom_eps[idx] = mo;
            }
            S2 += e1 * e1;
            const T ehe = dexp(hn + e1);
            const int rr = S.row_of[n];
#pragma unroll
            for (int r = 0; r < kMaxRows; ++r)
                if (r == rr) { A[r] += ehe; YR[r] += (T)yv; }
        }
    }

    // ---- step 2: gamma_g ----
    double lg = 0.0, ig = 0.0;
    if (active) {
        if ((a.mask >> 2) & 1u) {
            const double alpha1 = 0.5 * H.nu + 0.5 * N + 1.0;
            const double scale = 0.5 * H.nu * H.tau + 0.5 * (double)S2;
            GamF<T> f{(T)alpha1, (T)scale, gam};
            T w = ((T *)S.w_gam)[g];
            DrawRec rec;
            const T g1 = slice_draw<T>(f, gam, w, S.key0, S.key1, draw_counter((uint32_t)g, 2, 0, mm, chain, 0),
                                       a.K, a.cap, rec);
            if (tuning) {
                T wa = ((T *)S.wa_gam)[g];
                tune_width<T>(w, wa, gam, g1, a.m, a.burnin, a.tune_start);
                ((T *)S.w_gam)[g] = w;
                ((T *)S.wa_gam)[g] = wa;
            }
            gam = g1;
            gamp[g] = g1;
            bad |= rec.bad;
            if (dbg) S.dbg_gam[g] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
        }
        if (sampling) {
            double2 mo = S.mom_gam[g];
            welford(mo, (double)gam, kmom);
            S.mom_gam[g] = mo;
        }
        lg = ::log((double)gam);
        ig = 1.0 / (double)gam;
        if (tslot >= 0) trow[(int64_t)tslot * (L + 1)] = (float)gam;
    }
    {
        const double s0 = wave_sum(lg), s1 = wave_sum(ig);
        if (lane == 0) {
            S.partials[(int64_t)tile * kMaxParts + 0] = s0;
            S.partials[(int64_t)tile * kMaxParts + 1] = s1;
        }
    }

    // ---- step 5: beta_gl, l = 1..L in order ----
    // C_r = sum over the samples of distinct row r of exp(h_n + eps_gn + X_r beta_g)
    T C[kMaxRows];
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
        T xr = (T)0;
#pragma unroll
        for (int l = 0; l < kMaxL; ++l)
            if (l < L) xr += (T)S.Xrow[r * kMaxL + l] * beta[l];
        C[r] = (r < R) ? A[r] * dexp(xr) : (T)0;
    }
    const bool upd_beta = (a.mask >> 5) & 1u;
    for (int l = 0; l < L; ++l) {
        const int64_t idx = (int64_t)l * Gp + g;
        T b0 = (T)0;
#pragma unroll
        for (int j = 0; j < kMaxL; ++j)
            if (j == l) b0 = beta[j];
        T b1 = b0;
        if (active && upd_beta) {
            BetaF<T> f;
            f.Y = (T)0;
#pragma unroll
            for (int r = 0; r < kMaxRows; ++r)
                if (r < R) f.Y += (T)S.Xrow[r * kMaxL + l] * YR[r];
            f.nv = S.nv[l];
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
            const double th = H.theta[l], s2 = H.sig2[l];
            f.x0 = b0;
            f.dth = (T)((double)b0 - th);
            f.inv_s2 = (T)(1.0 / s2);
            T w = w_beta[idx];
            DrawRec rec;
            b1 = slice_draw<T>(f, b0, w, S.key0, S.key1, draw_counter((uint32_t)g, 5, (uint32_t)l, mm, chain, 0),
                               a.K, a.cap, rec);
            if (tuning) {
                T wa = wa_beta[idx];
                tune_width<T>(w, wa, b0, b1, a.m, a.burnin, a.tune_start);
                w_beta[idx] = w;
                wa_beta[idx] = wa;
            }
            betap[idx] = b1;
            bad |= rec.bad;
            if (dbg) S.dbg_beta[idx] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
            // move the row sums to the new beta_gl: C_r *= exp(X_rl (b1 - b0))
            T fac[kMaxVals];
#pragma unroll
            for (int k = 0; k < kMaxVals; ++k) fac[k] = rec.bad ? (T)1 : (T)1 + f.em1[k];
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
        if (active && sampling) {
            double2 mo = S.mom_beta[idx];
            welford(mo, (double)b1, kmom);
            S.mom_beta[idx] = mo;
        }
        if (tslot >= 0) trow[(int64_t)tslot * (L + 1) + 1 + l] = (float)b1;
        const double dv = active ? (double)b1 - H.theta[l] : 0.0;
        const double s0 = wave_sum(dv), s1 = wave_sum(dv * dv);
        if (lane == 0) {
            S.partials[(int64_t)tile * kMaxParts + 2 + 2 * l] = s0;
            S.partials[(int64_t)tile * kMaxParts + 3 + 2 * l] = s1;
        }
    }
    if (bad) raise_flag(err, 2);
}

// ---------------------------------------------------------------------------
// Hyperparameter kernel: one 256-thread workgroup per segment
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hyper_sweep(const SegInfo *__restrict__ segs, SweepArgs a,
                                                   int *err)
{
    const SegInfo &S = segs[blockIdx.x];
    HyperState &H = *S.hyp;
    const int L = S.L;
    const int nparts = 2 + 2 * L;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    __shared__ double part[4][kMaxParts];

    // Fixed-order reduction: thread t sums tiles t, t + 256, ... in order, then a
    // butterfly inside each wavefront, then the four wavefronts in order.
    double acc[kMaxParts];
#pragma unroll
    for (int j = 0; j < kMaxParts; ++j) acc[j] = 0.0;
    for (int64_t t = tid; t < S.ntiles; t += 256) {
#pragma unroll
        for (int j = 0; j < kMaxParts; ++j)
            if (j < nparts) acc[j] += S.partials[t * kMaxParts + j];
    }
#pragma unroll
    for (int j = 0; j < kMaxParts; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) part[wave][j] = v;
    }
    __syncthreads();
    if (tid != 0) return;

    double red[kMaxParts];
    for (int j = 0; j < nparts; ++j) red[j] = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];

    const double G = (double)S.G;
    const uint32_t mm = (uint32_t)a.m;
    const uint32_t chain = (uint32_t)S.chain;
    const bool tuning = a.m <= a.burnin;
    const bool sampling = a.m > a.burnin;
    const double kmom = (double)(a.m - a.burnin);
    int bad = 0;
    DrawRec rec;

    // step 3: nu
    if ((a.mask >> 3) & 1u) {
        NuF f{G, H.tau, red[0], red[1], S.d};
        const double x0 = H.nu;
        const double x1 = slice_draw<double>(f, x0, H.w_nu, S.key0, S.key1, draw_counter(0, 3, 0, mm, chain, 0),
                                             a.K, a.cap, rec);
        tune_width<double>(H.w_nu, H.wa_nu, x0, x1, a.m, a.burnin, a.tune_start);
        H.nu = x1;
        bad |= rec.bad;
        if (a.dbg) H.dbg[0] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
    }
    // step 4: tau
    if ((a.mask >> 4) & 1u) {
        TauF f{S.a + 0.5 * G * H.nu - 1.0, S.b + 0.5 * H.nu * red[1]};
        const double x0 = H.tau;
        const double x1 = slice_draw<double>(f, x0, H.w_tau, S.key0, S.key1, draw_counter(0, 4, 0, mm, chain, 0),
                                             a.K, a.cap, rec);
        tune_width<double>(H.w_tau, H.wa_tau, x0, x1, a.m, a.burnin, a.tune_start);
        H.tau = x1;
        bad |= rec.bad;
        if (a.dbg) H.dbg[1] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
    }
    // steps 6 and 7: theta_l then sigma_l^2.  The partials are sums of
    // (beta - s) and (beta - s)^2 with the shift s = theta_l before this step.
    for (int l = 0; l < L; ++l) {
        const double s = H.theta[l];
        const double d1 = red[2 + 2 * l], d2 = red[3 + 2 * l];
        const double sb = d1 + G * s;
        if ((a.mask >> 6) & 1u) {
            const double prec = G / H.sig2[l] + 1.0 / (S.c[l] * S.c[l]);
            const double mean = (sb / H.sig2[l]) / prec;
            const uint4 r = philox4x32_10(draw_counter(0, 6, (uint32_t)l, mm, chain, 0), S.key0, S.key1);
            const double zn = ::sqrt(-2.0 * ::log(u01<double>(r.x))) *
                              ::cos(6.283185307179586 * u01<double>(r.y));
            H.theta[l] = mean + zn / ::sqrt(prec);
        }
        const double dt = H.theta[l] - s;
        const double Ssq = d2 - 2.0 * dt * d1 + G * dt * dt;
        red[2 + 2 * l] = sb;
        red[3 + 2 * l] = Ssq;
        if ((a.mask >> 7) & 1u) {
            Sig2F f{0.5 * (G + 1.0), Ssq, S.s[l] * S.s[l]};
            const double x0 = H.sig2[l];
            const double x1 = slice_draw<double>(f, x0, H.w_sig2[l], S.key0, S.key1,
                                                 draw_counter(0, 7, (uint32_t)l, mm, chain, 0), a.K, a.cap, rec);
            tune_width<double>(H.w_sig2[l], H.wa_sig2[l], x0, x1, a.m, a.burnin, a.tune_start);
            H.sig2[l] = x1;
            bad |= rec.bad;
            if (a.dbg) H.dbg[2 + l] = make_int4(rec.kl, rec.nl, rec.nr, rec.nc);
        }
    }
    for (int j = 0; j < nparts; ++j) H.red[j] = red[j];
    if (sampling) {
        welford(H.mom[0], H.nu, kmom);
        welford(H.mom[1], H.tau, kmom);
        for (int l = 0; l < L; ++l) {
            welford(H.mom[2 + l], H.theta[l], kmom);
            welford(H.mom[2 + L + l], H.sig2[l], kmom);
        }
    }
    if (a.trace_point >= 0) {
        float *row = S.trace + (int64_t)a.trace_point * S.trace_stride;
        row[0] = (float)H.nu;
        row[1] = (float)H.tau;
        for (int l = 0; l < L; ++l) {
            row[2 + l] = (float)H.theta[l];
            row[2 + L + l] = (float)H.sig2[l];
        }
    }
    if (bad) raise_flag(err, 2);
    (void)tuning;
}

__global__ void philox_kernel(const uint4 *ctr, const uint2 *key, uint4 *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], key[i].x, key[i].y);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_gene(int precision, const SegInfo *segs, const int2 *tiles, int ntiles,
                       const SweepArgs &a, int *err, hipStream_t st)
{
    const int blocks = (ntiles + 3) / 4;
    if (blocks == 0) return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL(gene_sweep<double>, dim3(blocks), dim3(256), 0, st, segs, tiles, ntiles, a, err);
    else
        hipLaunchKernelGGL(gene_sweep<float>, dim3(blocks), dim3(256), 0, st, segs, tiles, ntiles, a, err);
    return hipGetLastError();
}

hipError_t launch_hyper(const SegInfo *segs, int nseg, const SweepArgs &a, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(hyper_sweep, dim3(nseg), dim3(256), 0, st, segs, a, err);
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
