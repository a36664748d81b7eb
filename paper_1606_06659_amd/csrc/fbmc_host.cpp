// fbmc_host.cpp -- host runtime behind the libfbmc C ABI (include/libfbmc.h).
//
// Owns the device buffers of every segment (one dataset x one chain), validates
// and analyses the design matrix, computes starting values, launches the two
// sweep kernels per sweep on the context's stream, and copies state, moments,
// traces and per-draw records back on request.
#include "libfbmc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fbmc_device.hpp"
#include "fbmc_mlp.hpp"
#include "fbmc_types.hpp"

namespace fbmc {
hipError_t launch_eps(int precision, const SegInfo *segs, const int4 *items, int nitems, const SweepArgs &a,
                      int nhyp_seg, int hsplit, const SweepArgs &ha, int *err, hipStream_t st);
hipError_t launch_gb(int precision, int mode, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                     const int4 *fb_items, int nfb, const SweepArgs &a, const MlpDev *net, int *err, hipStream_t st);
hipError_t launch_hyper(const SegInfo *segs, int nseg, int hsplit, const SweepArgs &a, int *err, hipStream_t st);
hipError_t launch_top(const SegInfo *segs, int nseg, int chains, TopState *top, const TopPriors &P,
                      const SweepArgs &a, hipStream_t st);
hipError_t launch_shift(int precision, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                        const SweepArgs &a, hipStream_t st);
hipError_t launch_gb_shift(int precision, int mode, int maxL, const SegInfo *segs, const int2 *tiles, int ntiles,
                           const SweepArgs &a, const MlpDev *net, int *err, hipStream_t st);
hipError_t launch_gb_pair(int precision, int maxL, bool shift, const SegInfo *segs, const int2 *tiles, int ntiles,
                          const SweepArgs &a, int *err, hipStream_t st);
hipError_t launch_mlp_sweep(int precision, const SegInfo *segs, const int2 *tiles, int ntiles, const MlpDev *net,
                            hipStream_t st);
hipError_t launch_philox(const uint4 *ctr, const uint2 *key, uint4 *out, int64_t n, hipStream_t st);
hipError_t launch_tile(int precision, int maxL, int maxN, const SegInfo *segs, const int2 *tiles, int ntiles,
                       const SweepArgs &a, int nhyp_seg, int hsplit, const SweepArgs &ha, int *err, hipStream_t st);
hipError_t launch_mlp_infer_raw(const float *phi, int64_t B, int L, const MlpDev *net, float *mu, float *ls,
                                float *off, hipStream_t st);
hipError_t launch_features(int precision, const SegInfo *seg, int64_t G, float *out, hipStream_t st);
hipError_t launch_gather_pairs(const float *pairs, int64_t P, int L, const float *master, float *X, float *Tg,
                               int B, uint32_t epoch, uint32_t step, uint32_t k0, uint32_t k1, hipStream_t st);
hipError_t launch_col_moments(const float *M, int64_t rows, int cols, double *work, double *out, hipStream_t st);
}  // namespace fbmc

using namespace fbmc;

namespace {

thread_local std::string g_thread_err;
constexpr int kErrWordsHost = 8;   // the kernels' error record (kErrWords)

struct Design {
    int R = 0;
    std::vector<int> row_of;            // [N]
    std::vector<double> Xrow;           // [R][L]
    std::vector<int> nv;                // [L]
    std::vector<double> vals;           // [L][kMaxVals]
    std::vector<int> xidx;              // [R][L]
};

struct DatasetH {
    int64_t G = 0, Gp = 0;
    int N = 0, L = 0;
    std::vector<int32_t> y;   // [G][N]
    std::vector<double> X, h, c, s;
    double a = 1, b = 1, d = 1000;
    uint64_t seed = 0;
    Design des;
    int32_t *d_y = nullptr;   // [N][Gp]
};

struct SegmentH {
    int dataset = 0, chain = 0;
    int64_t G = 0, Gp = 0, ntiles = 0;
    int N = 0, L = 0;
    SegInfo info{};
    HyperState *d_hyp = nullptr;
    std::vector<int64_t> trace_genes;
};

}  // namespace

struct fb_ctx {
    fb_options opt{};
    int prec = 0;
    size_t esz = 8;
    std::vector<DatasetH> ds;
    std::vector<SegmentH> seg;
    SegInfo *d_segs = nullptr;
    int2 *d_tiles = nullptr;
    int ntiles = 0;
    int maxL = 0;                     // largest L over the segments (picks the compiled bound)
    int maxN = 0;                     // largest N over the segments (LDS of the single-launch sweep)
    // the slice sweep (one beta lane, no shift step, no learned step) as one
    // launch per sweep (sweep_tile) instead of the eps and gamma/beta kernels
    bool tile = false;
    // eps work items (segment, tile, n0, n1): samples per wavefront `spw`
    int4 *d_items = nullptr;
    int nitems = 0, item_cap = 0, spw = 0;
    // the hyperparameter step rides in the next sweep's eps kernel (true) or
    // is a kernel of its own after the gamma/beta kernel (false)
    bool fuse = true;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int *d_err = nullptr;
    int sticky = FB_OK;
    int64_t m = 0;
    int64_t trace_n = 0, trace_dropped = 0;
    int trace_stride_max = 0;
    std::string err;
    std::vector<void *> allocs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t last_n = 0;
    // sampled per-kernel timing: events around the gene and hyper launches of
    // every `prof_every`-th sweep
    int32_t prof_every = 0, prof_cap = 0, prof_n = 0;
    int64_t prof_count = 0;
    std::vector<hipEvent_t> prof_ev;   // 8 per sample: eps, gamma/beta, hyperparameter, shift kernel
    std::vector<char> prof_hyp;        // sample has a separate hyperparameter kernel
    std::vector<char> prof_shift;      // sample has a shift kernel
    // learned beta proposal
    int beta_mode = FB_BETA_SLICE;
    bool learned_ready = false;
    // groups of up to 64 genes that keep the slice steps under the learned step:
    // (segment, first entry of the segment's list, count, partial column)
    int4 *d_fb_items = nullptr;
    int nfb_items = 0, fb_item_cap = 0;
    float *d_master = nullptr;        // kMlpParams FP32
    MlpDev *d_net = nullptr;          // packed inference copy
    MlpDev *d_idnet = nullptr;        // output map of the Laplace-only proposal: omean 0, oscale 1
    bool net_ready = false;
    float *d_pairs = nullptr;
    int64_t pair_cap = 0, pair_n = 0, totalG = 0;
    // graph replay (fb_set_graph): chunks of graph_k sweeps read their
    // arguments from d_args, filled from one of two pinned host buffers
    int64_t graph_k = 0, graph_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gsig;
    SweepArgs *d_args = nullptr;
    SweepArgs *h_args[2] = {nullptr, nullptr};
    hipEvent_t gcopied[2] = {nullptr, nullptr};
    int gslot = 0;
    // the slice sweep with the shift step runs gamma, beta and the shift in
    // one kernel (true) or the shift in a kernel of its own (false)
    bool fuse_shift = true;
    // lanes per gene in the slice sweep's beta draws (1: gb_sweep, 2: gb_pair_sweep)
    int beta_lanes = 1;
    bool hyper_split = true;          // one workgroup per chain of hyperparameter draws
    // three-level form (fb_set_top_level): one TopState per chain
    bool top_on = false;
    TopState *d_top = nullptr;
    TopPriors top_pri{};
};

namespace {

int fail(fb_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_thread_err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), FB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device memory from the context's allocator (fb_options.dev_alloc) or hipMalloc.
static int dmem(fb_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (c->opt.dev_alloc) {
        *p = c->opt.dev_alloc(bytes, c->opt.alloc_user);
        if (!*p) return fail(c, FB_ENOMEM, "dev_alloc returned NULL");
        if (reinterpret_cast<uintptr_t>(*p) % 256 != 0) {
            c->opt.dev_free(*p, c->opt.alloc_user);
            *p = nullptr;
            return fail(c, FB_EINVAL, "dev_alloc returned memory that is not 256-byte aligned");
        }
        // a caching allocator may hand out a block whose previous user's work
        // is still queued on another stream: let it finish before this
        // context's stream (or a synchronous copy) touches the block
        // (allocations are rare: context set-up, autotuning, training)
        const hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            c->opt.dev_free(*p, c->opt.alloc_user);
            *p = nullptr;
            return fail(c, FB_EDEVICE, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
        }
        return FB_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, FB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return FB_OK;
}

static void dfree(fb_ctx *c, void *p)
{
    if (!p) return;
    if (c->opt.dev_free) c->opt.dev_free(p, c->opt.alloc_user);
    else (void)hipFree(p);
}

int dalloc(fb_ctx *c, void **p, size_t bytes)
{
    int rc = dmem(c, p, bytes);
    if (rc) return rc;
    if (bytes == 0) bytes = 256;
    c->allocs.push_back(*p);
    hipError_t e;
    e = hipMemset(*p, 0, bytes);
    if (e != hipSuccess) return fail(c, FB_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
    return FB_OK;
}

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Distinct rows of X and, per column, the distinct non-zero values.
int analyse_design(const std::vector<double> &X, int N, int L, Design &D, std::string &msg)
{
    D.row_of.assign(N, -1);
    D.Xrow.clear();
    for (int n = 0; n < N; ++n) {
        int found = -1;
        for (int r = 0; r < (int)(D.Xrow.size() / L); ++r) {
            bool same = true;
            for (int l = 0; l < L; ++l)
                if (D.Xrow[r * L + l] != X[n * L + l]) { same = false; break; }
            if (same) { found = r; break; }
        }
        if (found < 0) {
            found = (int)(D.Xrow.size() / L);
            for (int l = 0; l < L; ++l) D.Xrow.push_back(X[n * L + l]);
        }
        D.row_of[n] = found;
    }
    D.R = (int)(D.Xrow.size() / L);
    if (D.R > kMaxRows) {
        msg = "the design matrix has " + std::to_string(D.R) + " distinct rows; at most " +
              std::to_string(kMaxRows) + " are supported";
        return FB_EINVAL;
    }
    D.nv.assign(L, 0);
    D.vals.assign((size_t)L * kMaxVals, 0.0);
    D.xidx.assign((size_t)D.R * L, -1);
    for (int l = 0; l < L; ++l) {
        for (int r = 0; r < D.R; ++r) {
            const double v = D.Xrow[r * L + l];
            if (v == 0.0) continue;
            int k = -1;
            for (int j = 0; j < D.nv[l]; ++j)
                if (D.vals[l * kMaxVals + j] == v) { k = j; break; }
            if (k < 0) {
                if (D.nv[l] == kMaxVals) {
                    msg = "column " + std::to_string(l) + " of X has more than " +
                          std::to_string(kMaxVals) + " distinct non-zero values";
                    return FB_EINVAL;
                }
                k = D.nv[l]++;
                D.vals[l * kMaxVals + k] = v;
            }
            D.xidx[r * L + l] = k;
        }
    }
    return FB_OK;
}

// Solve the symmetric positive definite system A x = b (Cholesky), n <= kMaxL.
bool chol_solve(std::vector<double> A, std::vector<double> &b, int n)
{
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0)) return false;
        const double dj = std::sqrt(s);
        A[j * n + j] = dj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / dj;
        }
    }
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[i * n + k] * b[k];
        b[i] = t / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * b[k];
        b[i] = t / A[i * n + i];
    }
    return true;
}

double std_normal(uint64_t seed, uint32_t g, uint32_t sub, uint32_t chain)
{
    const uint4 r = philox4x32_10(draw_counter(g, 9, sub, 0, chain, 0), (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u0 = ((double)r.x + 0.5) * 0x1p-32, u1 = ((double)r.y + 0.5) * 0x1p-32;
    return std::sqrt(-2.0 * std::log(u0)) * std::cos(6.283185307179586 * u1);
}

struct HostState {
    std::vector<double> eps, gam, beta;   // row-major [G][N], [G], [G][L]
    double nu = 10, tau = 0.1;
    std::vector<double> theta, sig2;
};

// Starting values: per-gene least squares of log(1 + y) - h on X.
void default_start(const DatasetH &D, int chain, bool jitter, HostState &S)
{
    const int64_t G = D.G;
    const int N = D.N, L = D.L;
    std::vector<double> XtX((size_t)L * L, 0.0);
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
            double s = (i == j) ? 1e-8 : 0.0;
            for (int n = 0; n < N; ++n) s += D.X[n * L + i] * D.X[n * L + j];
            XtX[i * L + j] = s;
        }
    S.eps.assign((size_t)G * N, 0.0);
    S.gam.assign(G, 0.1);
    S.beta.assign((size_t)G * L, 0.0);
    std::vector<double> rhs(L), z(N);
    for (int64_t g = 0; g < G; ++g) {
        for (int n = 0; n < N; ++n) z[n] = std::log1p((double)D.y[g * N + n]) - D.h[n];
        for (int l = 0; l < L; ++l) {
            double s = 0;
            for (int n = 0; n < N; ++n) s += D.X[n * L + l] * z[n];
            rhs[l] = s;
        }
        if (!chol_solve(XtX, rhs, L)) std::fill(rhs.begin(), rhs.end(), 0.0);
        double rss = 0;
        for (int n = 0; n < N; ++n) {
            double e = z[n];
            for (int l = 0; l < L; ++l) e -= D.X[n * L + l] * rhs[l];
            rss += e * e;
        }
        S.gam[g] = std::max(N > L ? rss / (N - L) : 0.1, 0.01);
        for (int l = 0; l < L; ++l) S.beta[g * L + l] = rhs[l];
    }
    std::vector<double> mean(L, 0.0), var(L, 0.0);
    for (int64_t g = 0; g < G; ++g)
        for (int l = 0; l < L; ++l) mean[l] += S.beta[g * L + l];
    for (int l = 0; l < L; ++l) mean[l] /= (double)G;
    for (int64_t g = 0; g < G; ++g)
        for (int l = 0; l < L; ++l) {
            const double dv = S.beta[g * L + l] - mean[l];
            var[l] += dv * dv;
        }
    for (int l = 0; l < L; ++l) var[l] = G > 1 ? var[l] / (double)(G - 1) : 1.0;
    if (jitter && chain > 0) {
        // overdispersed start: shift every beta by one across-gene sd, scale gamma
        for (int64_t g = 0; g < G; ++g) {
            for (int l = 0; l < L; ++l)
                S.beta[g * L + l] += std::sqrt(var[l]) * std_normal(D.seed, (uint32_t)g, (uint32_t)l, chain);
            S.gam[g] *= std::exp(0.5 * std_normal(D.seed, (uint32_t)g, 100, chain));
        }
    }
    S.theta.assign(L, 0.0);
    S.sig2.assign(L, 0.0);
    for (int64_t g = 0; g < G; ++g)
        for (int l = 0; l < L; ++l) S.theta[l] += S.beta[g * L + l];
    for (int l = 0; l < L; ++l) S.theta[l] /= (double)G;
    for (int64_t g = 0; g < G; ++g)
        for (int l = 0; l < L; ++l) {
            const double dv = S.beta[g * L + l] - S.theta[l];
            S.sig2[l] += dv * dv;
        }
    for (int l = 0; l < L; ++l) {
        double v = S.sig2[l] / (double)G;
        v = std::max(v, 1e-4);
        v = std::min(v, 0.25 * D.s[l] * D.s[l]);
        S.sig2[l] = v;
    }
    double tm = 0;
    for (int64_t g = 0; g < G; ++g) tm += S.gam[g];
    S.tau = tm / (double)G;
    S.nu = std::min(10.0, 0.5 * D.d);
    if (jitter && chain > 0) S.nu *= std::exp(0.3 * std_normal(D.seed, 0, 200, chain));
    S.nu = std::min(S.nu, 0.9 * D.d);
}

// Host row-major [G][K] doubles -> device [K][Gp] in the working precision.
void to_soa(const double *src, int64_t G, int K, int64_t Gp, int prec, std::vector<char> &buf,
            double pad)
{
    const size_t esz = prec == 0 ? 8 : 4;
    buf.assign((size_t)K * Gp * esz, 0);
    for (int k = 0; k < K; ++k)
        for (int64_t g = 0; g < Gp; ++g) {
            const double v = g < G ? src[g * K + k] : pad;
            if (prec == 0) reinterpret_cast<double *>(buf.data())[k * Gp + g] = v;
            else reinterpret_cast<float *>(buf.data())[k * Gp + g] = (float)v;
        }
}

void from_soa(const std::vector<char> &buf, int64_t G, int K, int64_t Gp, int prec, double *dst)
{
    for (int k = 0; k < K; ++k)
        for (int64_t g = 0; g < G; ++g)
            dst[g * K + k] = prec == 0 ? reinterpret_cast<const double *>(buf.data())[k * Gp + g]
                                       : (double)reinterpret_cast<const float *>(buf.data())[k * Gp + g];
}

int upload_array(fb_ctx *c, void *dst, const double *src, int64_t G, int K, int64_t Gp, double pad)
{
    std::vector<char> buf;
    to_soa(src, G, K, Gp, c->prec, buf, pad);
    HIPCHK(c, hipMemcpy(dst, buf.data(), buf.size(), hipMemcpyHostToDevice));
    return FB_OK;
}

int download_array(fb_ctx *c, const void *srcdev, int64_t G, int K, int64_t Gp, double *dst)
{
    std::vector<char> buf((size_t)K * Gp * c->esz);
    HIPCHK(c, hipMemcpy(buf.data(), srcdev, buf.size(), hipMemcpyDeviceToHost));
    from_soa(buf, G, K, Gp, c->prec, dst);
    return FB_OK;
}

int validate_options(const fb_options &o, std::string &msg)
{
    if (o.chains < 1 || o.chains > 65535) { msg = "chains must be in 1..65535"; return FB_EINVAL; }
    if (o.burnin < 0 || o.tune_start < 0 || o.tune_start > o.burnin) {
        msg = "need 0 <= tune_start <= burnin";
        return FB_EINVAL;
    }
    if (!(o.max_steps == 0 || o.max_steps == 1 || o.max_steps == 3 || o.max_steps == 7 || o.max_steps == 15)) {
        msg = "max_steps must be 0, 1, 3, 7 or 15";
        return FB_EINVAL;
    }
    if (!(o.w0 > 0) || !std::isfinite(o.w0)) { msg = "w0 must be a positive finite number"; return FB_EINVAL; }
    if (o.shrink_cap < 1) { msg = "shrink_cap must be >= 1"; return FB_EINVAL; }
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) {
        msg = "set both dev_alloc and dev_free, or neither";
        return FB_EINVAL;
    }
    if (o.precision != FB_FP64 && o.precision != FB_FP32) { msg = "unknown precision"; return FB_EINVAL; }
    if (o.thin < 0 || o.trace_genes < 0 || o.trace_capacity < 0) { msg = "negative trace option"; return FB_EINVAL; }
    return FB_OK;
}

int validate_dataset(const fb_dataset &d, std::string &msg)
{
    if (!d.counts || !d.X || !d.h) { msg = "counts, X and h must not be NULL"; return FB_EINVAL; }
    if (d.G < 1 || d.G > ((int64_t)1 << 31) - kTile) { msg = "G out of range"; return FB_EINVAL; }
    if (d.N < 1 || d.N > kMaxN) { msg = "N must be in 1.." + std::to_string(kMaxN); return FB_EINVAL; }
    if (d.L < 1 || d.L > kMaxL || d.L > d.N) { msg = "need 1 <= L <= min(N, " + std::to_string(kMaxL) + ")"; return FB_EINVAL; }
    for (int64_t i = 0; i < d.G * d.N; ++i)
        if (d.counts[i] < 0) { msg = "counts must be >= 0"; return FB_EINVAL; }
    if (!finite_all(d.X, (size_t)d.N * d.L) || !finite_all(d.h, d.N)) { msg = "X and h must be finite"; return FB_EINVAL; }
    if (d.priors) {
        const fb_priors &p = *d.priors;
        if (!(p.a > 0) || !(p.b > 0) || !(p.d > 0) || !std::isfinite(p.a) || !std::isfinite(p.b) || !std::isfinite(p.d)) {
            msg = "priors a, b, d must be positive and finite";
            return FB_EINVAL;
        }
        if (!p.c || !p.s) { msg = "priors c and s must not be NULL"; return FB_EINVAL; }
        for (int l = 0; l < d.L; ++l)
            if (!(p.c[l] > 0) || !(p.s[l] > 0) || !std::isfinite(p.c[l]) || !std::isfinite(p.s[l])) {
                msg = "priors c_l and s_l must be positive and finite";
                return FB_EINVAL;
            }
    }
    return FB_OK;
}

int write_state(fb_ctx *c, SegmentH &S, const HostState &hs)
{
    const DatasetH &D = c->ds[S.dataset];
    const int N = D.N, L = D.L;
    int rc;
    if ((rc = upload_array(c, S.info.eps, hs.eps.data(), S.G, N, S.Gp, 0.0))) return rc;
    if ((rc = upload_array(c, S.info.gam, hs.gam.data(), S.G, 1, S.Gp, 1.0))) return rc;
    if ((rc = upload_array(c, S.info.beta, hs.beta.data(), S.G, L, S.Gp, 0.0))) return rc;
    HyperState H{};
    HIPCHK(c, hipMemcpy(&H, S.d_hyp, sizeof(H), hipMemcpyDeviceToHost));
    H.nu = hs.nu;
    H.tau = hs.tau;
    for (int l = 0; l < L; ++l) { H.theta[l] = hs.theta[l]; H.sig2[l] = hs.sig2[l]; }
    HIPCHK(c, hipMemcpy(S.d_hyp, &H, sizeof(H), hipMemcpyHostToDevice));
    return FB_OK;
}

int build_items(fb_ctx *c, int spw);

int build_context(fb_ctx *c, const fb_dataset *dsv, int nds)
{
    int rc;
    std::string msg;
    c->prec = c->opt.precision;
    c->esz = c->prec == 0 ? 8 : 4;
    // datasets
    c->ds.resize(nds);
    for (int k = 0; k < nds; ++k) {
        const fb_dataset &in = dsv[k];
        DatasetH &D = c->ds[k];
        D.G = in.G;
        D.N = in.N;
        D.L = in.L;
        D.Gp = (in.G + kTile - 1) / kTile * kTile;
        D.y.assign(in.counts, in.counts + in.G * in.N);
        D.X.assign(in.X, in.X + in.N * in.L);
        D.h.assign(in.h, in.h + in.N);
        D.a = in.priors ? in.priors->a : 1.0;
        D.b = in.priors ? in.priors->b : 1.0;
        D.d = in.priors ? in.priors->d : 1000.0;
        D.c.assign(in.L, 10.0);
        D.s.assign(in.L, 100.0);
        if (in.priors)
            for (int l = 0; l < in.L; ++l) { D.c[l] = in.priors->c[l]; D.s[l] = in.priors->s[l]; }
        D.seed = in.seed;
        if ((rc = analyse_design(D.X, D.N, D.L, D.des, msg))) return fail(c, rc, msg);
        // counts, gene-contiguous
        std::vector<int32_t> yt((size_t)D.N * D.Gp, 0);
        for (int64_t g = 0; g < D.G; ++g)
            for (int n = 0; n < D.N; ++n) yt[(size_t)n * D.Gp + g] = D.y[g * D.N + n];
        if ((rc = dalloc(c, (void **)&D.d_y, yt.size() * sizeof(int32_t)))) return rc;
        HIPCHK(c, hipMemcpy(D.d_y, yt.data(), yt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    // segments
    const int C = c->opt.chains;
    c->seg.resize((size_t)nds * C);
    std::vector<int2> tiles;
    for (int k = 0; k < nds; ++k) {
        const DatasetH &D = c->ds[k];
        for (int ch = 0; ch < C; ++ch) {
            SegmentH &S = c->seg[(size_t)k * C + ch];
            S.dataset = k;
            S.chain = ch;
            S.G = D.G;
            S.Gp = D.Gp;
            S.ntiles = D.Gp / kTile;
            S.N = D.N;
            S.L = D.L;
            SegInfo &I = S.info;
            I.G = D.G; I.Gp = D.Gp; I.ntiles = S.ntiles;
            I.N = D.N; I.L = D.L; I.R = D.des.R;
            I.chain = ch;
            I.key0 = (uint32_t)D.seed;
            I.key1 = (uint32_t)(D.seed >> 32);
            I.dataset = k;
            for (int n = 0; n < D.N; ++n) {
                for (int l = 0; l < D.L; ++l) I.X[n * kMaxL + l] = D.X[n * D.L + l];
                I.h[n] = D.h[n];
                I.eh[n] = std::exp(D.h[n]);
                I.row_of[n] = D.des.row_of[n];
            }
            for (int i = 0; i < D.L; ++i)
                for (int j = 0; j < D.L; ++j) {
                    double x = 0.0;
                    for (int n = 0; n < D.N; ++n) x += D.X[n * D.L + i] * D.X[n * D.L + j];
                    I.XtX[i * kMaxL + j] = x;
                }
            for (int r = 0; r < D.des.R; ++r)
                for (int l = 0; l < D.L; ++l) {
                    I.Xrow[r * kMaxL + l] = D.des.Xrow[r * D.L + l];
                    I.xidx[r * kMaxL + l] = D.des.xidx[r * D.L + l];
                }
            for (int l = 0; l < D.L; ++l) {
                I.nv[l] = D.des.nv[l];
                I.pm[l] = (D.des.nv[l] == 2 && D.des.vals[l * kMaxVals + 1] == -D.des.vals[l * kMaxVals]) ? 1 : 0;
                for (int j = 0; j < kMaxVals; ++j) I.vals[l * kMaxVals + j] = D.des.vals[l * kMaxVals + j];
                I.c[l] = D.c[l];
                I.s[l] = D.s[l];
            }
            I.a = D.a; I.b = D.b; I.d = D.d;
            I.y = D.d_y;
            const size_t e = c->esz, Gp = (size_t)D.Gp, N = D.N, L = D.L;
            void **arrs_nk[] = {&I.eps, &I.w_eps, &I.wa_eps};
            for (void **p : arrs_nk) if ((rc = dalloc(c, p, N * Gp * e))) return rc;
            void **arrs_1[] = {&I.gam, &I.w_gam, &I.wa_gam};
            for (void **p : arrs_1) if ((rc = dalloc(c, p, Gp * e))) return rc;
            void **arrs_l[] = {&I.beta, &I.w_beta, &I.wa_beta};
            for (void **p : arrs_l) if ((rc = dalloc(c, p, L * Gp * e))) return rc;
            if ((rc = dalloc(c, (void **)&I.mom_eps, N * Gp * sizeof(double2)))) return rc;
            if ((rc = dalloc(c, (void **)&I.mom_gam, Gp * sizeof(double2)))) return rc;
            if ((rc = dalloc(c, (void **)&I.mom_beta, L * Gp * sizeof(double2)))) return rc;
            // partial columns: one per tile, then up to one per 64 fallback genes
            I.pstride = 2 * S.ntiles;
            if ((rc = dalloc(c, (void **)&I.partials, (size_t)I.pstride * kMaxParts * sizeof(double)))) return rc;
            // Y_r = sum over the samples of distinct row r of y_gn (constant)
            if ((rc = dalloc(c, &I.YR, (size_t)D.des.R * Gp * e))) return rc;
            {
                const int R = D.des.R;
                std::vector<double> yr((size_t)D.G * R, 0.0);
                for (int64_t g = 0; g < D.G; ++g)
                    for (int n = 0; n < D.N; ++n) yr[(size_t)g * R + D.des.row_of[n]] += (double)D.y[g * D.N + n];
                if ((rc = upload_array(c, I.YR, yr.data(), D.G, R, D.Gp, 0.0))) return rc;
            }
            if ((rc = dalloc(c, (void **)&S.d_hyp, sizeof(HyperState)))) return rc;
            I.hyp = S.d_hyp;
            if ((rc = dalloc(c, (void **)&I.hyp_flag, kHypFlags * sizeof(int64_t)))) return rc;
            if (c->opt.debug_counts) {
                if ((rc = dalloc(c, (void **)&I.dbg_eps, N * Gp * sizeof(int4)))) return rc;
                if ((rc = dalloc(c, (void **)&I.dbg_gam, Gp * sizeof(int4)))) return rc;
                if ((rc = dalloc(c, (void **)&I.dbg_beta, L * Gp * sizeof(int4)))) return rc;
            }
            // trace
            const int64_t T = std::min<int64_t>(c->opt.trace_genes, D.G);
            S.trace_genes.clear();
            for (int64_t i = 0; i < T; ++i) S.trace_genes.push_back(i * D.G / T);
            I.trace_T = (int32_t)T;
            I.trace_stride = (int32_t)(2 + 2 * L + T * (L + 1));
            c->trace_stride_max = std::max(c->trace_stride_max, I.trace_stride);
            std::vector<int32_t> slot(Gp, -1);
            for (int64_t i = 0; i < T; ++i) slot[S.trace_genes[i]] = (int32_t)i;
            if ((rc = dalloc(c, (void **)&I.trace_slot, Gp * sizeof(int32_t)))) return rc;
            HIPCHK(c, hipMemcpy(I.trace_slot, slot.data(), Gp * sizeof(int32_t), hipMemcpyHostToDevice));
            if (c->opt.thin > 0 && c->opt.trace_capacity > 0) {
                if ((rc = dalloc(c, (void **)&I.trace, (size_t)c->opt.trace_capacity * I.trace_stride * sizeof(float))))
                    return rc;
            }
            // widths and hyperparameter widths
            std::vector<double> w0v((size_t)D.G * std::max(D.N, D.L), c->opt.w0);
            if ((rc = upload_array(c, I.w_eps, w0v.data(), D.G, D.N, D.Gp, 1.0))) return rc;
            if ((rc = upload_array(c, I.w_gam, w0v.data(), D.G, 1, D.Gp, 1.0))) return rc;
            if ((rc = upload_array(c, I.w_beta, w0v.data(), D.G, D.L, D.Gp, 1.0))) return rc;
            HyperState H{};
            H.w_nu = H.w_tau = c->opt.w0;
            for (int l = 0; l < kMaxL; ++l) H.w_sig2[l] = c->opt.w0;
            HIPCHK(c, hipMemcpy(S.d_hyp, &H, sizeof(H), hipMemcpyHostToDevice));
            HostState hs;
            default_start(D, ch, c->opt.jitter != 0, hs);
            if ((rc = write_state(c, S, hs))) return rc;
            for (int64_t t = 0; t < S.ntiles; ++t) tiles.push_back(make_int2((int)(k * C + ch), (int)t));
        }
    }
    c->ntiles = (int)tiles.size();
    c->maxL = 0;
    c->maxN = 0;
    for (const auto &S : c->seg) {
        c->maxL = std::max(c->maxL, S.L);
        c->maxN = std::max(c->maxN, S.N);
    }
    if ((rc = dalloc(c, (void **)&c->d_tiles, tiles.size() * sizeof(int2)))) return rc;
    HIPCHK(c, hipMemcpy(c->d_tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice));
    std::vector<SegInfo> infos;
    for (auto &S : c->seg) infos.push_back(S.info);
    if ((rc = dalloc(c, (void **)&c->d_segs, infos.size() * sizeof(SegInfo)))) return rc;
    HIPCHK(c, hipMemcpy(c->d_segs, infos.data(), infos.size() * sizeof(SegInfo), hipMemcpyHostToDevice));
    if ((rc = dalloc(c, (void **)&c->d_err, kErrWordsHost * sizeof(int)))) return rc;
    if (c->opt.stream) {
        c->st = (hipStream_t)c->opt.stream;
    } else {
        HIPCHK(c, hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
        c->own_stream = true;
    }
    HIPCHK(c, hipEventCreate(&c->ev0));
    HIPCHK(c, hipEventCreate(&c->ev1));
    return build_items(c, 1);
}

bool valid_seg(const fb_ctx *c, int32_t seg) { return c && seg >= 0 && seg < (int32_t)c->seg.size(); }

}  // namespace

namespace {

struct SweepMode {
    bool learned_kernel = false;  // beta wavefront with features (IMH, pairs, counts)
    bool learned = false;         // IMH where the fallback mask is 0
    bool count_imh = false;       // add accepted IMH steps to the counters
    bool no_trace = false;        // trial sweeps of the autotuner: no trace rows
    bool laplace = false;         // IMH with the Laplace base alone: no network kernel
    int32_t collect_every = 0;
    int64_t collect_slot = 0;
};

// Work items of the eps kernel: every (segment, tile) split into sample ranges
// of `spw` samples, tile-major so the wavefronts of one tile share a workgroup.
int build_items(fb_ctx *c, int spw)
{
    std::vector<int4> items;
    for (size_t k = 0; k < c->seg.size(); ++k) {
        const SegmentH &S = c->seg[k];
        for (int64_t t = 0; t < S.ntiles; ++t)
            for (int n0 = 0; n0 < S.N; n0 += spw)
                items.push_back(make_int4((int)k, (int)t, n0, std::min(S.N, n0 + spw)));
    }
    if ((int)items.size() > c->item_cap) {
        int rc;
        if ((rc = dalloc(c, (void **)&c->d_items, items.size() * sizeof(int4)))) return rc;
        c->item_cap = (int)items.size();
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpy(c->d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice));
    c->nitems = (int)items.size();
    c->spw = spw;
    return FB_OK;
}

// The arguments of the next sweep; advances the host-side counters (sweep
// index, trace rows, training-pair slots).
static SweepArgs next_args(fb_ctx *c, SweepMode &md, int64_t m)
{
    const fb_options &o = c->opt;
    SweepArgs a{};
    a.m = m;
    a.burnin = o.burnin;
    a.tune_start = o.tune_start;
    a.inv_k = a.m > o.burnin ? 1.0 / (double)(a.m - o.burnin) : 0.0;
    a.K = o.max_steps;
    a.cap = o.shrink_cap;
    a.mask = o.update_mask;
    a.dbg = o.debug_counts;
    a.trace_point = -1;
    a.learned = md.learned ? 1 : 0;
    a.count_imh = md.count_imh ? 1 : 0;
    a.laplace = md.laplace ? 1 : 0;
    a.pair_base = -1;
    a.dev = nullptr;
    a.idx = 0;
    if (md.collect_every > 0 && a.m % md.collect_every == 0 && (md.collect_slot + 1) * c->totalG <= c->pair_cap) {
        a.pair_base = md.collect_slot * c->totalG;
        ++md.collect_slot;
        c->pair_n = md.collect_slot * c->totalG;
    }
    if (!md.no_trace && o.thin > 0 && o.trace_capacity > 0 && a.m % o.thin == 0 &&
        (!o.trace_after_burnin || a.m > o.burnin)) {
        if (c->trace_n < o.trace_capacity) a.trace_point = (int32_t)c->trace_n++;
        else ++c->trace_dropped;
    }
    return a;
}

// The gamma/beta kernel's form: the learned kernel in its MH-only form when
// no training pairs are taken.
static int gb_mode_of(const SweepMode &md, const SweepArgs &a)
{
    return !md.learned_kernel ? 0 : (md.learned && a.pair_base < 0) ? 2 : 1;
}

// The sweep runs as one launch (sweep_tile) when asked for and when it is the
// plain slice sweep with one lane per gene for beta.
static bool tile_sweep(const fb_ctx *c, const SweepMode &md, const SweepArgs &a)
{
    return c->tile && gb_mode_of(md, a) == 0 && c->beta_lanes == 1 && !((a.mask >> kKindShift) & 1u);
}

// Enqueue the sweeps args[0..n).  One sweep m is two launches: the eps kernel
// of sweep m, which also runs the hyperparameter step of sweep m - 1 in its
// first workgroups, then the gamma/beta kernel of sweep m (with the learned
// proposal the network kernel before it, with the shift step the shift kernel
// after it).  The hyperparameter step of the last sweep runs on its own at the
// end, so the state is whole between calls.  Unfused (c->fuse false), every
// sweep ends with its own hyperparameter kernel.  With dev set, every kernel
// takes sweep i's arguments from dev[i] (graph capture); profiling events are
// recorded only without it.
// Workgroups per segment of the hyperparameter step: one per chain of draws
// (nu then tau; theta_l then sigma_l^2 for each l), or one.
static int hsplit(const fb_ctx *c) { return c->hyper_split ? 1 + c->maxL : 1; }

static int launch_sweeps(fb_ctx *c, const SweepArgs *args, int64_t n, const SweepMode &md, const SweepArgs *dev)
{
    const int nseg = (int)c->seg.size();
    SweepArgs prev{};
    bool pending = false;
    for (int64_t i = 0; i < n; ++i) {
        SweepArgs a = args[i];
        if (dev) {
            a.dev = dev;
            a.idx = i;
        }
        const bool prof = !dev && c->prof_every > 0 && c->prof_n < c->prof_cap &&
                          (c->prof_count++ % c->prof_every) == 0;
        const bool shift = (args[i].mask >> kKindShift) & 1u;
        const int gbm = gb_mode_of(md, args[i]);
        // gamma, beta and the shift in one kernel: the slice steps, or the MH-only
        // learned kernel when no gene falls back (every beta of a tile is then
        // drawn by the tile's own workgroup)
        const bool fused_shift =
            shift && c->fuse_shift && (gbm == 0 || (gbm == 2 && (!md.learned || c->nfb_items == 0)));
        const MlpDev *gnet = md.laplace ? c->d_idnet : c->d_net;
        hipEvent_t *pe = prof ? &c->prof_ev[8 * (size_t)c->prof_n] : nullptr;
        if (prof) {
            c->prof_hyp[c->prof_n] = c->fuse ? 0 : 1;
            c->prof_shift[c->prof_n++] = (shift && !fused_shift) ? 1 : 0;
        }
        if (pe) HIPCHK(c, hipEventRecord(pe[0], c->st));
        if (tile_sweep(c, md, args[i])) {
            // the whole sweep in one launch; its time is reported as the eps kernel's
            HIPCHK(c, launch_tile(c->prec, c->maxL, c->maxN, c->d_segs, c->d_tiles, c->ntiles, a, pending ? nseg : 0,
                                  hsplit(c), prev, c->d_err, c->st));
            if (pe) {
                HIPCHK(c, hipEventRecord(pe[1], c->st));
                HIPCHK(c, hipEventRecord(pe[2], c->st));
                HIPCHK(c, hipEventRecord(pe[3], c->st));
            }
        } else {
            HIPCHK(c, launch_eps(c->prec, c->d_segs, c->d_items, c->nitems, a, pending ? nseg : 0, hsplit(c), prev,
                                 c->d_err, c->st));
            if (pe) HIPCHK(c, hipEventRecord(pe[1], c->st));
            if (pe) HIPCHK(c, hipEventRecord(pe[2], c->st));
            if (md.learned && !md.laplace)
                HIPCHK(c, launch_mlp_sweep(c->prec, c->d_segs, c->d_tiles, c->ntiles, c->d_net, c->st));
            if (gbm == 0 && c->beta_lanes == 2 && (!shift || fused_shift))
                HIPCHK(c, launch_gb_pair(c->prec, c->maxL, shift, c->d_segs, c->d_tiles, c->ntiles, a, c->d_err,
                                         c->st));
            else if (fused_shift)
                HIPCHK(c, launch_gb_shift(c->prec, gbm, c->maxL, c->d_segs, c->d_tiles, c->ntiles, a, gnet, c->d_err,
                                          c->st));
            else
                HIPCHK(c, launch_gb(c->prec, gbm, c->maxL, c->d_segs, c->d_tiles, c->ntiles, c->d_fb_items,
                                    md.learned ? c->nfb_items : 0, a, gnet, c->d_err, c->st));
            if (pe) HIPCHK(c, hipEventRecord(pe[3], c->st));
            if (shift && !fused_shift) {
                if (pe) HIPCHK(c, hipEventRecord(pe[6], c->st));
                HIPCHK(c, launch_shift(c->prec, c->maxL, c->d_segs, c->d_tiles, c->ntiles, a, c->st));
                if (pe) HIPCHK(c, hipEventRecord(pe[7], c->st));
            }
        }
        // top level psi(m) from the groups' phi(m - 1), before the hyperparameter step of m
        if (c->top_on) HIPCHK(c, launch_top(c->d_segs, nseg, c->opt.chains, c->d_top, c->top_pri, a, c->st));
        if (c->fuse) {
            prev = a;
            pending = true;
        } else {
            if (pe) HIPCHK(c, hipEventRecord(pe[4], c->st));
            HIPCHK(c, launch_hyper(c->d_segs, nseg, hsplit(c), a, c->d_err, c->st));
            if (pe) HIPCHK(c, hipEventRecord(pe[5], c->st));
        }
    }
    if (pending) HIPCHK(c, launch_hyper(c->d_segs, nseg, hsplit(c), prev, c->d_err, c->st));
    return FB_OK;
}

// What a captured chunk's launches depend on besides the arguments in device
// memory: launch shape, buffers, sizes and each sweep's set of kernels.
static std::vector<int64_t> graph_signature(const fb_ctx *c, const SweepMode &md, const SweepArgs *args, int64_t n)
{
    std::vector<int64_t> sig = {n, c->prec, c->maxL, c->fuse ? 1 : 0, (int64_t)(uintptr_t)c->d_segs,
                                (int64_t)(uintptr_t)c->d_items, c->nitems, (int64_t)(uintptr_t)c->d_tiles,
                                c->ntiles, (int64_t)(uintptr_t)c->d_fb_items, md.learned ? c->nfb_items : 0,
                                (int64_t)(uintptr_t)c->d_net, (int64_t)(uintptr_t)c->d_err,
                                (int64_t)(uintptr_t)c->st, md.learned ? 1 : 0, md.laplace ? 1 : 0,
                                (int64_t)(uintptr_t)c->d_idnet, c->top_on ? 1 : 0,
                                (int64_t)(uintptr_t)c->d_top};
    sig.push_back(c->fuse_shift ? 1 : 0);
    sig.push_back(c->beta_lanes);
    sig.push_back(c->hyper_split ? 1 : 0);
    sig.push_back(c->tile ? 1 : 0);
    for (int64_t i = 0; i < n; ++i) {
        sig.push_back(gb_mode_of(md, args[i]));
        sig.push_back((args[i].mask >> kKindShift) & 1u);
    }
    return sig;
}

void drop_graph(fb_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gsig.clear();
}

// One chunk of graph_k sweeps: arguments to pinned memory, then to the device
// array the captured kernels read, then a replay of the chunk's graph
// (captured again only when its signature changes).
static int graph_chunk(fb_ctx *c, SweepMode &md)
{
    const int64_t K = c->graph_k;
    const int slot = c->gslot;
    c->gslot ^= 1;
    HIPCHK(c, hipEventSynchronize(c->gcopied[slot]));     // the slot's previous copy is done
    SweepArgs *h = c->h_args[slot];
    for (int64_t i = 0; i < K; ++i) h[i] = next_args(c, md, c->m + 1 + i);
    std::vector<int64_t> sig = graph_signature(c, md, h, K);
    if (!c->gexec || sig != c->gsig) {
        drop_graph(c);
        HIPCHK(c, hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
        int rc = launch_sweeps(c, h, K, md, c->d_args);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        HIPCHK(c, e);
        c->graph = g;
        HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        c->gsig = sig;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_args, h, K * sizeof(SweepArgs), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipEventRecord(c->gcopied[slot], c->st));
    HIPCHK(c, hipGraphLaunch(c->gexec, c->st));
    c->m += K;
    return FB_OK;
}

int run_sweeps(fb_ctx *c, int64_t n, SweepMode &md)
{
    HIPCHK(c, hipEventRecord(c->ev0, c->st));
    int64_t done = 0;
    // graph replay in chunks of graph_k sweeps; sampled profiling and a
    // remainder shorter than a chunk launch directly
    if (c->graph_k > 0 && c->prof_every == 0) {
        int rc;
        while (n - done >= c->graph_k) {
            if ((rc = graph_chunk(c, md))) return rc;
            done += c->graph_k;
        }
    }
    if (done < n) {
        std::vector<SweepArgs> args((size_t)(n - done));
        for (int64_t i = 0; i < n - done; ++i) args[(size_t)i] = next_args(c, md, c->m + 1 + i);
        int rc = launch_sweeps(c, args.data(), n - done, md, nullptr);
        if (rc) return rc;
        c->m += n - done;
    }
    HIPCHK(c, hipEventRecord(c->ev1, c->st));
    c->last_n = n;
    return FB_OK;
}

int upload_segs(fb_ctx *c)
{
    std::vector<SegInfo> infos;
    for (auto &S : c->seg) infos.push_back(S.info);
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpy(c->d_segs, infos.data(), infos.size() * sizeof(SegInfo), hipMemcpyHostToDevice));
    return FB_OK;
}

// Buffers of the learned beta step: per segment the fallback mask and the IMH
// records.
int ensure_learned(fb_ctx *c)
{
    if (c->learned_ready) return FB_OK;
    int rc;
    c->totalG = 0;
    for (auto &S : c->seg) {
        const size_t Gp = (size_t)S.Gp;
        SegInfo &I = S.info;
        if ((rc = dalloc(c, (void **)&I.fallback, Gp * sizeof(int32_t)))) return rc;
        if ((rc = dalloc(c, (void **)&I.imh_count, Gp * sizeof(int32_t)))) return rc;
        if ((rc = dalloc(c, (void **)&I.imh_last, Gp * sizeof(int32_t)))) return rc;
        if ((rc = dalloc(c, (void **)&I.imh_stat, Gp * sizeof(int2)))) return rc;
        if ((rc = dalloc(c, (void **)&I.fb_genes, Gp * sizeof(int32_t)))) return rc;
        if ((rc = dalloc(c, (void **)&I.mlp_out, Gp * (size_t)mlp_outputs(S.L) * sizeof(float)))) return rc;
        I.nfbw = 0;
        c->totalG += S.G;
    }
    if ((rc = upload_segs(c))) return rc;
    c->learned_ready = true;
    return FB_OK;
}

// The output map of the Laplace-only proposal: with no network outputs the
// independence proposal is the per-gene Laplace base itself (omean 0, oscale
// 1; the kernels read nothing else of it in that mode).
int ensure_idnet(fb_ctx *c)
{
    if (c->d_idnet) return FB_OK;
    int rc;
    if ((rc = dalloc(c, (void **)&c->d_idnet, sizeof(MlpDev)))) return rc;     // zero-filled
    float one[8];
    for (float &v : one) v = 1.0f;
    HIPCHK(c, hipMemcpy((char *)c->d_idnet + offsetof(MlpDev, oscale), one, sizeof(one), hipMemcpyHostToDevice));
    return FB_OK;
}

// The fallback lists from the device masks: per segment the flagged genes in
// ascending order, cut into groups of 64, each with its own partial column
// after the segment's tiles.
int build_fallback(fb_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::vector<int4> items;
    for (size_t k = 0; k < c->seg.size(); ++k) {
        SegmentH &S = c->seg[k];
        std::vector<int32_t> mask((size_t)S.Gp), list;
        HIPCHK(c, hipMemcpy(mask.data(), S.info.fallback, mask.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t g = 0; g < S.G; ++g)
            if (mask[g]) list.push_back((int32_t)g);
        if (!list.empty())
            HIPCHK(c, hipMemcpy((void *)S.info.fb_genes, list.data(), list.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice));
        const int n = (int)list.size();
        S.info.nfbw = (n + kTile - 1) / kTile;
        for (int i = 0; i < S.info.nfbw; ++i)
            items.push_back(make_int4((int)k, i * kTile, std::min(kTile, n - i * kTile), (int)(S.ntiles + i)));
    }
    if ((int)items.size() > c->fb_item_cap) {
        int rc;
        if ((rc = dalloc(c, (void **)&c->d_fb_items, items.size() * sizeof(int4)))) return rc;
        c->fb_item_cap = (int)items.size();
    }
    if (!items.empty())
        HIPCHK(c, hipMemcpy(c->d_fb_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice));
    c->nfb_items = (int)items.size();
    return upload_segs(c);
}

int ensure_net(fb_ctx *c)
{
    int rc;
    if (!c->d_master && (rc = dalloc(c, (void **)&c->d_master, kMlpParams * sizeof(float)))) return rc;
    if (!c->d_net && (rc = dalloc(c, (void **)&c->d_net, sizeof(MlpDev)))) return rc;
    return FB_OK;
}

int pack_net(fb_ctx *c, const float *d_master, MlpDev *d_net, hipStream_t st)
{
    const int total = std::max((kMlpH / 16) * (kMlpH / 32) * 64 * 8, kWtFrags * 64 * 8);
    hipLaunchKernelGGL(pack_mlp, dim3((total + 255) / 256), dim3(256), 0, st, d_master, d_net);
    HIPCHK(c, hipGetLastError());
    return FB_OK;
}

// Host fb_mlp <-> contiguous master block.
bool mlp_to_block(const fb_mlp *w, std::vector<float> &blk)
{
    if (!w || !w->fmean || !w->fscale || !w->W1 || !w->b1 || !w->W2 || !w->b2 || !w->W3 || !w->b3 ||
        !w->omean || !w->oscale)
        return false;
    blk.assign(kMlpParams, 0.0f);
    std::copy(w->fmean, w->fmean + kMlpF, blk.begin() + kOffFmean);
    std::copy(w->fscale, w->fscale + kMlpF, blk.begin() + kOffFscale);
    std::copy(w->W1, w->W1 + kMlpF * kMlpH, blk.begin() + kOffW1);
    std::copy(w->b1, w->b1 + kMlpH, blk.begin() + kOffB1);
    std::copy(w->W2, w->W2 + kMlpH * kMlpH, blk.begin() + kOffW2);
    std::copy(w->b2, w->b2 + kMlpH, blk.begin() + kOffB2);
    std::copy(w->W3, w->W3 + kMlpH * kMlpO, blk.begin() + kOffW3);
    std::copy(w->b3, w->b3 + kMlpO, blk.begin() + kOffB3);
    std::copy(w->omean, w->omean + 8, blk.begin() + kOffOmean);
    std::copy(w->oscale, w->oscale + 8, blk.begin() + kOffOscale);
    return true;
}

void block_to_mlp(const std::vector<float> &blk, fb_mlp *w)
{
    auto put = [&](float *dst, int off, int n) { if (dst) std::copy(blk.begin() + off, blk.begin() + off + n, dst); };
    put(w->fmean, kOffFmean, kMlpF);
    put(w->fscale, kOffFscale, kMlpF);
    put(w->W1, kOffW1, kMlpF * kMlpH);
    put(w->b1, kOffB1, kMlpH);
    put(w->W2, kOffW2, kMlpH * kMlpH);
    put(w->b2, kOffB2, kMlpH);
    put(w->W3, kOffW3, kMlpH * kMlpO);
    put(w->b3, kOffB3, kMlpO);
    put(w->omean, kOffOmean, 8);
    put(w->oscale, kOffOscale, 8);
}

// Device memory that one call allocates for its own use (dalloc after the
// scope opens) and gives back when the call returns, after the stream has
// finished with it.
struct TempScope {
    fb_ctx *c;
    size_t mark;
    explicit TempScope(fb_ctx *ctx) : c(ctx), mark(ctx->allocs.size()) {}
    ~TempScope()
    {
        if (c->allocs.size() <= mark) return;
        if (c->st) (void)hipStreamSynchronize(c->st);
        for (size_t i = mark; i < c->allocs.size(); ++i) dfree(c, c->allocs[i]);
        c->allocs.resize(mark);
    }
    TempScope(const TempScope &) = delete;
    TempScope &operator=(const TempScope &) = delete;
};

// Scratch of one forward/backward pass on B rows.
int alloc_train(fb_ctx *c, TrainBufs &t, int B, int L)
{
    int rc;
    const size_t b = (size_t)B;
    float **bufs[] = {&t.Z1, &t.H1, &t.Z2, &t.H2, &t.dH, &t.dZ2, &t.dZ1};
    for (float **p : bufs) if ((rc = dalloc(c, (void **)p, b * kMlpH * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&t.X, b * kMlpF * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&t.Tg, b * (size_t)std::max(L, 1) * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&t.O, b * kMlpO * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&t.dO, b * kMlpO * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&t.loss, b * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&t.grad, kMlpParams * sizeof(float)))) return rc;
    t.B = B;
    return FB_OK;
}

double std_normal_key(uint64_t seed, uint32_t i, uint32_t j)
{
    const uint4 r = philox4x32_10(make_uint4(i, j, 0xA11Cu, 0), (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u0 = ((double)r.x + 0.5) * 0x1p-32, u1 = ((double)r.y + 0.5) * 0x1p-32;
    return std::sqrt(-2.0 * std::log(u0)) * std::cos(6.283185307179586 * u1);
}

}  // namespace

namespace fbmc {
// The per-thread last error that fb_last_error(NULL) reports, for entry points
// in other source files.
void set_thread_error(const char *msg) { g_thread_err = msg; }
}  // namespace fbmc

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void fb_default_options(fb_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->chains = 1;
    o->burnin = 1000;
    o->tune_start = 100;
    o->max_steps = 15;
    o->w0 = 1.0;
    o->shrink_cap = 200;
    o->precision = FB_FP64;
    o->update_mask = FB_UPDATE_ALL;
    o->thin = 0;
    o->trace_genes = 0;
    o->trace_after_burnin = 1;
    o->trace_capacity = 0;
    o->debug_counts = 0;
    o->jitter = 1;
    o->stream = nullptr;
}

int fb_create_batch(fb_ctx **out, const fb_dataset *ds, int32_t n_datasets, const fb_options *opt)
{
    if (!out) return fail(nullptr, FB_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!ds || n_datasets < 1) return fail(nullptr, FB_EINVAL, "need at least one dataset");
    fb_options o;
    fb_default_options(&o);
    if (opt) o = *opt;
    std::string msg;
    int rc = validate_options(o, msg);
    if (rc) return fail(nullptr, rc, msg);
    for (int k = 0; k < n_datasets; ++k)
        if ((rc = validate_dataset(ds[k], msg))) return fail(nullptr, rc, "dataset " + std::to_string(k) + ": " + msg);
    fb_ctx *c = new (std::nothrow) fb_ctx();
    if (!c) return fail(nullptr, FB_ENOMEM, "out of host memory");
    c->opt = o;
    rc = build_context(c, ds, n_datasets);
    if (rc) {
        g_thread_err = c->err;
        fb_destroy(c);
        return rc;
    }
    *out = c;
    return FB_OK;
}

int fb_create(fb_ctx **out, const int32_t *counts, int64_t G, int32_t N, const double *X, int32_t L,
              const double *h, const fb_priors *pri, uint64_t seed, const fb_options *opt)
{
    fb_dataset d{counts, G, N, X, L, h, pri, seed};
    return fb_create_batch(out, &d, 1, opt);
}

void fb_destroy(fb_ctx *c)
{
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    drop_graph(c);
    for (int i = 0; i < 2; ++i) {
        if (c->h_args[i]) (void)hipHostFree(c->h_args[i]);
        if (c->gcopied[i]) (void)hipEventDestroy(c->gcopied[i]);
    }
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    for (void *p : c->allocs) dfree(c, p);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
    delete c;
}

int fb_sweep(fb_ctx *c, int64_t n)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (n < 0) return fail(c, FB_EINVAL, "n must be >= 0");
    if (c->sticky) return c->sticky;
    SweepMode md;
    md.learned = c->beta_mode == FB_BETA_LEARNED || c->beta_mode == FB_BETA_LAPLACE;
    md.learned_kernel = md.learned;
    md.laplace = c->beta_mode == FB_BETA_LAPLACE;
    return run_sweeps(c, n, md);
}

int fb_set_graph(fb_ctx *c, int32_t sweeps)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (sweeps < 0 || sweeps > 4096) return fail(c, FB_EINVAL, "sweeps per graph must be in 0..4096");
    HIPCHK(c, hipStreamSynchronize(c->st));
    drop_graph(c);
    if (sweeps > c->graph_cap) {
        int rc;
        if ((rc = dalloc(c, (void **)&c->d_args, (size_t)sweeps * sizeof(SweepArgs)))) return rc;
        for (int i = 0; i < 2; ++i) {
            if (c->h_args[i]) HIPCHK(c, hipHostFree(c->h_args[i]));
            c->h_args[i] = nullptr;
            HIPCHK(c, hipHostMalloc((void **)&c->h_args[i], (size_t)sweeps * sizeof(SweepArgs), hipHostMallocDefault));
            if (!c->gcopied[i]) HIPCHK(c, hipEventCreateWithFlags(&c->gcopied[i], hipEventDisableTiming));
        }
        c->graph_cap = sweeps;
    }
    c->graph_k = sweeps;
    return FB_OK;
}

int32_t fb_get_graph(const fb_ctx *c) { return c ? (int32_t)c->graph_k : 0; }

int fb_sync(fb_ctx *c)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    HIPCHK(c, hipStreamSynchronize(c->st));
    int e[kErrWordsHost] = {};
    HIPCHK(c, hipMemcpy(e, c->d_err, sizeof(e), hipMemcpyDeviceToHost));
    const int flag = e[0];
    if ((flag & 4) && !c->sticky) {
        c->sticky = FB_EDEVICE;
        c->err = "single-launch sweep: a wait for the hyperparameter step timed out";
    }
    if (flag && !c->sticky) {
        c->sticky = FB_ENUMERIC;
        c->err = "a slice draw reached the shrink cap or met a non-finite log density";
        if (e[1]) {
            static const char *kinds[] = {"?", "eps", "gamma", "hyperparameter", "tau", "beta"};
            const int k = e[2] >= 1 && e[2] <= 5 ? e[2] : 0;
            char buf[200];
            std::snprintf(buf, sizeof buf, " (first: %s draw, dataset %d, chain %d, gene %d, sweep %d, index %d)",
                          kinds[k], e[3], e[4], e[5], e[6], e[7]);
            c->err += buf;
        }
    }
    return c->sticky;
}

int32_t fb_num_segments(const fb_ctx *c) { return c ? (int32_t)c->seg.size() : 0; }

int fb_segment_dims(const fb_ctx *c, int32_t seg, int64_t *G, int32_t *N, int32_t *L, int32_t *dataset,
                    int32_t *chain)
{
    if (!valid_seg(c, seg)) return fail(const_cast<fb_ctx *>(c), FB_EINVAL, "bad segment");
    const SegmentH &S = c->seg[seg];
    if (G) *G = S.G;
    if (N) *N = S.N;
    if (L) *L = S.L;
    if (dataset) *dataset = S.dataset;
    if (chain) *chain = S.chain;
    return FB_OK;
}

int fb_get_state(fb_ctx *c, int32_t seg, fb_state *s)
{
    if (!valid_seg(c, seg) || !s) return fail(c, FB_EINVAL, "bad segment or NULL state");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    SegmentH &S = c->seg[seg];
    const int N = S.N, L = S.L;
    const SegInfo &I = S.info;
    struct { double *dst; const void *src; int K; } blocks[] = {
        {s->eps, I.eps, N}, {s->w_eps, I.w_eps, N}, {s->waux_eps, I.wa_eps, N},
        {s->gam, I.gam, 1}, {s->w_gam, I.w_gam, 1}, {s->waux_gam, I.wa_gam, 1},
        {s->beta, I.beta, L}, {s->w_beta, I.w_beta, L}, {s->waux_beta, I.wa_beta, L}};
    for (auto &b : blocks)
        if (b.dst && (rc = download_array(c, b.src, S.G, b.K, S.Gp, b.dst))) return rc;
    HyperState H;
    HIPCHK(c, hipMemcpy(&H, S.d_hyp, sizeof(H), hipMemcpyDeviceToHost));
    if (s->hyp) {
        s->hyp[0] = H.nu;
        s->hyp[1] = H.tau;
        for (int l = 0; l < L; ++l) { s->hyp[2 + l] = H.theta[l]; s->hyp[2 + L + l] = H.sig2[l]; }
    }
    if (s->w_hyp) {
        s->w_hyp[0] = H.w_nu; s->w_hyp[1] = H.w_tau;
        for (int l = 0; l < L; ++l) s->w_hyp[2 + l] = H.w_sig2[l];
    }
    if (s->waux_hyp) {
        s->waux_hyp[0] = H.wa_nu; s->waux_hyp[1] = H.wa_tau;
        for (int l = 0; l < L; ++l) s->waux_hyp[2 + l] = H.wa_sig2[l];
    }
    s->m = c->m;
    return c->sticky;
}

int fb_set_state(fb_ctx *c, int32_t seg, const fb_state *s)
{
    if (!valid_seg(c, seg) || !s) return fail(c, FB_EINVAL, "bad segment or NULL state");
    if (s->m < 0) return fail(c, FB_EINVAL, "m must be >= 0");
    SegmentH &S = c->seg[seg];
    const DatasetH &D = c->ds[S.dataset];
    const int N = S.N, L = S.L;
    const int64_t G = S.G;
    auto all_pos = [](const double *p, size_t n) {
        for (size_t i = 0; i < n; ++i) if (!(p[i] > 0) || !std::isfinite(p[i])) return false;
        return true;
    };
    if (s->eps && !finite_all(s->eps, (size_t)G * N)) return fail(c, FB_EINVAL, "eps must be finite");
    if (s->beta && !finite_all(s->beta, (size_t)G * L)) return fail(c, FB_EINVAL, "beta must be finite");
    if (s->gam && !all_pos(s->gam, G)) return fail(c, FB_EINVAL, "gamma must be > 0");
    if (s->w_eps && !all_pos(s->w_eps, (size_t)G * N)) return fail(c, FB_EINVAL, "widths must be > 0");
    if (s->w_gam && !all_pos(s->w_gam, G)) return fail(c, FB_EINVAL, "widths must be > 0");
    if (s->w_beta && !all_pos(s->w_beta, (size_t)G * L)) return fail(c, FB_EINVAL, "widths must be > 0");
    if (s->w_hyp && !all_pos(s->w_hyp, 2 + L)) return fail(c, FB_EINVAL, "widths must be > 0");
    if (s->waux_eps && !finite_all(s->waux_eps, (size_t)G * N)) return fail(c, FB_EINVAL, "waux must be finite");
    if (s->waux_gam && !finite_all(s->waux_gam, G)) return fail(c, FB_EINVAL, "waux must be finite");
    if (s->waux_beta && !finite_all(s->waux_beta, (size_t)G * L)) return fail(c, FB_EINVAL, "waux must be finite");
    if (s->waux_hyp && !finite_all(s->waux_hyp, 2 + L)) return fail(c, FB_EINVAL, "waux must be finite");
    if (s->hyp) {
        if (!finite_all(s->hyp, 2 + 2 * L)) return fail(c, FB_EINVAL, "hyperparameters must be finite");
        if (!(s->hyp[0] > 0 && s->hyp[0] < D.d)) return fail(c, FB_EINVAL, "need 0 < nu < d");
        if (!(s->hyp[1] > 0)) return fail(c, FB_EINVAL, "need tau > 0");
        for (int l = 0; l < L; ++l)
            if (!(s->hyp[2 + L + l] > 0 && s->hyp[2 + L + l] < D.s[l] * D.s[l]))
                return fail(c, FB_EINVAL, "need 0 < sigma^2_l < s_l^2");
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    const SegInfo &I = S.info;
    int rc;
    struct { const double *src; void *dst; int K; double pad; } blocks[] = {
        {s->eps, I.eps, N, 0.0}, {s->w_eps, I.w_eps, N, 1.0}, {s->waux_eps, I.wa_eps, N, 0.0},
        {s->gam, I.gam, 1, 1.0}, {s->w_gam, I.w_gam, 1, 1.0}, {s->waux_gam, I.wa_gam, 1, 0.0},
        {s->beta, I.beta, L, 0.0}, {s->w_beta, I.w_beta, L, 1.0}, {s->waux_beta, I.wa_beta, L, 0.0}};
    for (auto &b : blocks)
        if (b.src && (rc = upload_array(c, b.dst, b.src, G, b.K, S.Gp, b.pad))) return rc;
    HyperState H;
    HIPCHK(c, hipMemcpy(&H, S.d_hyp, sizeof(H), hipMemcpyDeviceToHost));
    if (s->hyp) {
        H.nu = s->hyp[0];
        H.tau = s->hyp[1];
        for (int l = 0; l < L; ++l) { H.theta[l] = s->hyp[2 + l]; H.sig2[l] = s->hyp[2 + L + l]; }
    }
    if (s->w_hyp) {
        H.w_nu = s->w_hyp[0]; H.w_tau = s->w_hyp[1];
        for (int l = 0; l < L; ++l) H.w_sig2[l] = s->w_hyp[2 + l];
    }
    if (s->waux_hyp) {
        H.wa_nu = s->waux_hyp[0]; H.wa_tau = s->waux_hyp[1];
        for (int l = 0; l < L; ++l) H.wa_sig2[l] = s->waux_hyp[2 + l];
    }
    HIPCHK(c, hipMemcpy(S.d_hyp, &H, sizeof(H), hipMemcpyHostToDevice));
    c->m = s->m;
    // the sweep index may go back: clear what the single-launch sweep waits on
    for (auto &Sg : c->seg) HIPCHK(c, hipMemset(Sg.info.hyp_flag, 0, kHypFlags * sizeof(int64_t)));
    // back in burn-in: the acceptance counts restart with the next sampling
    // sweep, as the running moments do
    if (c->m <= c->opt.burnin)
        for (auto &Sg : c->seg)
            if (Sg.info.imh_stat) HIPCHK(c, hipMemset(Sg.info.imh_stat, 0, (size_t)Sg.Gp * sizeof(int2)));
    return FB_OK;
}

int fb_summaries(fb_ctx *c, int32_t seg, fb_summary *s)
{
    if (!valid_seg(c, seg) || !s) return fail(c, FB_EINVAL, "bad segment or NULL summary");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    SegmentH &S = c->seg[seg];
    const int N = S.N, L = S.L;
    const int64_t G = S.G, Gp = S.Gp;
    auto get = [&](const double2 *src, int K, double *mean, double *msq) -> int {
        if (!mean && !msq) return FB_OK;
        std::vector<double2> buf((size_t)K * Gp);
        HIPCHK(c, hipMemcpy(buf.data(), src, buf.size() * sizeof(double2), hipMemcpyDeviceToHost));
        for (int k = 0; k < K; ++k)
            for (int64_t g = 0; g < G; ++g) {
                if (mean) mean[g * K + k] = buf[(size_t)k * Gp + g].x;
                if (msq) msq[g * K + k] = buf[(size_t)k * Gp + g].y;
            }
        return FB_OK;
    };
    if ((rc = get(S.info.mom_eps, N, s->mean_eps, s->msq_eps))) return rc;
    if ((rc = get(S.info.mom_gam, 1, s->mean_gam, s->msq_gam))) return rc;
    if ((rc = get(S.info.mom_beta, L, s->mean_beta, s->msq_beta))) return rc;
    HyperState H;
    HIPCHK(c, hipMemcpy(&H, S.d_hyp, sizeof(H), hipMemcpyDeviceToHost));
    for (int j = 0; j < 2 + 2 * L; ++j) {
        if (s->mean_hyp) s->mean_hyp[j] = H.mom[j].x;
        if (s->msq_hyp) s->msq_hyp[j] = H.mom[j].y;
    }
    if (s->imh_steps || s->imh_accepts) {
        std::vector<int2> st((size_t)G, make_int2(0, 0));
        if (S.info.imh_stat)
            HIPCHK(c, hipMemcpy(st.data(), S.info.imh_stat, st.size() * sizeof(int2), hipMemcpyDeviceToHost));
        for (int64_t g = 0; g < G; ++g) {
            if (s->imh_steps) s->imh_steps[g] = st[(size_t)g].x;
            if (s->imh_accepts) s->imh_accepts[g] = st[(size_t)g].y;
        }
    }
    s->count = c->m > c->opt.burnin ? c->m - c->opt.burnin : 0;
    return c->sticky;
}

int fb_trace_genes(const fb_ctx *c, int32_t seg, int64_t *genes, int32_t *T)
{
    if (!valid_seg(c, seg)) return fail(const_cast<fb_ctx *>(c), FB_EINVAL, "bad segment");
    const SegmentH &S = c->seg[seg];
    if (T) *T = (int32_t)S.trace_genes.size();
    if (genes) std::copy(S.trace_genes.begin(), S.trace_genes.end(), genes);
    return FB_OK;
}

int fb_trace(fb_ctx *c, int32_t seg, float *buf, int64_t cap, int64_t *n_out, int64_t *dropped)
{
    if (!valid_seg(c, seg) || cap < 0) return fail(c, FB_EINVAL, "bad segment or capacity");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    SegmentH &S = c->seg[seg];
    const int64_t n = std::min<int64_t>(c->trace_n, cap);
    if (n > 0 && buf) {
        if (!S.info.trace) return fail(c, FB_ESTATE, "tracing is off");
        HIPCHK(c, hipMemcpy(buf, S.info.trace, (size_t)n * S.info.trace_stride * sizeof(float),
                            hipMemcpyDeviceToHost));
    }
    if (n_out) *n_out = buf ? n : c->trace_n;
    if (dropped) *dropped = c->trace_dropped;
    return c->sticky;
}

int fb_trace_reset(fb_ctx *c)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->trace_n = 0;
    c->trace_dropped = 0;
    return FB_OK;
}

int fb_debug_counts(fb_ctx *c, int32_t seg, int32_t *eps, int32_t *gam, int32_t *beta, int32_t *hyp)
{
    if (!valid_seg(c, seg)) return fail(c, FB_EINVAL, "bad segment");
    if (!c->opt.debug_counts) return fail(c, FB_ESTATE, "debug_counts is off");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    SegmentH &S = c->seg[seg];
    const int N = S.N, L = S.L;
    const int64_t G = S.G, Gp = S.Gp;
    auto get = [&](const int4 *src, int K, int32_t *dst) -> int {
        if (!dst) return FB_OK;
        std::vector<int4> buf((size_t)K * Gp);
        HIPCHK(c, hipMemcpy(buf.data(), src, buf.size() * sizeof(int4), hipMemcpyDeviceToHost));
        for (int k = 0; k < K; ++k)
            for (int64_t g = 0; g < G; ++g) {
                const int4 v = buf[(size_t)k * Gp + g];
                int32_t *o = dst + 4 * (g * K + k);
                o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
            }
        return FB_OK;
    };
    if ((rc = get(S.info.dbg_eps, N, eps))) return rc;
    if ((rc = get(S.info.dbg_gam, 1, gam))) return rc;
    if ((rc = get(S.info.dbg_beta, L, beta))) return rc;
    if (hyp) {
        HyperState H;
        HIPCHK(c, hipMemcpy(&H, S.d_hyp, sizeof(H), hipMemcpyDeviceToHost));
        for (int j = 0; j < 2 + L; ++j) {
            hyp[4 * j] = H.dbg[j].x; hyp[4 * j + 1] = H.dbg[j].y;
            hyp[4 * j + 2] = H.dbg[j].z; hyp[4 * j + 3] = H.dbg[j].w;
        }
    }
    return c->sticky;
}

int fb_reductions(fb_ctx *c, int32_t seg, double *out)
{
    if (!valid_seg(c, seg) || !out) return fail(c, FB_EINVAL, "bad segment or NULL output");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    HyperState H;
    HIPCHK(c, hipMemcpy(&H, c->seg[seg].d_hyp, sizeof(H), hipMemcpyDeviceToHost));
    std::copy(H.red, H.red + 2 + 2 * c->seg[seg].L, out);
    return c->sticky;
}

int fb_set_contrasts(fb_ctx *c, int32_t n_events, int32_t n_rows, const int32_t *row_event, const double *v,
                     const double *b)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (n_events < 0 || n_events > kMaxEv || n_rows < n_events || n_rows > kMaxCtr ||
        (n_rows > 0 && (!row_event || !v || !b)))
        return fail(c, FB_EINVAL, "need 0 <= events <= 8, events <= rows <= 16 and the row arrays");
    const int L = c->seg.front().L;
    for (const auto &S : c->seg)
        if (S.L != L) return fail(c, FB_EINVAL, "contrasts need every dataset of the context to have the same L");
    for (int r = 0; r < n_rows; ++r) {
        if (row_event[r] < 0 || row_event[r] >= n_events) return fail(c, FB_EINVAL, "row_event out of range");
        for (int l = 0; l < L; ++l)
            if (!std::isfinite(v[r * L + l])) return fail(c, FB_EINVAL, "non-finite contrast");
        if (!std::isfinite(b[r])) return fail(c, FB_EINVAL, "non-finite bound");
    }
    for (int e = 0; e < n_events; ++e) {
        bool seen = false;
        for (int r = 0; r < n_rows; ++r) seen = seen || row_event[r] == e;
        if (!seen) return fail(c, FB_EINVAL, "every event needs at least one row");
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (auto &S : c->seg) {
        SegInfo &I = S.info;
        const size_t bytes = (size_t)kMaxEv * (size_t)S.Gp * sizeof(int32_t);
        int rc;
        if (!I.ev_count && (rc = dalloc(c, (void **)&I.ev_count, bytes))) return rc;
        HIPCHK(c, hipMemset(I.ev_count, 0, bytes));
        I.n_ev = n_events;
        I.n_crow = n_rows;
        I.ev_from = c->m;
        for (int r = 0; r < kMaxCtr; ++r) {
            I.crow_event[r] = r < n_rows ? row_event[r] : 0;
            I.cb[r] = r < n_rows ? b[r] : 0.0;
            for (int l = 0; l < kMaxL; ++l) I.cv[r * kMaxL + l] = (r < n_rows && l < L) ? v[r * L + l] : 0.0;
        }
    }
    return upload_segs(c);
}

int fb_set_top_level(fb_ctx *c, const fb_top_priors *p)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (c->m > c->opt.burnin) return fail(c, FB_EINVAL, "the top level is set before burn-in ends");
    drop_graph(c);
    if (!p) {
        c->top_on = false;
        for (auto &S : c->seg) S.info.top = nullptr;
        return upload_segs(c);
    }
    const int L = c->seg.front().L;
    for (const auto &S : c->seg)
        if (S.L != L) return fail(c, FB_EINVAL, "a top level needs every dataset of the context to have the same L");
    if (!(p->a_b > 0.0) || !(p->b_b > 0.0) || !p->c0 || (p->mask & ~3u))
        return fail(c, FB_EINVAL, "need a_b > 0, b_b > 0, c0[L] and mask bits 0..1");
    for (int l = 0; l < L; ++l)
        if (!(p->c0[l] > 0.0) || !std::isfinite(p->c0[l])) return fail(c, FB_EINVAL, "need 0 < c0[l] < inf");
    const int C = c->opt.chains;
    int rc;
    if (!c->d_top && (rc = dalloc(c, (void **)&c->d_top, (size_t)C * sizeof(TopState)))) return rc;
    TopPriors P{};
    P.a_b = p->a_b;
    P.b_b = p->b_b;
    for (int l = 0; l < L; ++l) P.c0[l] = p->c0[l];
    P.key0 = (uint32_t)p->seed;
    P.key1 = (uint32_t)(p->seed >> 32);
    P.L = L;
    P.mask = p->mask;
    // start: b = the first dataset's prior rate, psi = 0 (the two-level priors)
    std::vector<TopState> init((size_t)C);
    for (auto &T : init) {
        T = TopState{};
        T.b = c->seg.front().info.b;
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpy(c->d_top, init.data(), init.size() * sizeof(TopState), hipMemcpyHostToDevice));
    c->top_pri = P;
    c->top_on = true;
    for (auto &S : c->seg) S.info.top = c->d_top + S.chain;
    return upload_segs(c);
}

int fb_get_top(fb_ctx *c, int32_t chain, double *b, double *psi, double *mean, double *msq, int32_t *tries)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (!c->top_on) return fail(c, FB_EINVAL, "no top level (fb_set_top_level)");
    if (chain < 0 || chain >= c->opt.chains) return fail(c, FB_EINVAL, "bad chain");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    TopState T;
    HIPCHK(c, hipMemcpy(&T, c->d_top + chain, sizeof(TopState), hipMemcpyDeviceToHost));
    const int L = c->top_pri.L;
    if (b) *b = T.b;
    if (tries) *tries = T.tries;
    for (int l = 0; l < L; ++l) {
        if (psi) psi[l] = T.psi[l];
    }
    for (int i = 0; i < 1 + L; ++i) {
        if (mean) mean[i] = T.mom[i].x;
        if (msq) msq[i] = T.mom[i].y;
    }
    return c->sticky;
}

int fb_set_top(fb_ctx *c, int32_t chain, double b, const double *psi)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (!c->top_on) return fail(c, FB_EINVAL, "no top level (fb_set_top_level)");
    if (chain < 0 || chain >= c->opt.chains || !psi) return fail(c, FB_EINVAL, "bad chain or psi");
    if (!(b > 0.0) || !std::isfinite(b)) return fail(c, FB_EINVAL, "need 0 < b < inf");
    const int L = c->top_pri.L;
    for (int l = 0; l < L; ++l)
        if (!std::isfinite(psi[l])) return fail(c, FB_EINVAL, "non-finite psi");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    TopState T;
    HIPCHK(c, hipMemcpy(&T, c->d_top + chain, sizeof(TopState), hipMemcpyDeviceToHost));
    T.b = b;
    for (int l = 0; l < L; ++l) T.psi[l] = psi[l];
    HIPCHK(c, hipMemcpy(c->d_top + chain, &T, sizeof(TopState), hipMemcpyHostToDevice));
    return c->sticky;
}

int fb_event_counts(fb_ctx *c, int32_t seg, int32_t *counts, int64_t *n_sweeps)
{
    if (!valid_seg(c, seg)) return fail(c, FB_EINVAL, "bad segment");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    const SegmentH &S = c->seg[seg];
    const SegInfo &I = S.info;
    if (n_sweeps) {
        const int64_t from = I.n_ev > 0 ? std::max<int64_t>(c->opt.burnin, I.ev_from) : c->m;
        *n_sweeps = c->m > from ? c->m - from : 0;
    }
    if (counts && I.n_ev > 0) {
        std::vector<int32_t> buf((size_t)I.n_ev * (size_t)S.Gp);
        HIPCHK(c, hipMemcpy(buf.data(), I.ev_count, buf.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t g = 0; g < S.G; ++g)
            for (int e = 0; e < I.n_ev; ++e) counts[g * I.n_ev + e] = buf[(size_t)e * (size_t)S.Gp + (size_t)g];
    }
    return c->sticky;
}

int fb_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n)
{
    if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(nullptr, FB_EINVAL, "bad arguments");
    if (n == 0) return FB_OK;
    void *dc = nullptr, *dk = nullptr, *dout = nullptr;
    auto cleanup = [&]() { (void)hipFree(dc); (void)hipFree(dk); (void)hipFree(dout); };
    if (hipMalloc(&dc, n * 16) != hipSuccess || hipMalloc(&dk, n * 8) != hipSuccess ||
        hipMalloc(&dout, n * 16) != hipSuccess) {
        cleanup();
        return fail(nullptr, FB_ENOMEM, "hipMalloc failed");
    }
    hipError_t e = hipMemcpy(dc, ctr, n * 16, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dk, key, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_philox((const uint4 *)dc, (const uint2 *)dk, (uint4 *)dout, n, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, dout, n * 16, hipMemcpyDeviceToHost);
    cleanup();
    if (e != hipSuccess) return fail(nullptr, FB_EDEVICE, std::string("fb_philox: ") + hipGetErrorString(e));
    return FB_OK;
}

int fb_last_sweep_time(fb_ctx *c, double *ms, int64_t *sweeps)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    HIPCHK(c, hipEventSynchronize(c->ev1));
    float t = 0;
    HIPCHK(c, hipEventElapsedTime(&t, c->ev0, c->ev1));
    if (ms) *ms = t;
    if (sweeps) *sweeps = c->last_n;
    return FB_OK;
}

int fb_profile(fb_ctx *c, int32_t every, int32_t max_samples)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (every < 0 || max_samples < 0) return fail(c, FB_EINVAL, "every and max_samples must be >= 0");
    HIPCHK(c, hipStreamSynchronize(c->st));
    const size_t need = 8 * (size_t)max_samples;
    while (c->prof_ev.size() < need) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->prof_ev.push_back(e);
    }
    c->prof_hyp.assign((size_t)max_samples, 0);
    c->prof_shift.assign((size_t)max_samples, 0);
    c->prof_every = every;
    c->prof_cap = max_samples;
    c->prof_n = 0;
    c->prof_count = 0;
    return FB_OK;
}

int fb_kernel_times(fb_ctx *c, double *eps_ms, double *gb_ms, double *hyper_ms, double *shift_ms,
                    int64_t *samples)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    HIPCHK(c, hipStreamSynchronize(c->st));
    double te = 0, tg = 0, th = 0, ts = 0;
    int64_t nh = 0, ns = 0;
    for (int32_t i = 0; i < c->prof_n; ++i) {
        const hipEvent_t *pe = &c->prof_ev[8 * (size_t)i];
        float a = 0, b = 0, h = 0, sh = 0;
        HIPCHK(c, hipEventElapsedTime(&a, pe[0], pe[1]));
        HIPCHK(c, hipEventElapsedTime(&b, pe[2], pe[3]));
        if (c->prof_hyp[i]) {
            HIPCHK(c, hipEventElapsedTime(&h, pe[4], pe[5]));
            th += h;
            ++nh;
        }
        if (c->prof_shift[i]) {
            HIPCHK(c, hipEventElapsedTime(&sh, pe[6], pe[7]));
            ts += sh;
            ++ns;
        }
        te += a;
        tg += b;
    }
    if (eps_ms) *eps_ms = c->prof_n ? te / c->prof_n : 0.0;
    if (gb_ms) *gb_ms = c->prof_n ? tg / c->prof_n : 0.0;
    if (hyper_ms) *hyper_ms = nh ? th / nh : 0.0;
    if (shift_ms) *shift_ms = ns ? ts / ns : 0.0;
    if (samples) *samples = c->prof_n;
    c->prof_n = 0;
    c->prof_count = 0;
    return FB_OK;
}

int fb_set_launch(fb_ctx *c, int32_t samples_per_wave, int32_t fuse_hyper)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    int maxN = 1;
    for (auto &S : c->seg) maxN = std::max(maxN, S.N);
    if (samples_per_wave < 1 || samples_per_wave > maxN)
        return fail(c, FB_EINVAL, "samples_per_wave must be in [1, max N]");
    if (fuse_hyper != 0 && fuse_hyper != 1) return fail(c, FB_EINVAL, "fuse_hyper must be 0 or 1");
    int rc;
    if (samples_per_wave != c->spw && (rc = build_items(c, samples_per_wave))) return rc;
    c->fuse = fuse_hyper != 0;
    return FB_OK;
}

int fb_set_beta_lanes(fb_ctx *c, int32_t lanes)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (lanes != 1 && lanes != 2) return fail(c, FB_EINVAL, "lanes must be 1 or 2");
    c->beta_lanes = lanes;
    return FB_OK;
}

int32_t fb_get_beta_lanes(const fb_ctx *c) { return c ? c->beta_lanes : 0; }

int fb_set_hyper_split(fb_ctx *c, int32_t on)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (on != 0 && on != 1) return fail(c, FB_EINVAL, "on must be 0 or 1");
    c->hyper_split = on != 0;
    return FB_OK;
}

int32_t fb_get_hyper_split(const fb_ctx *c) { return c ? (c->hyper_split ? 1 : 0) : 0; }

int fb_set_tile_sweep(fb_ctx *c, int32_t on)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (on != 0 && on != 1) return fail(c, FB_EINVAL, "on must be 0 or 1");
    c->tile = on != 0;
    return FB_OK;
}

int32_t fb_get_tile_sweep(const fb_ctx *c) { return c ? (c->tile ? 1 : 0) : 0; }

int fb_set_shift_fusion(fb_ctx *c, int32_t fused)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (fused != 0 && fused != 1) return fail(c, FB_EINVAL, "fused must be 0 or 1");
    c->fuse_shift = fused != 0;
    return FB_OK;
}

int fb_get_launch(const fb_ctx *c, int32_t *samples_per_wave, int32_t *fuse_hyper)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (samples_per_wave) *samples_per_wave = c->spw;
    if (fuse_hyper) *fuse_hyper = c->fuse ? 1 : 0;
    return FB_OK;
}

namespace {

// Every device buffer a sweep writes, except traces and training pairs.
void sweep_buffers(fb_ctx *c, std::vector<std::pair<void *, size_t>> &out)
{
    out.clear();
    for (auto &S : c->seg) {
        const SegInfo &I = S.info;
        const size_t Gp = (size_t)S.Gp, N = (size_t)S.N, L = (size_t)S.L, e = c->esz;
        for (void *p : {I.eps, I.w_eps, I.wa_eps}) out.push_back({p, N * Gp * e});
        for (void *p : {I.gam, I.w_gam, I.wa_gam}) out.push_back({p, Gp * e});
        for (void *p : {I.beta, I.w_beta, I.wa_beta}) out.push_back({p, L * Gp * e});
        out.push_back({(void *)I.mom_eps, N * Gp * sizeof(double2)});
        out.push_back({(void *)I.mom_gam, Gp * sizeof(double2)});
        out.push_back({(void *)I.mom_beta, L * Gp * sizeof(double2)});
        out.push_back({(void *)I.partials, (size_t)I.pstride * kMaxParts * sizeof(double)});
        out.push_back({(void *)S.d_hyp, sizeof(HyperState)});
        out.push_back({(void *)I.hyp_flag, kHypFlags * sizeof(int64_t)});
        if (I.dbg_eps) {
            out.push_back({(void *)I.dbg_eps, N * Gp * sizeof(int4)});
            out.push_back({(void *)I.dbg_gam, Gp * sizeof(int4)});
            out.push_back({(void *)I.dbg_beta, L * Gp * sizeof(int4)});
        }
        if (I.imh_last) {
            out.push_back({(void *)I.imh_count, Gp * sizeof(int32_t)});
            out.push_back({(void *)I.imh_last, Gp * sizeof(int32_t)});
            out.push_back({(void *)I.imh_stat, Gp * sizeof(int2)});
        }
    }
    out.push_back({(void *)c->d_err, kErrWordsHost * sizeof(int)});
}

}  // namespace

int fb_autotune(fb_ctx *c, int32_t trial_sweeps, int32_t *samples_per_wave, int32_t *fuse_hyper,
                double *ms_per_sweep, double *table)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (trial_sweeps < 1) return fail(c, FB_EINVAL, "trial_sweeps must be >= 1");
    if (c->sticky) return c->sticky;
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::vector<std::pair<void *, size_t>> bufs;
    sweep_buffers(c, bufs);
    size_t total = 0;
    for (auto &b : bufs) total += (b.second + 255) / 256 * 256;
    char *snap = nullptr;
    if (int rcm = dmem(c, (void **)&snap, total)) return rcm;
    auto copy_all = [&](bool save) -> hipError_t {
        size_t off = 0;
        for (auto &b : bufs) {
            hipError_t e = save ? hipMemcpyAsync(snap + off, b.first, b.second, hipMemcpyDeviceToDevice, c->st)
                                : hipMemcpyAsync(b.first, snap + off, b.second, hipMemcpyDeviceToDevice, c->st);
            if (e != hipSuccess) return e;
            off += (b.second + 255) / 256 * 256;
        }
        return hipStreamSynchronize(c->st);
    };
    int maxN = 1;
    for (auto &S : c->seg) maxN = std::max(maxN, S.N);
    const int64_t m0 = c->m;
    const int spw0 = c->spw;
    const bool fuse0 = c->fuse;
    int best_spw = spw0, rc = FB_OK;
    bool best_fuse = fuse0, best_tile = false;
    c->tile = false;
    double best = 1e300;
    hipError_t e = copy_all(true);
    // one trial from the saved state: two warm-up sweeps, then trial_sweeps timed
    auto trial = [&](double &per) -> bool {
        SweepMode md;
        md.learned = c->beta_mode == FB_BETA_LEARNED || c->beta_mode == FB_BETA_LAPLACE;
        md.learned_kernel = md.learned;
        md.laplace = c->beta_mode == FB_BETA_LAPLACE;
        md.no_trace = true;
        if ((rc = run_sweeps(c, 2, md))) return false;
        if ((e = hipStreamSynchronize(c->st)) != hipSuccess) return false;
        if ((rc = run_sweeps(c, trial_sweeps, md))) return false;
        if ((e = hipEventSynchronize(c->ev1)) != hipSuccess) return false;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, c->ev0, c->ev1)) != hipSuccess) return false;
        per = ms / trial_sweeps;
        c->m = m0;
        e = copy_all(false);
        return e == hipSuccess;
    };
    if (table)
        for (int i = 0; i < 10; ++i) table[i] = -1.0;
    for (int k = 0; e == hipSuccess && rc == FB_OK && k < 8; ++k) {
        const int spw = 1 << (k >> 1), fz = k & 1;
        if (spw > std::min(maxN, 8)) continue;
        if ((rc = build_items(c, spw))) break;
        c->fuse = fz != 0;
        double per = 0.0;
        if (!trial(per)) break;
        if (table) table[k] = per;
        if (per < best) { best = per; best_spw = spw; best_fuse = fz != 0; }
    }
    // the single-launch sweep (slice steps for beta, one lane, no shift step)
    const bool plain_slice = c->beta_mode == FB_BETA_SLICE && !((c->opt.update_mask >> kKindShift) & 1u);
    const int lanes_in = c->beta_lanes;
    for (int fz = 1; plain_slice && fz >= 0 && e == hipSuccess && rc == FB_OK; --fz) {
        c->tile = true;
        c->beta_lanes = 1;
        c->fuse = fz != 0;
        double per = 0.0;
        const bool ok = trial(per);
        c->tile = false;
        c->beta_lanes = lanes_in;
        if (!ok) break;
        if (table) table[8 + (1 - fz)] = per;
        if (per < best) { best = per; best_fuse = fz != 0; best_tile = true; }
    }
    // with the slice steps for beta, the other number of lanes per gene at the best shape
    const int lanes0 = c->beta_lanes;
    int best_lanes = lanes0;
    const bool slice_beta = c->beta_mode == FB_BETA_SLICE &&
                            (!((c->opt.update_mask >> kKindShift) & 1u) || c->fuse_shift);
    if (!best_tile && slice_beta && e == hipSuccess && rc == FB_OK && (rc = build_items(c, best_spw)) == FB_OK) {
        c->fuse = best_fuse;
        c->beta_lanes = 3 - lanes0;
        double per = 0.0;
        if (trial(per) && per < best) {
            best = per;
            best_lanes = c->beta_lanes;
        }
    }
    c->beta_lanes = best_tile ? 1 : best_lanes;
    c->tile = best_tile;
    c->m = m0;
    if (e == hipSuccess) e = copy_all(false);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    dfree(c, snap);
    if (e != hipSuccess) return fail(c, FB_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    if (rc) return rc;
    c->fuse = best_fuse;
    if ((rc = build_items(c, best_spw))) return rc;
    if (samples_per_wave) *samples_per_wave = best_spw;
    if (fuse_hyper) *fuse_hyper = best_fuse ? 1 : 0;
    if (ms_per_sweep) *ms_per_sweep = best;
    (void)spw0;
    return FB_OK;
}

void fb_default_train_opts(fb_train_opts *o)
{
    if (!o) return;
    o->epochs = 200;
    o->pairs_per_epoch = 10240;
    o->minibatch = 1024;
    o->lr = 1e-3;
    o->seed = 1;
}

static int same_design(fb_ctx *c)
{
    for (auto &S : c->seg) {
        const DatasetH &D = c->ds[S.dataset], &D0 = c->ds[c->seg[0].dataset];
        if (D.L != D0.L || D.des.R != D0.des.R) return fail(c, FB_EINVAL, "the proposal needs one design for every segment");
        if (2 * D.des.R + 2 * D.L > kMlpF) return fail(c, FB_EINVAL, "too many features for the proposal network");
    }
    return FB_OK;
}

int fb_proposal_collect(fb_ctx *c, int64_t sweeps, int32_t every)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (sweeps < 0 || every < 1) return fail(c, FB_EINVAL, "need sweeps >= 0 and every >= 1");
    if (c->sticky) return c->sticky;
    int rc;
    if ((rc = same_design(c)) || (rc = ensure_learned(c))) return rc;
    const int64_t slots = std::max<int64_t>(1, sweeps / every + 1);
    const int64_t need = slots * c->totalG;
    if (need > c->pair_cap) {
        if ((rc = dalloc(c, (void **)&c->d_pairs, (size_t)need * kPairStride * sizeof(float)))) return rc;
        c->pair_cap = need;
    }
    int64_t off = 0;
    for (auto &S : c->seg) {
        S.info.pairs = c->d_pairs + off * kPairStride;
        off += S.G;
    }
    if ((rc = upload_segs(c))) return rc;
    c->pair_n = 0;
    SweepMode md;
    md.learned_kernel = true;
    md.learned = false;
    md.collect_every = every;
    return run_sweeps(c, sweeps, md);
}

int fb_proposal_train(fb_ctx *c, const fb_train_opts *opts, double *epoch_loss)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    fb_train_opts o;
    fb_default_train_opts(&o);
    if (opts) o = *opts;
    if (o.epochs < 1 || o.minibatch < 32 || o.minibatch % 32 || o.pairs_per_epoch < o.minibatch || !(o.lr > 0))
        return fail(c, FB_EINVAL, "bad training options");
    if (c->pair_n < 2) return fail(c, FB_ESTATE, "no training pairs: call fb_proposal_collect first");
    int rc;
    if ((rc = ensure_net(c))) return rc;
    // the moments, Adam state, minibatch buffers and loss sums of this call
    // are given back when it returns
    TempScope scratch_of_call(c);
    const int L = c->seg[0].L;
    const int64_t P = c->pair_n;
    HIPCHK(c, hipStreamSynchronize(c->st));
    // standardisation from the pairs
    double *d_mom = nullptr, *d_momw = nullptr;
    if ((rc = dalloc(c, (void **)&d_mom, 2 * kPairStride * sizeof(double)))) return rc;
    if ((rc = dalloc(c, (void **)&d_momw, 2 * (size_t)kPairStride * kColChunks * sizeof(double)))) return rc;
    HIPCHK(c, launch_col_moments(c->d_pairs, P, kPairStride, d_momw, d_mom, c->st));
    std::vector<double> mom(2 * kPairStride);
    HIPCHK(c, hipMemcpyAsync(mom.data(), d_mom, mom.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::vector<float> blk(kMlpParams, 0.0f);
    for (int k = 0; k < kMlpF; ++k) {
        const double mu = mom[2 * k] / (double)P;
        const double var = std::max(0.0, mom[2 * k + 1] / (double)P - mu * mu);
        blk[kOffFmean + k] = (float)mu;
        blk[kOffFscale + k] = var > 1e-12 ? (float)(1.0 / std::sqrt(var)) : 0.0f;
    }
    // The targets are already whitened by the per-gene Laplace approximation,
    // so the output map stays at the identity (omean 0, oscale 1) and the
    // output layer starts at zero: the untrained network is exactly the
    // Laplace proposal, and training only moves it where the pairs show a
    // departure from it.
    for (int l = 0; l < 8; ++l) {
        blk[kOffOmean + l] = 0.0f;
        blk[kOffOscale + l] = 1.0f;
    }
    // seeded initial weights of the hidden layers: N(0, 1 / fan_in)
    for (int i = 0; i < kMlpF * kMlpH; ++i)
        blk[kOffW1 + i] = (float)(std_normal_key(o.seed, 1, i) / std::sqrt((double)kMlpF));
    for (int i = 0; i < kMlpH * kMlpH; ++i)
        blk[kOffW2 + i] = (float)(std_normal_key(o.seed, 2, i) / std::sqrt((double)kMlpH));
    HIPCHK(c, hipMemcpy(c->d_master, blk.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    float *d_m = nullptr, *d_v = nullptr;
    if ((rc = dalloc(c, (void **)&d_m, kMlpParams * sizeof(float)))) return rc;
    if ((rc = dalloc(c, (void **)&d_v, kMlpParams * sizeof(float)))) return rc;
    TrainBufs t;
    if ((rc = alloc_train(c, t, o.minibatch, L))) return rc;
    const int steps = o.pairs_per_epoch / o.minibatch;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int64_t it = 0;
    // per-epoch sums of the per-row losses, added on the device after each
    // step (no host round trip inside the loop)
    double *d_esum = nullptr;
    if (epoch_loss && (rc = dalloc(c, (void **)&d_esum, (size_t)o.epochs * sizeof(double)))) return rc;
    const int64_t nopt = kOffOmean - kOffW1;   // W1 .. b3 are trained
    for (int e = 0; e < o.epochs; ++e) {
        for (int sidx = 0; sidx < steps; ++sidx) {
            HIPCHK(c, launch_gather_pairs(c->d_pairs, P, L, c->d_master, t.X, t.Tg, o.minibatch, (uint32_t)e,
                                          (uint32_t)sidx, (uint32_t)o.seed, (uint32_t)(o.seed >> 32), c->st));
            HIPCHK(c, mlp_forward_backward(c->d_master, t, L, c->st));
            ++it;
            const float c1 = 1.0f - std::pow(b1, (float)it), c2 = 1.0f - std::pow(b2, (float)it);
            hipLaunchKernelGGL(adam_step, dim3((unsigned)((nopt + 255) / 256)), dim3(256), 0, c->st,
                               c->d_master + kOffW1, t.grad + kOffW1, d_m + kOffW1, d_v + kOffW1, nopt, (float)o.lr,
                               b1, b2, eps, c1, c2);
            HIPCHK(c, hipGetLastError());
            if (epoch_loss) {
                hipLaunchKernelGGL(sum_rows_into, dim3(1), dim3(256), 0, c->st, t.loss, (int64_t)o.minibatch,
                                   d_esum + e);
                HIPCHK(c, hipGetLastError());
            }
        }
    }
    if (epoch_loss) {
        std::vector<double> es((size_t)o.epochs);
        HIPCHK(c, hipMemcpyAsync(es.data(), d_esum, es.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        for (int e = 0; e < o.epochs; ++e) epoch_loss[e] = es[(size_t)e] / ((double)steps * o.minibatch);
    }
    HIPCHK(c, hipMemcpyAsync(blk.data(), c->d_master, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (float v : blk)
        if (!std::isfinite(v)) return fail(c, FB_ENUMERIC, "training produced non-finite parameters");
    if ((rc = pack_net(c, c->d_master, c->d_net, c->st))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->net_ready = true;
    return FB_OK;
}

int fb_proposal_calibrate(fb_ctx *c, int64_t sweeps, double min_accept)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (sweeps < 1) return fail(c, FB_EINVAL, "need sweeps >= 1");
    const bool lap = c->beta_mode == FB_BETA_LAPLACE;
    if (!lap && !c->net_ready) return fail(c, FB_ESTATE, "no network: train or load one first");
    if (c->sticky) return c->sticky;
    int rc;
    if ((rc = ensure_learned(c))) return rc;
    if (lap && (rc = ensure_idnet(c))) return rc;
    for (auto &S : c->seg) {
        HIPCHK(c, hipMemsetAsync(S.info.fallback, 0, (size_t)S.Gp * sizeof(int32_t), c->st));
        HIPCHK(c, hipMemsetAsync(S.info.imh_count, 0, (size_t)S.Gp * sizeof(int32_t), c->st));
    }
    if ((rc = build_fallback(c))) return rc;     // no fallback groups while calibrating
    SweepMode md;
    md.learned_kernel = true;
    md.learned = true;
    md.laplace = lap;
    md.count_imh = true;
    if ((rc = run_sweeps(c, sweeps, md))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (auto &S : c->seg) {
        std::vector<int32_t> cnt((size_t)S.Gp), mask((size_t)S.Gp, 0);
        HIPCHK(c, hipMemcpy(cnt.data(), S.info.imh_count, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t g = 0; g < S.G; ++g) mask[g] = ((double)cnt[g] / (double)sweeps) < min_accept ? 1 : 0;
        HIPCHK(c, hipMemcpy(S.info.fallback, mask.data(), mask.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    return build_fallback(c);
}

int fb_set_beta_update(fb_ctx *c, int32_t mode)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    if (mode != FB_BETA_SLICE && mode != FB_BETA_LEARNED && mode != FB_BETA_LAPLACE)
        return fail(c, FB_EINVAL, "unknown beta update");
    if (mode == FB_BETA_LEARNED) {
        if (!c->net_ready) return fail(c, FB_ESTATE, "no network: train or load one first");
        int rc;
        if ((rc = same_design(c)) || (rc = ensure_learned(c))) return rc;
    }
    if (mode == FB_BETA_LAPLACE) {
        int rc;
        if ((rc = ensure_learned(c)) || (rc = ensure_idnet(c))) return rc;
    }
    c->beta_mode = mode;
    return FB_OK;
}

int fb_proposal_get(fb_ctx *c, fb_mlp *out)
{
    if (!c || !out) return fail(c, FB_EINVAL, "NULL argument");
    if (!c->net_ready) return fail(c, FB_ESTATE, "no network");
    std::vector<float> blk(kMlpParams);
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpy(blk.data(), c->d_master, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    block_to_mlp(blk, out);
    return FB_OK;
}

int fb_proposal_set(fb_ctx *c, const fb_mlp *in)
{
    if (!c) return fail(nullptr, FB_EINVAL, "NULL context");
    std::vector<float> blk;
    if (!mlp_to_block(in, blk)) return fail(c, FB_EINVAL, "every parameter array is required");
    for (float v : blk) if (!std::isfinite(v)) return fail(c, FB_EINVAL, "parameters must be finite");
    for (int l = 0; l < 8; ++l) if (!(blk[kOffOscale + l] > 0)) return fail(c, FB_EINVAL, "oscale must be > 0");
    int rc;
    if ((rc = same_design(c)) || (rc = ensure_net(c)) || (rc = ensure_learned(c))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpy(c->d_master, blk.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    if ((rc = pack_net(c, c->d_master, c->d_net, c->st))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->net_ready = true;
    return FB_OK;
}

int fb_fallback(fb_ctx *c, int32_t seg, int32_t *get, const int32_t *set)
{
    if (!valid_seg(c, seg)) return fail(c, FB_EINVAL, "bad segment");
    int rc;
    if ((rc = ensure_learned(c))) return rc;
    SegmentH &S = c->seg[seg];
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (set) {
        std::vector<int32_t> m((size_t)S.Gp, 0);
        for (int64_t g = 0; g < S.G; ++g) m[g] = set[g] ? 1 : 0;
        HIPCHK(c, hipMemcpy(S.info.fallback, m.data(), m.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        if ((rc = build_fallback(c))) return rc;
    }
    if (get) HIPCHK(c, hipMemcpy(get, S.info.fallback, (size_t)S.G * sizeof(int32_t), hipMemcpyDeviceToHost));
    return FB_OK;
}

int fb_imh_last(fb_ctx *c, int32_t seg, int32_t *last)
{
    if (!valid_seg(c, seg) || !last) return fail(c, FB_EINVAL, "bad segment or NULL output");
    if (!c->learned_ready) return fail(c, FB_ESTATE, "no learned-proposal sweep has run");
    int rc = fb_sync(c);
    if (rc && rc != FB_ENUMERIC) return rc;
    HIPCHK(c, hipMemcpy(last, c->seg[seg].info.imh_last, (size_t)c->seg[seg].G * sizeof(int32_t),
                        hipMemcpyDeviceToHost));
    return c->sticky;
}

int fb_features(fb_ctx *c, int32_t seg, float *phi)
{
    if (!valid_seg(c, seg) || !phi) return fail(c, FB_EINVAL, "bad segment or NULL output");
    SegmentH &S = c->seg[seg];
    float *d = nullptr;
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (int rcm = dmem(c, (void **)&d, (size_t)S.G * 32 * sizeof(float))) return rcm;
    hipError_t e = launch_features(c->prec, c->d_segs + seg, S.G, d, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e == hipSuccess) e = hipMemcpy(phi, d, (size_t)S.G * 32 * sizeof(float), hipMemcpyDeviceToHost);
    dfree(c, d);
    if (e != hipSuccess) return fail(c, FB_EDEVICE, std::string("fb_features: ") + hipGetErrorString(e));
    return FB_OK;
}

// ---- test entry points on host data, each with its own temporary context ----
int fb_mfma_probe(const float *A, const float *B, float *C)
{
    if (!A || !B || !C) return fail(nullptr, FB_EINVAL, "NULL argument");
    float *d = nullptr;
    if (hipMalloc((void **)&d, (512 + 512 + 1024) * sizeof(float)) != hipSuccess) return fail(nullptr, FB_ENOMEM, "hipMalloc");
    hipError_t e = hipMemcpy(d, A, 512 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + 512, B, 512 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(mfma_probe, dim3(1), dim3(64), 0, nullptr, d, d + 512, d + 1024);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(C, d + 1024, 1024 * sizeof(float), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(nullptr, FB_EDEVICE, std::string("fb_mfma_probe: ") + hipGetErrorString(e));
    return FB_OK;
}

int fb_mlp_forward(const fb_mlp *w, int32_t L, const float *phi, int64_t B, float *mu, float *ls, float *off)
{
    std::vector<float> blk;
    if (!mlp_to_block(w, blk) || L < 1 || L > kMaxL || B < 0 || (B > 0 && (!phi || !mu || !ls)))
        return fail(nullptr, FB_EINVAL, "bad arguments");
    if (B == 0) return FB_OK;
    fb_ctx tmp;
    int rc;
    float *d_master = nullptr, *d_phi = nullptr, *d_out = nullptr;
    MlpDev *d_net = nullptr;
    if ((rc = dalloc(&tmp, (void **)&d_master, kMlpParams * sizeof(float))) ||
        (rc = dalloc(&tmp, (void **)&d_net, sizeof(MlpDev))) ||
        (rc = dalloc(&tmp, (void **)&d_phi, (size_t)B * 32 * sizeof(float))) ||
        (rc = dalloc(&tmp, (void **)&d_out, (size_t)B * mlp_outputs(L) * sizeof(float)))) {
        g_thread_err = tmp.err;
        for (void *p : tmp.allocs) (void)hipFree(p);
        return rc;
    }
    hipError_t e = hipMemcpy(d_master, blk.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_phi, phi, (size_t)B * 32 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess && pack_net(&tmp, d_master, d_net, nullptr) != FB_OK) e = hipErrorUnknown;
    const size_t K = (size_t)L * (L - 1) / 2;
    float *d_off = d_out + 2 * (size_t)B * L;
    if (e == hipSuccess) e = launch_mlp_infer_raw(d_phi, B, L, d_net, d_out, d_out + (size_t)B * L, d_off, nullptr);
    if (e == hipSuccess) e = hipMemcpy(mu, d_out, (size_t)B * L * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ls, d_out + (size_t)B * L, (size_t)B * L * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess && off && K > 0)
        e = hipMemcpy(off, d_off, (size_t)B * K * sizeof(float), hipMemcpyDeviceToHost);
    for (void *p : tmp.allocs) (void)hipFree(p);
    if (e != hipSuccess) return fail(nullptr, FB_EDEVICE, std::string("fb_mlp_forward: ") + hipGetErrorString(e));
    return FB_OK;
}

int fb_mlp_loss_grad(const fb_mlp *w, int32_t L, const float *phi, const float *target, int64_t B, float *loss,
                     fb_mlp *grad)
{
    std::vector<float> blk;
    if (!mlp_to_block(w, blk) || L < 1 || L > kMaxL || B < 32 || B % 32 || !phi || !target)
        return fail(nullptr, FB_EINVAL, "bad arguments (B must be a positive multiple of 32)");
    fb_ctx tmp;
    int rc;
    float *d_master = nullptr, *d_pairs = nullptr;
    TrainBufs t;
    if ((rc = dalloc(&tmp, (void **)&d_master, kMlpParams * sizeof(float))) ||
        (rc = dalloc(&tmp, (void **)&d_pairs, (size_t)B * kPairStride * sizeof(float))) ||
        (rc = alloc_train(&tmp, t, (int)B, L))) {
        g_thread_err = tmp.err;
        for (void *p : tmp.allocs) (void)hipFree(p);
        return rc;
    }
    // rows in order: standardise on the host side of the copy (plain arithmetic)
    std::vector<float> X((size_t)B * kMlpF);
    for (int64_t b = 0; b < B; ++b)
        for (int k = 0; k < kMlpF; ++k)
            X[b * kMlpF + k] = std::min(std::max((phi[b * 32 + k] - blk[kOffFmean + k]) * blk[kOffFscale + k],
                                                 -kMlpClip), kMlpClip);
    hipError_t e = hipMemcpy(d_master, blk.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.X, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.Tg, target, (size_t)B * L * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = mlp_forward_backward(d_master, t, L, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<float> lv((size_t)B), gb(kMlpParams);
    if (e == hipSuccess) e = hipMemcpy(lv.data(), t.loss, lv.size() * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(gb.data(), t.grad, gb.size() * sizeof(float), hipMemcpyDeviceToHost);
    for (void *p : tmp.allocs) (void)hipFree(p);
    if (e != hipSuccess) return fail(nullptr, FB_EDEVICE, std::string("fb_mlp_loss_grad: ") + hipGetErrorString(e) + " " + tmp.err);
    if (loss) {
        double sum = 0.0;
        for (float v : lv) sum += v;
        *loss = (float)(sum / (double)B);
    }
    if (grad) block_to_mlp(gb, grad);
    return FB_OK;
}

const char *fb_last_error(const fb_ctx *c) { return c ? c->err.c_str() : g_thread_err.c_str(); }

const char *fb_strerror(int code)
{
    switch (code) {
    case FB_OK: return "ok";
    case FB_EINVAL: return "invalid argument";
    case FB_ENOMEM: return "out of memory";
    case FB_EDEVICE: return "HIP runtime error";
    case FB_ENUMERIC: return "numeric failure in a draw";
    case FB_ESTATE: return "call not valid in this state";
    default: return "unknown error";
    }
}

}  // extern "C"
