// fbmc_mlp.hip -- the learned beta proposal's network on gfx950 matrix cores.
//
// The network maps a gene's 32 features to a Gaussian proposal for its L
// coefficients -- the mean, the log-diagonal of a lower-triangular factor and
// its strict lower triangle -- with two 128-wide GELU layers
// (F = 32 -> H = 128 -> H = 128 -> O = 64 padded outputs, 2L + L(L-1)/2 used).
// Products use v_mfma_f32_32x32x16_bf16: BF16 operands, FP32 accumulation.
// Weights and activations live in FP32; a fragment is rounded to BF16 as it is
// loaded into the matrix core.
//
// 32x32x16 operand layout (wavefront of 64 lanes, lane = 32 h + i):
//   A (32 x 16): lane holds A[i][8 h + j], j = 0..7
//   B (16 x 32): lane holds B[8 h + j][i], j = 0..7
//   C (32 x 32): lane holds C[8 (r / 4) + 4 h + (r % 4)][i], r = 0..15
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fbmc_mlp.hpp"

namespace fbmc {

__device__ inline bf16x8 to_bf16x8(const float *v)
{
    bf16x8 r;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = (__bf16)v[j];
    return r;
}

// One MFMA on explicit operands: used to check the lane layout on the device.
__global__ void mfma_probe(const float *A, const float *B, float *C)
{
    const int lane = (int)threadIdx.x;
    const int i = lane & 31, h = lane >> 5;
    float a[8], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = A[i * 16 + 8 * h + j];      // A is 32 x 16 row-major
        b[j] = B[(8 * h + j) * 32 + i];    // B is 16 x 32 row-major
    }
    floatx16 acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(to_bf16x8(a), to_bf16x8(b), acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) C[(8 * (r >> 2) + 4 * h + (r & 3)) * 32 + i] = acc[r];
}

// C[M][N] = (accumulate ? C : 0) + op(A) op(B), op(A) is M x K, op(B) is K x N.
// A is [M][lda] (or [K][lda] read transposed when tA), B is [K][ldb] (or [N][ldb]
// when tB).  M, N multiples of 32 and K a multiple of 16.  One workgroup of
// kSplit wavefronts per 32 x 32 tile of C: wavefront w takes the k-steps
// w, w + kSplit, ... (16 columns of op(A) each), and the partial tiles are
// added in wavefront order through LDS, so a long K (the weight gradients,
// K = minibatch) runs on kSplit times as many wavefronts in a fixed order.
template <int kSplit>
__global__ __launch_bounds__(64 * kSplit) void gemm_bf16(const float *__restrict__ A, int lda, int tA,
                                                         const float *__restrict__ B, int ldb, int tB,
                                                         float *__restrict__ C, int ldc, int M, int N, int K,
                                                         int accumulate)
{
    const int tilesN = N / 32;
    const int m0 = (int)(blockIdx.x / tilesN) * 32, n0 = (int)(blockIdx.x % tilesN) * 32;
    if (m0 >= M) return;      // the whole workgroup
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int i = lane & 31, h = lane >> 5;
    floatx16 acc = {};
    // the operands of up to kGroup k-steps are loaded before their MFMAs (as
    // BF16 fragments), so a wavefront waits for memory once per group rather
    // than once per step
    constexpr int kGroup = 4;
#pragma unroll 1
    for (int g0 = 16 * wave; g0 < K; g0 += 16 * kSplit * kGroup) {
        bf16x8 fa[kGroup], fb[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            const int kb = g0 + 16 * kSplit * q + 8 * h;
            float a[8], b[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a[j] = 0.0f;
                b[j] = 0.0f;
            }
            if (kb < K) {
                if (tA) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) a[j] = A[(int64_t)(kb + j) * lda + m0 + i];
                } else {
                    const float4 *p = reinterpret_cast<const float4 *>(A + (int64_t)(m0 + i) * lda + kb);
                    const float4 u = p[0], v = p[1];
                    a[0] = u.x; a[1] = u.y; a[2] = u.z; a[3] = u.w; a[4] = v.x; a[5] = v.y; a[6] = v.z; a[7] = v.w;
                }
                if (tB) {
                    const float4 *p = reinterpret_cast<const float4 *>(B + (int64_t)(n0 + i) * ldb + kb);
                    const float4 u = p[0], v = p[1];
                    b[0] = u.x; b[1] = u.y; b[2] = u.z; b[3] = u.w; b[4] = v.x; b[5] = v.y; b[6] = v.z; b[7] = v.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 8; ++j) b[j] = B[(int64_t)(kb + j) * ldb + n0 + i];
                }
            }
            fa[q] = to_bf16x8(a);
            fb[q] = to_bf16x8(b);
        }
#pragma unroll
        for (int q = 0; q < kGroup; ++q)
            if (g0 + 16 * kSplit * q < K) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[q], fb[q], acc, 0, 0, 0);
    }
    if constexpr (kSplit > 1) {
        __shared__ float part[kSplit - 1][16][64];
        if (wave > 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) part[wave - 1][r][lane] = acc[r];
        }
        __syncthreads();
        if (wave > 0) return;
        for (int w = 0; w < kSplit - 1; ++w) {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] += part[w][r][lane];
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + 8 * (r >> 2) + 4 * h + (r & 3);
        float *dst = C + (int64_t)row * ldc + n0 + i;
        *dst = accumulate ? *dst + acc[r] : acc[r];
    }
}

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_df(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * __expf(-0.5f * z * z) * 0.3989422804014327f;
}

// Z[b][j] += bias[j]; H = gelu(Z) (H may alias nothing).
__global__ void bias_gelu(float *Z, const float *bias, float *H, int rows, int cols, int apply_gelu)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * cols) return;
    const int j = (int)(t % cols);
    const float z = Z[t] + bias[j];
    Z[t] = z;
    if (apply_gelu) H[t] = gelu_f(z);
}

// dZ = dH * gelu'(Z)
__global__ void gelu_backward(const float *Z, const float *dH, float *dZ, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dZ[t] = dH[t] * gelu_df(Z[t]);
}

// Gaussian NLL of targets T [B][L] under N(mu, Lc Lc^T) from the outputs
// O [B][Op]: mu_l = omean_l + oscale_l O_l, Lc = diag(oscale) Ls with
// Ls_ll = exp(O_{L+l}) and Ls_lj = O_{2L + l(l-1)/2 + j} (j < l).  Per row:
// loss = sum_l (log oscale_l + O_{L+l}) + |u|^2 / 2 with Ls u = (T - mu) / oscale
// (forward substitution), v = Ls^{-T} u (back substitution); the gradient of
// the batch mean is -v_l for the mean outputs, 1 - v_l u_l Ls_ll for the
// log-diagonal and -v_l u_j for the off-diagonal (l, j).  Writes dO (zero
// beyond the used outputs) and per-row losses.
__global__ void nll_grad(const float *O, int Op, const float *T, int L, const float *omean,
                         const float *oscale, float *dO, float *loss, int B)
{
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= B) return;
    const float invB = 1.0f / (float)B;
    const float *o = O + (int64_t)b * Op;
    float *g = dO + (int64_t)b * Op;
    // zero the row beyond the used outputs as float4s (Op is a multiple of 4
    // and rows are 16-byte aligned); the used ones are written below
    const int used = 2 * L + L * (L - 1) / 2;
    for (int j = used & ~3; j < Op; j += 4) *reinterpret_cast<float4 *>(g + j) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float u[8], v[8], dg[8];
    float tot = 0.0f;
    for (int l = 0; l < L; ++l) {
        dg[l] = __expf(o[L + l]);
        float s = (T[(int64_t)b * L + l] - (omean[l] + oscale[l] * o[l])) / oscale[l];
        for (int j = 0; j < l; ++j) s -= o[2 * L + l * (l - 1) / 2 + j] * u[j];
        u[l] = s / dg[l];
        tot += __logf(oscale[l]) + o[L + l] + 0.5f * u[l] * u[l];
    }
    for (int l = L - 1; l >= 0; --l) {
        float s = u[l];
        for (int i = l + 1; i < L; ++i) s -= o[2 * L + i * (i - 1) / 2 + l] * v[i];
        v[l] = s / dg[l];
    }
    for (int l = 0; l < L; ++l) {
        g[l] = -v[l] * invB;
        g[L + l] = (1.0f - v[l] * u[l] * dg[l]) * invB;
        for (int j = 0; j < l; ++j) g[2 * L + l * (l - 1) / 2 + j] = -v[l] * u[j] * invB;
    }
    loss[b] = tot;
}

// out[j] = sum_b M[b][j]: one 256-thread workgroup per column; thread t sums
// rows t, t + 256, ... in order, then a fixed-order tree in LDS (the result
// does not depend on scheduling).
__global__ __launch_bounds__(256) void col_sum(const float *Mx, int rows, int cols, float *out)
{
    __shared__ float part[256];
    const int j = (int)blockIdx.x, t = (int)threadIdx.x;
    float s = 0.0f;
    if (j < cols)
        for (int b = t; b < rows; b += 256) s += Mx[(int64_t)b * cols + j];
    part[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0 && j < cols) out[j] = part[0];
}

// FP32 master parameters -> the inference copy (BF16 fragments in MFMA B order:
// lane 32 h + i of fragment (ks, ct) holds W[16 ks + 8 h + j][32 ct + i]).
__global__ void pack_mlp(const float *master, MlpDev *out)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    auto pack = [&](const float *W, int K, int N, __bf16 *dst, int idx) {
        const int nct = N / 32;
        const int total = (K / 16) * nct * 64 * 8;
        if (idx >= total) return;
        const int j = idx & 7, lane = (idx >> 3) & 63, frag = idx >> 9;
        const int ks = frag / nct, ct = frag % nct;
        const int k = 16 * ks + 8 * (lane >> 5) + j, n = 32 * ct + (lane & 31);
        dst[idx] = (__bf16)W[k * N + n];
    };
    pack(master + kOffW1, kMlpF, kMlpH, out->W1p, t);
    pack(master + kOffW2, kMlpH, kMlpH, out->W2p, t);
    pack(master + kOffW3, kMlpH, kMlpO, out->W3p, t);
    if (t < kWtFrags * 64 * 8) {
        const int j = t & 7, lane = (t >> 3) & 63, frag = t >> 9;
        const int h = lane >> 5, i = lane & 31;
        float w;
        if (frag < 8) {
            const int ot = frag >> 1, ks = frag & 1;
            w = master[kOffW1 + (16 * ks + 8 * h + j) * kMlpH + 32 * ot + i];
        } else if (frag < 40) {
            const int ot = (frag - 8) >> 3, ks = (frag - 8) & 7;
            w = master[kOffW2 + wt_unit(ks, h, j) * kMlpH + 32 * ot + i];
        } else {
            const int ot = (frag - 40) >> 3, ks = (frag - 40) & 7;
            w = master[kOffW3 + wt_unit(ks, h, j) * kMlpO + 32 * ot + i];
        }
        out->Wt[t] = (__bf16)w;
    }
    if (t < kMlpF) { out->fmean[t] = master[kOffFmean + t]; out->fscale[t] = master[kOffFscale + t]; }
    if (t < kMlpH) { out->b1[t] = master[kOffB1 + t]; out->b2[t] = master[kOffB2 + t]; }
    if (t < kMlpO) out->b3[t] = master[kOffB3 + t];
    if (t < 8) { out->omean[t] = master[kOffOmean + t]; out->oscale[t] = master[kOffOscale + t]; }
}

__global__ void fill_f32(float *p, int64_t n, float v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// X[b][k] = (phi[b][k] - fmean_k) fscale_k clipped to [-kMlpClip, kMlpClip], the
// network's input standardisation.
__global__ void standardise_rows(const float *phi, const float *master, float *X, int64_t B)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * kMlpF) return;
    const int k = (int)(t % kMlpF);
    const float v = (phi[t] - master[kOffFmean + k]) * master[kOffFscale + k];
    X[t] = fminf(fmaxf(v, -kMlpClip), kMlpClip);
}

// out = mean of v[0..n): one 256-thread workgroup; thread t sums v[t],
// v[t + 256], ... in FP64 in order, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void mean_rows(const float *v, int64_t n, float *out)
{
    __shared__ double part[256];
    const int t = (int)threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < n; i += 256) s += (double)v[i];
    part[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) *out = (float)(part[0] / (double)n);
}

// Wavefronts per tile: at least four k-steps each, at most 8 (512 threads keep
// the register budget above what a group of four k-steps needs).
// *acc += sum of v[0..n): one 256-thread workgroup; thread t sums v[t],
// v[t + 256], ... in FP64 in order, then a fixed-order tree in LDS.  Training
// adds each minibatch's per-row losses to its epoch's slot on the device.
__global__ __launch_bounds__(256) void sum_rows_into(const float *v, int64_t n, double *acc)
{
    __shared__ double part[256];
    const int t = (int)threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < n; i += 256) s += (double)v[i];
    part[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) *acc += part[0];
}

static hipError_t gemm(const float *A, int lda, int tA, const float *B, int ldb, int tB, float *C, int ldc, int M,
                       int N, int K, hipStream_t st)
{
    const int tiles = (M / 32) * (N / 32);
    const int steps = K / 16;
    const dim3 grid((unsigned)tiles);
    if (steps >= 32)
        hipLaunchKernelGGL(gemm_bf16<8>, grid, dim3(512), 0, st, A, lda, tA, B, ldb, tB, C, ldc, M, N, K, 0);
    else if (steps >= 16)
        hipLaunchKernelGGL(gemm_bf16<4>, grid, dim3(256), 0, st, A, lda, tA, B, ldb, tB, C, ldc, M, N, K, 0);
    else if (steps >= 8)
        hipLaunchKernelGGL(gemm_bf16<2>, grid, dim3(128), 0, st, A, lda, tA, B, ldb, tB, C, ldc, M, N, K, 0);
    else
        hipLaunchKernelGGL(gemm_bf16<1>, grid, dim3(64), 0, st, A, lda, tA, B, ldb, tB, C, ldc, M, N, K, 0);
    return hipGetLastError();
}

hipError_t mlp_forward_backward(const float *master, const TrainBufs &t, int L, hipStream_t st)
{
    const int B = t.B;
    const float *W1 = master + kOffW1, *W2 = master + kOffW2, *W3 = master + kOffW3;
    auto ew = [&](int64_t n) { return dim3((unsigned)((n + 255) / 256)); };
    hipError_t e;
#define FBMC_TRY(expr)                          \
    do {                                        \
        if ((e = (expr)) != hipSuccess) return e; \
    } while (0)
    FBMC_TRY(gemm(t.X, kMlpF, 0, W1, kMlpH, 0, t.Z1, kMlpH, B, kMlpH, kMlpF, st));
    hipLaunchKernelGGL(bias_gelu, ew((int64_t)B * kMlpH), dim3(256), 0, st, t.Z1, master + kOffB1, t.H1, B, kMlpH, 1);
    FBMC_TRY(gemm(t.H1, kMlpH, 0, W2, kMlpH, 0, t.Z2, kMlpH, B, kMlpH, kMlpH, st));
    hipLaunchKernelGGL(bias_gelu, ew((int64_t)B * kMlpH), dim3(256), 0, st, t.Z2, master + kOffB2, t.H2, B, kMlpH, 1);
    FBMC_TRY(gemm(t.H2, kMlpH, 0, W3, kMlpO, 0, t.O, kMlpO, B, kMlpO, kMlpH, st));
    hipLaunchKernelGGL(bias_gelu, ew((int64_t)B * kMlpO), dim3(256), 0, st, t.O, master + kOffB3, (float *)nullptr, B,
                       kMlpO, 0);
    hipLaunchKernelGGL(nll_grad, ew(B), dim3(256), 0, st, t.O, kMlpO, t.Tg, L, master + kOffOmean,
                       master + kOffOscale, t.dO, t.loss, B);
    // a fill kernel, not a memset, so the sequence can be captured in a graph
    hipLaunchKernelGGL(fill_f32, ew(kMlpParams), dim3(256), 0, st, t.grad, (int64_t)kMlpParams, 0.0f);
    float *g = t.grad;
    // layer 3
    FBMC_TRY(gemm(t.H2, kMlpH, 1, t.dO, kMlpO, 0, g + kOffW3, kMlpO, kMlpH, kMlpO, B, st));
    hipLaunchKernelGGL(col_sum, dim3(kMlpO), dim3(256), 0, st, t.dO, B, kMlpO, g + kOffB3);
    FBMC_TRY(gemm(t.dO, kMlpO, 0, W3, kMlpO, 1, t.dH, kMlpH, B, kMlpH, kMlpO, st));
    hipLaunchKernelGGL(gelu_backward, ew((int64_t)B * kMlpH), dim3(256), 0, st, t.Z2, t.dH, t.dZ2, (int64_t)B * kMlpH);
    // layer 2
    FBMC_TRY(gemm(t.H1, kMlpH, 1, t.dZ2, kMlpH, 0, g + kOffW2, kMlpH, kMlpH, kMlpH, B, st));
    hipLaunchKernelGGL(col_sum, dim3(kMlpH), dim3(256), 0, st, t.dZ2, B, kMlpH, g + kOffB2);
    FBMC_TRY(gemm(t.dZ2, kMlpH, 0, W2, kMlpH, 1, t.dH, kMlpH, B, kMlpH, kMlpH, st));
    hipLaunchKernelGGL(gelu_backward, ew((int64_t)B * kMlpH), dim3(256), 0, st, t.Z1, t.dH, t.dZ1, (int64_t)B * kMlpH);
    // layer 1
    FBMC_TRY(gemm(t.X, kMlpF, 1, t.dZ1, kMlpH, 0, g + kOffW1, kMlpH, kMlpF, kMlpH, B, st));
    hipLaunchKernelGGL(col_sum, dim3(kMlpH), dim3(256), 0, st, t.dZ1, B, kMlpH, g + kOffB1);
#undef FBMC_TRY
    return hipGetLastError();
}

// Adam on FP32 master weights; p, g, m, v of length n.
__global__ void adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                          float b2, float eps, float c1, float c2)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (__builtin_sqrtf(vt / c2) + eps);
}

}  // namespace fbmc
