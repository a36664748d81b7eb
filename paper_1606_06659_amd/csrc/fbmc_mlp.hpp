// fbmc_mlp.hpp -- shapes and kernels of the learned beta proposal's network.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fbmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kMlpF = 32;    // features (zero-padded)
constexpr int kMlpH = 128;   // hidden width
constexpr float kMlpClip = 8.0f;   // standardised inputs (and training targets) clipped to +-8
constexpr int kMlpO = 64;    // outputs: 2L + L(L-1)/2 <= 44 used, padded to two 32-wide tiles

// Outputs of the network for L coefficients: mean, log-diagonal of the factor,
// its strict lower triangle (row-major).
__host__ __device__ constexpr int mlp_outputs(int L) { return 2 * L + L * (L - 1) / 2; }

// FP32 master parameters, one contiguous block (offsets in floats).
constexpr int kOffFmean = 0;
constexpr int kOffFscale = kOffFmean + kMlpF;
constexpr int kOffW1 = kOffFscale + kMlpF;                 // [F][H]
constexpr int kOffB1 = kOffW1 + kMlpF * kMlpH;
constexpr int kOffW2 = kOffB1 + kMlpH;                     // [H][H]
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;                     // [H][O]
constexpr int kOffB3 = kOffW3 + kMlpH * kMlpO;
constexpr int kOffOmean = kOffB3 + kMlpO;                  // [8]
constexpr int kOffOscale = kOffOmean + 8;
constexpr int kMlpParams = kOffOscale + 8;

// Inference copy of the weights.  W1p..W3p: BF16 MFMA B fragments
// [kstep][coltile][lane][8] of the row-major layers (training-side checks).
// Wt: the A fragments of the transposed layers out^T = W^T in^T that the sweep
// runs (one wavefront per 64 genes; the output tile of one layer is, register
// for register, the B fragments of the next), kWtFrags fragments of
// [64 lanes][8]: layer 1 at (ot, ks) -> 2 ot + ks, layer 2 -> 8 + 8 ot + ks,
// layer 3 -> 40 + 8 ot + ks.  Lane 32 h + i, element j of fragment (ot, ks)
// holds W[k][32 ot + i] with k = 16 ks + 8 h + j in layer 1 (inputs in natural
// order) and k = wt_unit(ks, h, j) in layers 2 and 3 (the order in which a
// 32 x 32 accumulator tile holds its rows).
constexpr int kWtFrags = 4 * 2 + 4 * 8 + 2 * 8;
__host__ __device__ constexpr int wt_unit(int ks, int h, int j)
{
    return 32 * (ks >> 1) + 16 * (ks & 1) + 8 * (j >> 2) + 4 * h + (j & 3);
}

struct MlpDev {
    float fmean[kMlpF], fscale[kMlpF];
    float b1[kMlpH], b2[kMlpH], b3[kMlpO];
    float omean[8], oscale[8];
    __bf16 W1p[(kMlpF / 16) * (kMlpH / 32) * 64 * 8];
    __bf16 W2p[(kMlpH / 16) * (kMlpH / 32) * 64 * 8];
    __bf16 W3p[(kMlpH / 16) * (kMlpO / 32) * 64 * 8];
    __attribute__((aligned(16))) __bf16 Wt[kWtFrags * 64 * 8];
};

// Device buffers of one forward and backward pass over B rows (B a multiple
// of 32): standardised inputs X [B][F], targets Tg [B][L], pre-activations and
// activations Z1, H1, Z2, H2 [B][H], outputs O and their gradient dO [B][O],
// backward temporaries dH, dZ2, dZ1 [B][H], per-row losses [B], and the
// gradient block grad [kMlpParams] in the master layout.
struct TrainBufs {
    float *X = nullptr, *Tg = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr;
    float *O = nullptr, *dO = nullptr, *dH = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *loss = nullptr;
    float *grad = nullptr;
    int B = 0;
};

// Enqueues the forward pass, the per-row Gaussian NLL and the backward pass of
// the batch mean on `st`; reads master, t.X and t.Tg, writes every other
// buffer of t (grad entirely: the blocks with no gradient are set to zero).
hipError_t mlp_forward_backward(const float *master, const TrainBufs &t, int L, hipStream_t st);

__global__ void mfma_probe(const float *A, const float *B, float *C);
__global__ void bias_gelu(float *Z, const float *bias, float *H, int rows, int cols, int apply_gelu);
__global__ void gelu_backward(const float *Z, const float *dH, float *dZ, int64_t n);
__global__ void nll_grad(const float *O, int Op, const float *T, int L, const float *omean,
                         const float *oscale, float *dO, float *loss, int B);
__global__ void col_sum(const float *Mx, int rows, int cols, float *out);
__global__ void pack_mlp(const float *master, MlpDev *out);
__global__ void fill_f32(float *p, int64_t n, float v);
__global__ void standardise_rows(const float *phi, const float *master, float *X, int64_t B);
__global__ void mean_rows(const float *v, int64_t n, float *out);
__global__ void sum_rows_into(const float *v, int64_t n, double *acc);
__global__ void adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                          float b2, float eps, float c1, float c2);

}  // namespace fbmc
