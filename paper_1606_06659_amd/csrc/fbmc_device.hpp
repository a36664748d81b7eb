// fbmc_device.hpp -- device building blocks of libfbmc (gfx950).
//
//  * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): counter-based random
//    words, so every draw is a pure function of (seed, sweep, kind, index).
//  * The univariate stepping-out slice sampler of Algorithm 2 (Appendix A), in
//    log space, written as one evaluation per loop trip: the step-out and
//    shrink phases share the trip so a wavefront's trip count is the largest
//    per-lane evaluation count of the draw, not the sum of per-phase maxima.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fbmc {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Ten Philox rounds; the key advances by the Weyl constants between rounds.
__host__ __device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return c;
}

// Counter of block j of a draw: (gene, kind << 24 | sub, sweep, chain << 16 | j).
__host__ __device__ inline uint4 draw_counter(uint32_t g, uint32_t kind, uint32_t sub, uint32_t m,
                                              uint32_t chain, uint32_t j)
{
    return make_uint4(g, (kind << 24) | sub, m, (chain << 16) | j);
}

// Uniform (0, 1) from one 32-bit word.  Double: (r + 1/2) 2^-32, exact.  Float:
// the top 24 bits, (r >> 8 + 1/2) 2^-24, exact in float and strictly inside (0, 1).
template <typename T> __device__ inline T u01(uint32_t r);
template <> __device__ inline double u01<double>(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
template <> __device__ inline float u01<float>(uint32_t r) { return ((float)(r >> 8) + 0.5f) * 0x1p-24f; }

// Window offset: the high 28 bits of the word (the low 4 bits give K_L).
template <typename T> __device__ inline T uwin(uint32_t r);
template <> __device__ inline double uwin<double>(uint32_t r) { return ((double)(r >> 4) + 0.5) * 0x1p-28; }
template <> __device__ inline float uwin<float>(uint32_t r) { return ((float)(r >> 8) + 0.5f) * 0x1p-24f; }

__device__ inline double dlog(double x) { return ::log(x); }
__device__ inline float dlog(float x) { return ::logf(x); }
__device__ inline double dexpm1(double x) { return ::expm1(x); }
__device__ inline float dexpm1(float x) { return ::expm1f(x); }
__device__ inline double dexp(double x) { return ::exp(x); }
__device__ inline float dexp(float x) { return ::expf(x); }
__device__ inline double dlog1p(double x) { return ::log1p(x); }
__device__ inline float dlog1p(float x) { return ::log1pf(x); }
__device__ inline double dabs(double x) { return ::fabs(x); }
__device__ inline float dabs(float x) { return ::fabsf(x); }
template <typename T> __device__ inline T neg_inf();
template <> __device__ inline double neg_inf<double>() { return -__builtin_inf(); }
template <> __device__ inline float neg_inf<float>() { return -__builtin_inff(); }

// What one draw did: K_L, step-outs taken to the left and right, shrink
// candidates evaluated; bad = shrink cap reached (the draw keeps x0).
struct DrawRec {
    int kl, nl, nr, nc;
    bool bad;
};

// One slice draw from x0 with width w (Algorithm 2 steps 1-6).  `f` provides
//   f.base(x0) : the reference level (0 when f returns log f(x) - log f(x0))
//   f(x)       : the value compared with base + log u
// A point x is in the slice when f(x) > f.base + log u, u ~ U(0, 1).
template <typename T, typename F>
__device__ inline T slice_draw(F &f, T x0, T w, uint32_t k0, uint32_t k1, uint4 ctr, int K,
                               int cap, DrawRec &rec)
{
    uint4 r = philox4x32_10(ctr, k0, k1);
    const T thr = f.base(x0) + dlog(u01<T>(r.x));
    const T v = w * uwin<T>(r.y);
    T L = x0 - v;
    T R = L + w;
    const int KL = (int)(r.y & (uint32_t)K);
    const int KR = K - KL;
    int nl = 0, nr = 0, t = 0;
    int phase = KL > 0 ? 0 : (KR > 0 ? 1 : 2);
    uint32_t blk = 0;
    T x1 = x0;
    bool bad = false;
    for (;;) {
        T x;
        if (phase == 0) {
            x = L;
        } else if (phase == 1) {
            x = R;
        } else {
            // shrink candidate t + 1 reads word q = t + 2 of the draw's stream
            const uint32_t q = (uint32_t)t + 2u;
            if ((q >> 2) != blk) {
                blk = q >> 2;
                r = philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, (ctr.w & 0xFFFF0000u) | blk), k0, k1);
            }
            const uint32_t s = q & 3u;
            const uint32_t word = s == 0 ? r.x : (s == 1 ? r.y : (s == 2 ? r.z : r.w));
            x = L + u01<T>(word) * (R - L);
        }
        const bool in = f(x) > thr;
        if (phase == 0) {
            if (in) { L = L - w; ++nl; }
            if (!in || nl == KL) phase = KR > 0 ? 1 : 2;
        } else if (phase == 1) {
            if (in) { R = R + w; ++nr; }
            if (!in || nr == KR) phase = 2;
        } else {
            ++t;
            if (in) { x1 = x; break; }
            if (x > x0) R = x; else L = x;
            if (t >= cap) { bad = true; break; }
        }
    }
    rec.kl = KL;
    rec.nl = nl;
    rec.nr = nr;
    rec.nc = t;
    rec.bad = bad;
    return x1;
}

// Algorithm 2 step 7: tuning of w during burn-in (m <= M_B).
template <typename T>
__device__ inline void tune_width(T &w, T &waux, T x0, T x1, int64_t m, int64_t burnin,
                                  int64_t tune_start)
{
    if (m <= burnin) {
        waux += (T)m * dabs(x1 - x0);
        if (m > tune_start) {
            const T wn = waux / ((T)0.5 * (T)m * (T)(m + 1));
            if (wn > (T)0 && wn < (T)__builtin_inf()) w = wn;
        }
    }
}

// Welford's running mean and mean of squares (Section 3.1), k = m - M_B.
__device__ inline void welford(double2 &mm, double x, double k)
{
    mm.x += (x - mm.x) / k;
    mm.y += (x * x - mm.y) / k;
}

}  // namespace fbmc
