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
// the top 24 bits, (r >> 8 + 1/2) 2^-24 rounded to float.  For r >> 8 >= 2^23
// the half is lost to rounding, and the top word (r >> 8 = 2^24 - 1) would round
// to exactly 1: a slice level log u = 0 then asks for points strictly above
// log f(x0), which FP32 evaluations near the mode may never give (the draw ran
// into the shrink cap once in a few 10^10 draws).  That one value is mapped to
// the largest float below 1, so every result lies strictly inside (0, 1).
template <typename T> __device__ inline T u01(uint32_t r);
template <> __device__ inline double u01<double>(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
template <> __device__ inline float u01<float>(uint32_t r)
{
    const float u = ((float)(r >> 8) + 0.5f) * 0x1p-24f;
    return u < 1.0f ? u : 0x1.fffffep-1f;
}

// Window offset: the high 28 bits of the word (the low 4 bits give K_L); float,
// as u01<float>, strictly below 1 so x0 lies inside the window.
template <typename T> __device__ inline T uwin(uint32_t r);
template <> __device__ inline double uwin<double>(uint32_t r) { return ((double)(r >> 4) + 0.5) * 0x1p-28; }
template <> __device__ inline float uwin<float>(uint32_t r)
{
    const float u = ((float)(r >> 8) + 0.5f) * 0x1p-24f;
    return u < 1.0f ? u : 0x1.fffffep-1f;
}

__device__ inline double dlog(double x) { return ::log(x); }
__device__ inline float dlog(float x) { return ::logf(x); }
__device__ inline double dexpm1(double x) { return ::expm1(x); }
// float expm1: for |x| <= ln(2)/2 the degree-7 Taylor polynomial of e^x - 1
// (truncation below 1.4e-8 relative, under one float ulp); elsewhere e^x - 1,
// whose magnitude is then at least 0.29 so the subtraction loses no accuracy.
// Both are computed and one is selected, so a wavefront never branches here.
__device__ inline float dexpm1(float x)
{
    const float p = x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f +
                    x * (1.0f / 120.0f + x * (1.0f / 720.0f + x * (1.0f / 5040.0f)))))));
    const float e = __expf(x) - 1.0f;
    return __builtin_fabsf(x) <= 0.34657359f ? p : e;
}
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
//
// Each trip evaluates one point.  The trip is written without branches: the
// point of every phase is formed and the one of the lane's phase selected, and
// the interval, counters and phase are updated with selects, so lanes in
// different phases share one instruction stream.  Only the rare shrink
// candidates 3, 4, ... (words of further Philox blocks) branch.
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
    // shrink candidate t + 1 reads word t + 2 of the draw's stream: candidates
    // 1 and 2 words 2 and 3 of block 0, later ones words of further blocks
    const T u1 = u01<T>(r.z), u2 = u01<T>(r.w);
    for (;;) {
        T u = t == 0 ? u1 : u2;
        if (phase == 2 && t >= 2) {
            const uint32_t q = (uint32_t)t + 2u;
            if ((q >> 2) != blk) {
                blk = q >> 2;
                r = philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, (ctr.w & 0xFFFF0000u) | blk), k0, k1);
            }
            // word q & 3 of the block, chosen by selects on its two bits
            const uint32_t wlo = (q & 1u) ? r.y : r.x;
            const uint32_t whi = (q & 1u) ? r.w : r.z;
            u = u01<T>((q & 2u) ? whi : wlo);
        }
        const T xs = L + u * (R - L);
        const bool p0 = phase == 0, p1 = phase == 1, p2 = phase == 2;
        const T x = p0 ? L : (p1 ? R : xs);
        const bool in = f(x) > thr;
        // step out (phases 0 and 1)
        const bool mvl = p0 && in, mvr = p1 && in;
        L = mvl ? L - w : L;
        R = mvr ? R + w : R;
        nl += mvl ? 1 : 0;
        nr += mvr ? 1 : 0;
        const int after_left = KR > 0 ? 1 : 2;
        const int ph_left = (!in || nl == KL) ? after_left : 0;
        const int ph_right = (!in || nr == KR) ? 2 : 1;
        // shrink (phase 2)
        t += p2 ? 1 : 0;
        const bool acc = p2 && in;
        const bool rej = p2 && !in;
        R = (rej && x > x0) ? x : R;
        L = (rej && !(x > x0)) ? x : L;
        x1 = acc ? x : x1;
        const bool capped = rej && t >= cap;
        phase = p0 ? ph_left : (p1 ? ph_right : 2);
        if (acc || capped) {
            bad = capped;
            break;
        }
    }
    rec.kl = KL;
    rec.nl = nl;
    rec.nr = nr;
    rec.nc = t;
    rec.bad = bad;
    return x1;
}

// The value held by the even (odd) lane of this lane's pair (2j, 2j + 1):
// DPP quad permutations [0, 0, 2, 2] and [1, 1, 3, 3], a register move inside
// each group of four lanes instead of a round trip through the LDS crossbar.
__device__ inline uint32_t pair_even_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xA0, 0xF, 0xF, false);
}
__device__ inline uint32_t pair_odd_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xF5, 0xF, 0xF, false);
}
template <typename T> __device__ inline T pair_even(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, pair_even_u32(__builtin_bit_cast(uint32_t, v)));
    } else {
        uint2 u = __builtin_bit_cast(uint2, v);
        u.x = pair_even_u32(u.x);
        u.y = pair_even_u32(u.y);
        return __builtin_bit_cast(T, u);
    }
}
template <typename T> __device__ inline T pair_odd(T v)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, pair_odd_u32(__builtin_bit_cast(uint32_t, v)));
    } else {
        uint2 u = __builtin_bit_cast(uint2, v);
        u.x = pair_odd_u32(u.x);
        u.y = pair_odd_u32(u.y);
        return __builtin_bit_cast(T, u);
    }
}

// The same draw by a pair of lanes (2j and 2j + 1, which hold the same
// variable and the same f).  The step-out to the left (even lane) and to the
// right (odd lane) do not depend on each other and run at the same time.  In
// the shrink phase the even lane evaluates candidate t + 1 and the odd lane
// candidate t + 2 on the interval that rejecting candidate t + 1 leaves (an
// update of the interval depends only on the candidate and x0); the first
// candidate in the slice is the sequential result.  Points, decisions, the
// result and the counters are those of slice_draw; both lanes return them,
// and both must call (the mates exchange values by DPP, pair_even / pair_odd).
template <typename T, typename F>
__device__ inline T slice_draw_pair(F &f, T x0, T w, uint32_t k0, uint32_t k1, uint4 ctr, int K, int cap,
                                    DrawRec &rec)
{
    const int lane = (int)(threadIdx.x & 63);
    const bool odd = (lane & 1) != 0;
    uint4 r = philox4x32_10(ctr, k0, k1);
    const T thr = f.base(x0) + dlog(u01<T>(r.x));
    const T v = w * uwin<T>(r.y);
    const T L0 = x0 - v;
    const T R0 = L0 + w;
    const int KL = (int)(r.y & (uint32_t)K);
    const int KR = K - KL;
    // step out: the left end on the even lane, the right end on the odd lane
    const int kb = odd ? KR : KL;
    T e = odd ? R0 : L0;
    int ns = 0;
    while (ns < kb) {
        if (!(f(e) > thr)) break;
        e = odd ? e + w : e - w;
        ++ns;
    }
    T L = pair_even(e), R = pair_odd(e);
    const int nl = (int)pair_even_u32((uint32_t)ns), nr = (int)pair_odd_u32((uint32_t)ns);
    // shrink: candidates t + 1 and t + 2 read words t + 2 and t + 3 of the
    // draw's stream (t even, so both sit in one Philox block)
    T x1 = x0;
    int t = 0;
    bool bad = false;
    uint32_t blk = 0;
    for (;;) {
        const uint32_t q = (uint32_t)t + 2u;
        if ((q >> 2) != blk) {
            blk = q >> 2;
            r = philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, (ctr.w & 0xFFFF0000u) | blk), k0, k1);
        }
        const T ua = u01<T>((q & 2u) ? r.z : r.x), ub = u01<T>((q & 2u) ? r.w : r.y);
        const T xa = L + ua * (R - L);
        const bool ga = xa > x0;
        const T La = ga ? L : xa, Ra = ga ? xa : R;
        const T xb = La + ub * (Ra - La);
        const int in = f(odd ? xb : xa) > thr ? 1 : 0;
        const int in_a = (int)pair_even_u32((uint32_t)in), in_b = (int)pair_odd_u32((uint32_t)in);
        if (in_a) { x1 = xa; t += 1; break; }
        if (t + 1 >= cap) { t += 1; bad = true; break; }
        if (in_b) { x1 = xb; t += 2; break; }
        const bool gb = xb > x0;
        L = gb ? La : xb;
        R = gb ? xb : Ra;
        t += 2;
        if (t >= cap) { bad = true; break; }
    }
    rec.kl = KL;
    rec.nl = nl;
    rec.nr = nr;
    rec.nc = t;
    rec.bad = bad;
    return x1;
}

// The same draw by a whole wavefront for one scalar (hyperparameters).  One
// round of evaluations covers the reference point x0 (lane 63) and the
// step-out points L - k w (lanes 0..15) and R + k w (lanes 32..47); the first
// failure on each side ends its step-out as in the sequential algorithm.  The
// shrink candidates then come 16 per round: the chain of intervals that
// assumes every earlier candidate was rejected is known in advance (each update
// depends only on the candidate and x0), every lane runs it, lane c evaluates
// candidate c, and the first point in the slice is the sequential result.
// Points are formed by the same operations as the sequential code, so the
// result and the counters match it.  All 64 lanes must call; `words` is 20
// doubles of LDS private to the wavefront.
template <typename F>
__device__ inline double slice_draw_wave(F &f, double x0, double w, uint32_t k0, uint32_t k1, uint4 ctr,
                                         int K, int cap, DrawRec &rec, double *words)
{
    constexpr int kRound = 16;
    const int lane = (int)(threadIdx.x & 63);
    const uint4 r0 = philox4x32_10(ctr, k0, k1);
    const double lu = dlog(u01<double>(r0.x));
    const double v = w * uwin<double>(r0.y);
    const double L0 = x0 - v;
    const double R0 = L0 + w;
    const int KL = (int)(r0.y & (uint32_t)K);
    const int KR = K - KL;
    const int j = lane & 31;
    const bool left = lane < 32;
    double pt = left ? L0 : R0;
    for (int i = 0; i < j && i < 15; ++i) pt = left ? pt - w : pt + w;
    if (lane == 63) pt = x0;
    const double fv = f(pt);
    const double thr = __shfl(fv, 63, 64) + lu;
    const bool need = left ? (j < KL) : (j < KR);
    const bool in = need && (fv > thr);
    const uint64_t fail_l = __ballot(left && need && !in);
    const uint64_t fail_r = __ballot(!left && need && !in) >> 32;
    const int nl = fail_l ? __builtin_ctzll(fail_l) : KL;
    const int nr = fail_r ? __builtin_ctzll(fail_r) : KR;
    double L = L0, R = R0;
    for (int i = 0; i < nl; ++i) L = L - w;
    for (int i = 0; i < nr; ++i) R = R + w;
    double x1 = x0;
    int nc = cap;
    bool found = false;
    const int c = lane & (kRound - 1);
    for (int base = 0; base < cap && !found; base += kRound) {
        // candidates base + 1 .. base + 16 read words q = base + 2 .. base + 17
        const uint32_t b0 = (uint32_t)(base + 2) >> 2;
        if (lane < 5) {
            const uint32_t b = b0 + (uint32_t)lane;
            const uint4 rb = b == 0 ? r0
                             : philox4x32_10(make_uint4(ctr.x, ctr.y, ctr.z, (ctr.w & 0xFFFF0000u) | b), k0, k1);
            words[4 * lane + 0] = u01<double>(rb.x);
            words[4 * lane + 1] = u01<double>(rb.y);
            words[4 * lane + 2] = u01<double>(rb.z);
            words[4 * lane + 3] = u01<double>(rb.w);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int off = base + 2 - 4 * (int)b0;
        double Lc = L, Rc = R, xc = 0.0;
#pragma unroll
        for (int i = 0; i < kRound; ++i) {
            const double x = Lc + words[off + i] * (Rc - Lc);
            xc = i == c ? x : xc;
            const bool gt = x > x0;
            Rc = gt ? x : Rc;
            Lc = gt ? Lc : x;
        }
        const bool acc = base + c < cap && f(xc) > thr;
        const uint64_t hit = __ballot(lane < kRound && acc);
        if (hit) {
            const int first = __builtin_ctzll(hit);
            x1 = __shfl(xc, first, 64);
            nc = base + first + 1;
            found = true;
        } else {
            L = Lc;
            R = Rc;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    rec.kl = KL;
    rec.nl = nl;
    rec.nr = nr;
    rec.nc = found ? nc : cap;
    rec.bad = !found;
    return found ? x1 : x0;
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

// Gamma(alpha, 1) variates for the exact conjugate draws (an option: the
// gamma and inverse-gamma conditionals that Section 4.2 slice-samples are
// drawn directly).  Marsaglia and Tsang (ACM TOMS 26(3), 2000): with
// d = alpha' - 1/3 and c = (9 d)^-1/2, a standard normal x and a uniform u,
// d (1 + c x)^3 is a Gamma(alpha') variate when t = 1 + c x > 0 and
// log u < x^2/2 + d (1 - t^3 + log t^3).  For alpha < 1 the sampler runs with
// alpha' = alpha + 1 and the variate is scaled by U^(1/alpha).
// Attempt k reads the Philox block (g, kind << 24 | sub, m, chain << 16 | k):
// x from words 0 and 1 by Box-Muller, u from word 2, U from word 3.  The
// candidate becomes q / X (inverse = true) or X / q and must lie in
// (0, upper).  Returns the attempt count (1..kExactTries) with `out` set, or
// 0 when alpha <= 0 or every attempt failed (the caller then slice-samples).
// FP64 throughout, in either precision mode.
constexpr int kExactTries = 64;

__device__ inline int exact_gamma_draw(uint32_t kind, double alpha, double q, bool inverse, double upper,
                                       uint32_t k0, uint32_t k1, uint32_t g, uint32_t sub, uint32_t m,
                                       uint32_t chain, double &out)
{
    if (!(alpha > 0.0)) return 0;
    const bool boost = alpha < 1.0;
    const double ap = boost ? alpha + 1.0 : alpha;
    const double d = ap - 1.0 / 3.0;
    const double c = 1.0 / ::sqrt(9.0 * d);
    for (int k = 0; k < kExactTries; ++k) {
        const uint4 r = philox4x32_10(draw_counter(g, kind, sub, m, chain, (uint32_t)k), k0, k1);
        const double x = ::sqrt(-2.0 * ::log(u01<double>(r.x))) * ::cos(6.283185307179586 * u01<double>(r.y));
        const double t = 1.0 + c * x;
        if (!(t > 0.0)) continue;
        const double v = t * t * t;
        if (!(::log(u01<double>(r.z)) < 0.5 * x * x + d - d * v + d * ::log(v))) continue;
        double X = d * v;
        if (boost) X *= ::exp(::log(u01<double>(r.w)) / alpha);
        const double val = inverse ? q / X : X / q;
        if (!(val > 0.0) || !(val < __builtin_inf()) || !(val < upper)) continue;
        out = val;
        return k + 1;
    }
    return 0;
}

// Welford's running mean and mean of squares (Section 3.1) with weight
// inv_k = 1 / k, k = m - M_B (a product instead of two FP64 divisions).
__device__ inline void welford(double2 &mm, double x, double inv_k)
{
    mm.x += (x - mm.x) * inv_k;
    mm.y += (x * x - mm.y) * inv_k;
}

}  // namespace fbmc
