// Internal definitions shared by the library's HIP sources (not part of the
// C ABI).  Device-side metric primitives, the per-level threshold table and
// the device views passed to kernels by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fnn {

enum { M_L2 = 0, M_ANG = 1, M_HAM = 2, M_LEV = 3 };

// Levels l = -LOFF .. NLEV-LOFF-1 are tabulated; a distance 2^l outside this
// range cannot occur for float32 inputs.
constexpr int LOFF = 200;
constexpr int NLEV = 400;
constexpr int MAX_LEV_WORDS = 4;   // strings of up to 256 symbols
constexpr int MAX_SIGMA = 255;     // Levenshtein symbols 0..254 (0xFF pads)
constexpr int WAVE = 64;

// Error flags raised by kernels (bitmask in a device word).
enum {
    ERR_CAPACITY = 1,    // an output buffer was too small (host resizes)
    ERR_INDEX = 2,       // an index left its buffer (internal bug)
    ERR_INPUT = 4,       // NaN / Inf coordinate, zero angular row, bad symbol
    ERR_RANGE = 8,       // coordinate magnitude beyond what FP32 keys can hold
};

// Device view of a point set.  During the build the rows are in input
// order; after it, in tree order.
struct Pts {
    int metric;
    int n;
    int dim;              // coordinates (L2/ANG), bits (HAM), stride (LEV)
    int dp;               // float row stride (L2/ANG), words (HAM), bytes (LEV)
    int W;                // Levenshtein words per pattern
    int sigma;            // Levenshtein alphabet size
    const float *x;       // raw coordinates [n][dp], zero padded
    const float *xn;      // angular: unit rows [n][dp]
    const uint64_t *h;    // Hamming words [n][dp]
    const uint8_t *s;     // Levenshtein bytes [n][dp]
    const int32_t *len;   // Levenshtein lengths [n]
    const uint64_t *peq;  // Levenshtein match masks [n][sigma][W]
};

// Thresholds of the comparison "d <= tau" for tau = eps or tau = 2^l, in the
// FP32 key space of each metric: key < lo => surely within, key > hi =>
// surely not, otherwise decide with the FP64 reference predicate using p64.
struct Thr {
    float lo, hi;
    double p64;
};

struct LevelTab {
    Thr t[NLEV];
};

// Per-cloud query thresholds (a batch of independent clouds, each with its
// own eps): the exact comparison, the pruning eps as a distance, the MFMA
// filter's eps^2 in key space and the eps the cost-model features divide by.
struct CloudThr {
    Thr E;
    float peps, e2f, feps, pad_;
};

// ---------------------------------------------------------------------------
// FP32 keys.  L2: squared distance (direct differences, fused multiply-add).
// Angular: squared chord between unit vectors, 2 - 2 cos(theta).  Hamming,
// Levenshtein: the exact integer distance as a float.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float sqdiff_key(const float *__restrict__ a,
                                            const float *__restrict__ b,
                                            int dp)
{
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int k = 0; k < dp; k += 4) {
        float4 u = *reinterpret_cast<const float4 *>(a + k);
        float4 v = *reinterpret_cast<const float4 *>(b + k);
        float d0 = u.x - v.x, d1 = u.y - v.y, d2 = u.z - v.z, d3 = u.w - v.w;
        s0 = fmaf(d0, d0, s0);
        s1 = fmaf(d1, d1, s1);
        s2 = fmaf(d2, d2, s2);
        s3 = fmaf(d3, d3, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

__device__ __forceinline__ int ham_words(const uint64_t *__restrict__ a,
                                         const uint64_t *__restrict__ b,
                                         int W)
{
    int h = 0;
    for (int w = 0; w < W; ++w)
        h += __popcll(a[w] ^ b[w]);
    return h;
}

// Unit-cost edit distance by the bit-parallel dynamic programme of Myers
// (1999) in Hyyro's formulation for whole-string distance: the pattern's
// vertical deltas live in bit vectors, one text symbol is consumed per
// step, the top row's horizontal delta is always +1.  Multi-word: the
// addition carries and the shifts carry between 64-bit words.
template <int W>
__device__ inline int lev_bitpar(const uint64_t *__restrict__ peq, int m,
                                 const uint8_t *__restrict__ text, int tl)
{
    if (m == 0)
        return tl;
    if (tl == 0)
        return m;
    uint64_t pv[W], mv[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        pv[w] = ~0ull;
        mv[w] = 0ull;
    }
    const int lastw = (m - 1) >> 6;
    const uint64_t lastbit = 1ull << ((m - 1) & 63);
    int score = m;
    for (int j = 0; j < tl; ++j) {
        const uint64_t *eqv = peq + (int)text[j] * W;
        uint64_t cadd = 0ull, cph = 1ull, cmh = 0ull;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (w <= lastw) {
                uint64_t eq = eqv[w];
                uint64_t xv = eq | mv[w];
                uint64_t t = eq & pv[w];
                uint64_t s1 = t + pv[w];
                uint64_t c1 = s1 < t ? 1ull : 0ull;
                uint64_t s2 = s1 + cadd;
                uint64_t c2 = s2 < s1 ? 1ull : 0ull;
                cadd = c1 | c2;
                uint64_t xh = (s2 ^ pv[w]) | eq;
                uint64_t ph = mv[w] | ~(xh | pv[w]);
                uint64_t mh = pv[w] & xh;
                if (w == lastw) {
                    if (ph & lastbit)
                        ++score;
                    else if (mh & lastbit)
                        --score;
                }
                uint64_t phs = (ph << 1) | cph;
                uint64_t mhs = (mh << 1) | cmh;
                cph = ph >> 63;
                cmh = mh >> 63;
                pv[w] = mhs | ~(xv | phs);
                mv[w] = phs & xv;
            }
        }
    }
    return score;
}

// The same recurrence for alphabets of at most 4 symbols: the pattern's
// match masks sit in registers and the text is read four symbols per load,
// so a step waits on no memory (the per-symbol loads of lev_bitpar make a
// single distance a chain of dependent memory round trips).
template <int W>
__device__ inline int lev_bitpar4(const uint64_t *__restrict__ peq, int sigma, int m,
                                  const uint8_t *__restrict__ text, int tl)
{
    if (m == 0)
        return tl;
    if (tl == 0)
        return m;
    uint64_t eqr[4][W], pv[W], mv[W];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int w = 0; w < W; ++w)
            eqr[c][w] = c < sigma ? peq[c * W + w] : 0ull;  // the table holds sigma rows
#pragma unroll
    for (int w = 0; w < W; ++w) {
        pv[w] = ~0ull;
        mv[w] = 0ull;
    }
    const int lastw = (m - 1) >> 6;
    const uint64_t lastbit = 1ull << ((m - 1) & 63);
    int score = m;
    auto step = [&](unsigned ch) {
        uint64_t cadd = 0ull, cph = 1ull, cmh = 0ull;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (w <= lastw) {
                const uint64_t eq = ch == 0 ? eqr[0][w]
                                    : ch == 1 ? eqr[1][w]
                                    : ch == 2 ? eqr[2][w]
                                              : eqr[3][w];
                uint64_t xv = eq | mv[w];
                uint64_t t = eq & pv[w];
                uint64_t s1 = t + pv[w];
                uint64_t c1 = s1 < t ? 1ull : 0ull;
                uint64_t s2 = s1 + cadd;
                uint64_t c2 = s2 < s1 ? 1ull : 0ull;
                cadd = c1 | c2;
                uint64_t xh = (s2 ^ pv[w]) | eq;
                uint64_t ph = mv[w] | ~(xh | pv[w]);
                uint64_t mh = pv[w] & xh;
                if (w == lastw) {
                    if (ph & lastbit)
                        ++score;
                    else if (mh & lastbit)
                        --score;
                }
                uint64_t phs = (ph << 1) | cph;
                uint64_t mhs = (mh << 1) | cmh;
                cph = ph >> 63;
                cmh = mh >> 63;
                pv[w] = mhs | ~(xv | phs);
                mv[w] = phs & xv;
            }
        }
    };
    int j = 0;
    if (((uintptr_t)text & 3) == 0)
        for (; j + 4 <= tl; j += 4) {
            const unsigned wd = *(const unsigned *)(text + j);
            step(wd & 255u);
            step((wd >> 8) & 255u);
            step((wd >> 16) & 255u);
            step(wd >> 24);
        }
    for (; j < tl; ++j)
        step(text[j]);
    return score;
}

__device__ inline int lev_dispatch(const uint64_t *peq, int m,
                                   const uint8_t *text, int tl, int W, int sigma)
{
    if (sigma <= 4) {
        switch (W) {
        case 1:
            return lev_bitpar4<1>(peq, sigma, m, text, tl);
        case 2:
            return lev_bitpar4<2>(peq, sigma, m, text, tl);
        default:
            break;  // longer patterns: the general form
        }
    }
    switch (W) {
    case 1:
        return lev_bitpar<1>(peq, m, text, tl);
    case 2:
        return lev_bitpar<2>(peq, m, text, tl);
    case 3:
        return lev_bitpar<3>(peq, m, text, tl);
    default:
        return lev_bitpar<4>(peq, m, text, tl);
    }
}

// The squared difference accumulated in index order (one running sum), the order of
// the leaf tiles: an edge's FP32 distance then has the same bits whichever
// kernel decided it.
__device__ __forceinline__ float sqdiff_seq(const float *__restrict__ a,
                                            const float *__restrict__ b, int dp)
{
    float s = 0.f;
    for (int k = 0; k < dp; k += 4) {
        float4 u = *reinterpret_cast<const float4 *>(a + k);
        float4 v = *reinterpret_cast<const float4 *>(b + k);
        float d0 = u.x - v.x, d1 = u.y - v.y, d2 = u.z - v.z, d3 = u.w - v.w;
        s = fmaf(d0, d0, s);
        s = fmaf(d1, d1, s);
        s = fmaf(d2, d2, s);
        s = fmaf(d3, d3, s);
    }
    return s;
}

template <int M>
__device__ __forceinline__ float key32_seq(const Pts &P, int i, int j)
{
    if constexpr (M == M_L2)
        return sqdiff_seq(P.x + (size_t)i * P.dp, P.x + (size_t)j * P.dp, P.dp);
    else
        return sqdiff_seq(P.xn + (size_t)i * P.dp, P.xn + (size_t)j * P.dp, P.dp);
}

// FP32 key between rows i and j of P.
template <int M>
__device__ __forceinline__ float key32(const Pts &P, int i, int j)
{
    if constexpr (M == M_L2) {
        return sqdiff_key(P.x + (size_t)i * P.dp, P.x + (size_t)j * P.dp, P.dp);
    } else if constexpr (M == M_ANG) {
        return sqdiff_key(P.xn + (size_t)i * P.dp, P.xn + (size_t)j * P.dp,
                          P.dp);
    } else if constexpr (M == M_HAM) {
        return (float)ham_words(P.h + (size_t)i * P.dp, P.h + (size_t)j * P.dp,
                                P.dp);
    } else {
        return (float)lev_dispatch(P.peq + (size_t)i * P.sigma * P.W, P.len[i],
                                   P.s + (size_t)j * P.dp, P.len[j], P.W, P.sigma);
    }
}

// ---------------------------------------------------------------------------
// FP64 reference predicates (no contraction, sums in index order), used only
// for pairs whose FP32 key falls inside the rounding band of a threshold.
// ---------------------------------------------------------------------------

__device__ __noinline__ double l2_sq64(const float *a, const float *b, int d)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        s = s + t * t;
    }
    return s;
}

__device__ __noinline__ bool ang_within64(const float *a, const float *b,
                                          int d, double C)
{
#pragma clang fp contract(off)
    double g = 0.0, aa = 0.0, bb = 0.0;
    for (int k = 0; k < d; ++k) {
        double x = (double)a[k], y = (double)b[k];
        g = g + x * y;
        aa = aa + x * x;
        bb = bb + y * y;
    }
    double t = ((C * C) * aa) * bb;
    double g2 = g * g;
    if (C >= 0.0)
        return g >= 0.0 && g2 >= t;
    return g >= 0.0 || g2 <= t;
}

// Kahan's angle: 2 atan2(|xh - yh|, |xh + yh|), xh = x/|x|, in FP64.
__device__ __noinline__ double ang_dist64(const float *a, const float *b,
                                          int d)
{
#pragma clang fp contract(off)
    double aa = 0.0, bb = 0.0;
    for (int k = 0; k < d; ++k) {
        aa = aa + (double)a[k] * (double)a[k];
        bb = bb + (double)b[k] * (double)b[k];
    }
    double na = sqrt(aa), nb = sqrt(bb);
    double u = 0.0, v = 0.0;
    for (int k = 0; k < d; ++k) {
        double xh = (double)a[k] / na, yh = (double)b[k] / nb;
        double m = xh - yh, p = xh + yh;
        u = u + m * m;
        v = v + p * p;
    }
    return 2.0 * atan2(sqrt(u), sqrt(v));
}

// Exact decision "d(i, j) <= tau" given the FP32 key and the threshold.
template <int M>
__device__ __forceinline__ bool within(const Pts &P, int i, int j, float key,
                                       const Thr &T, unsigned long long *nrecheck)
{
    if constexpr (M == M_HAM || M == M_LEV) {
        return key <= T.lo;
    } else {
        if (key < T.lo)
            return true;
        if (key > T.hi)
            return false;
        if (nrecheck)
            atomicAdd(nrecheck, 1ull);
        if constexpr (M == M_L2)
            return l2_sq64(P.x + (size_t)i * P.dp, P.x + (size_t)j * P.dp,
                           P.dim) <= T.p64;
        else
            return ang_within64(P.x + (size_t)i * P.dp, P.x + (size_t)j * P.dp,
                                P.dim, T.p64);
    }
}

// Reported distance of an edge.  L2 uses sqrt of the FP32 key unless the
// dimension makes its rounding bound exceed 1e-5 (then FP64), angular always
// FP64 (its FP32 chord is not accurate enough for small angles), integer
// metrics the exact key.
template <int M>
__device__ __forceinline__ float edge_dist(const Pts &P, int i, int j,
                                           float key, bool fp64_dist)
{
    if constexpr (M == M_L2) {
        if (fp64_dist)
            return (float)sqrt(l2_sq64(P.x + (size_t)i * P.dp,
                                       P.x + (size_t)j * P.dp, P.dim));
        return sqrtf(key);
    } else if constexpr (M == M_ANG) {
        return (float)ang_dist64(P.x + (size_t)i * P.dp, P.x + (size_t)j * P.dp,
                                 P.dim);
    } else {
        return key;
    }
}

// Distance (not key) from an FP32 key, for pruning tests: a value within a
// relative 1e-5 (plus 1e-6 absolute) of the true distance.
template <int M>
__device__ __forceinline__ float key_to_dist(float key)
{
    if constexpr (M == M_L2) {
        return sqrtf(key);
    } else if constexpr (M == M_ANG) {
        float c = sqrtf(fmaxf(key, 0.f)) * 0.5f;
        return 2.f * asinf(fminf(c, 1.f));
    } else {
        return key;
    }
}

// Wave-level helpers (wave64).
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

}  // namespace fnn
