// MFMA Gram filter for the Euclidean and angular leaf tiles.
//
// d(x,y)^2 = |x|^2 + |y|^2 - 2 x.y.  The inner products of a tile are taken
// on the matrix cores from BF16, FP16 (scaled by a power of two) or FP8
// E4M3 copies of the centred points
// (each cloud of a batch about its own mean), accumulated in FP32.  With u
// the unit roundoff of the input format, |q(x).q(y) - x.y| <= (2u + u^2)
// |x||y| (Cauchy-Schwarz), plus the
// FP32 accumulation and the rounding of the norms; all of it is below
// c1 * (|x|^2 + |y|^2).  A pair is rejected only if
//     (1 - c1)(|x|^2 + |y|^2) - 2 g~ > eps^2,
// which implies d^2 > eps^2: the filter never drops an edge.  On the GPU the
// test reads g~ - ax < ay with ax = ((1 - c1)|x|^2 - eps^2') / 2 and
// ay = (1 - c1)|y|^2 / 2; the accumulators start at -ax, so the matrix
// cores produce g~ - ax directly (the FP32 accumulation then runs over
// kq + 1 terms, which the FP32 part of c1 and the enlargement of eps^2'
// cover), and a wave compares the largest value of each lane with its ay.  A surviving
// pair is recomputed by direct FP32 difference and decided exactly like the
// plain tiles (rounding band -> FP64 reference predicate).
//
// Work decomposition: query packs are grouped GW (4) at a time (consecutive
// pack ids).  A work-group (GW waves) takes one group and a run of the union
// of its members' interaction lists; wave w holds pack GW*g+w (<= 64 rows) in
// registers, the B pack of each step is staged once in LDS and read by all
// GW waves (the narrow kernel reads its B rows itself, see k_gram_direct).
// Every unordered point pair is evaluated once: a wave skips B packs with a
// smaller id, and inside its own pack keeps only pairs whose first point
// precedes the second in tree order.  Over a single cloud whose pack pairs
// are all kept, the list is every group against every later pack, and the
// packs are full runs of 64 consecutive tree positions.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <vector>

#include <string.h>

#include "gram.h"

namespace fnn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) int i32x8;

constexpr int GP = 64;           // rows per pack (max) on the MFMA path
constexpr int GW = 4;            // packs per group = waves per work-group
constexpr int UNIT_MAX = 64;     // list entries per work unit (at most)
// two waves per SIMD: the second wave hides the first one's LDS and MFMA
// dependency stalls (one wave per SIMD with 512 registers measured 1.7x
// slower)
constexpr int GRAM_WAVES_PER_SIMD = 2;
// survivor-list slots a wave reserves per atomic on the shared count (one
// atomic per tile with survivors serialised the whole filter on that count)
constexpr int SURV_CHUNK = 512;

// ---------------------------------------------------------------- prep ---

// Centre of each point: the mean of its cloud (tree positions of a cloud are
// contiguous; one cloud: pcl null).  Every pair the filter compares lies in
// one cloud, so per-cloud centring changes none of its distances and keeps
// the quantisation margin relative to the cloud's own spread.
struct Centre {
    const float *sums;     // [clouds][dp] column sums
    const float *inv;      // [clouds] 1 / cloud size
    const int32_t *pcl;    // [n] cloud of a tree position, or null
    int dp;
    __device__ __forceinline__ int cloud(long long i) const { return pcl ? pcl[i] : 0; }
    __device__ __forceinline__ float mu(int cl, int c) const
    {
        return sums[(size_t)cl * dp + c] * inv[cl];
    }
};

// Column sums per cloud: block b takes rows [b*R, (b+1)*R); with dp below
// the block size its threads split into row phases (thread t: column
// t % dp, rows r0 + t / dp + P j), so every thread reads.  A phase flushes a
// partial sum whenever the cloud changes (clouds are contiguous).
__global__ void k_colsum(const float *__restrict__ x, int n, int dp,
                         const int32_t *__restrict__ pcl, float *__restrict__ sums)
{
    const int R = 1024;
    const int r0 = blockIdx.x * R, r1 = min(n, r0 + R);
    const int B = blockDim.x;
    const int P = dp < B ? B / dp : 1;  // row phases
    const int ph = dp < B ? (int)threadIdx.x / dp : 0;
    if (ph >= P)
        return;
    for (int c = dp < B ? (int)threadIdx.x % dp : (int)threadIdx.x; c < dp;
         c += dp < B ? dp : B) {
        if (!pcl) {
            // one cloud: four independent partial sums keep loads in flight
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
            int r = r0 + ph;
            for (; r + 3 * P < r1; r += 4 * P) {
                s0 += x[(size_t)r * dp + c];
                s1 += x[(size_t)(r + P) * dp + c];
                s2 += x[(size_t)(r + 2 * P) * dp + c];
                s3 += x[(size_t)(r + 3 * P) * dp + c];
            }
            for (; r < r1; r += P)
                s0 += x[(size_t)r * dp + c];
            if (r0 + ph < r1)
                atomicAdd(&sums[c], (s0 + s1) + (s2 + s3));
            continue;
        }
        float s = 0.f;
        int cc = r0 + ph < r1 ? pcl[r0 + ph] : 0;
        for (int r = r0 + ph; r < r1; r += P) {
            const int cl = pcl[r];
            if (cl != cc) {
                atomicAdd(&sums[(size_t)cc * dp + c], s);
                s = 0.f;
                cc = cl;
            }
            s += x[(size_t)r * dp + c];
        }
        if (r0 + ph < r1)
            atomicAdd(&sums[(size_t)cc * dp + c], s);
    }
}

// Quantised rows of x - mu (tree order) and the per-point norm term.
template <int PREC>
__global__ void k_quant(const float *__restrict__ x, int n, int dp, int kq,
                        Centre C, float scale, float one_minus_c1, void *__restrict__ q,
                        float *__restrict__ hx)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int i = blockIdx.x * wpb + threadIdx.x / WAVE; i < n;
         i += gridDim.x * wpb) {
        float ss = 0.f;
        const int cl = C.cloud(i);
        for (int k = lane; k < kq; k += WAVE) {
            float v = 0.f;
            if (k < dp) {
                v = x[(size_t)i * dp + k] - C.mu(cl, k);
                // FP16: the filter works in units scaled by a power of two
                if constexpr (PREC == FNN_PREC_FP16)
                    v *= scale;
                ss = fmaf(v, v, ss);
            }
            if constexpr (PREC == FNN_PREC_BF16) {
                ((__bf16 *)q)[(size_t)i * kq + k] = (__bf16)v;
            } else if constexpr (PREC == FNN_PREC_FP16) {
                ((_Float16 *)q)[(size_t)i * kq + k] = (_Float16)v;
            } else {
                float s = fminf(fmaxf(v * scale, -448.f), 448.f);
                unsigned w = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(s, 0.f, 0, false);
                ((uint8_t *)q)[(size_t)i * kq + k] = (uint8_t)(w & 0xFF);
            }
        }
        ss = wave_sum(ss);
        if (lane == 0)
            hx[i] = one_minus_c1 * ss;
    }
}

// ------------------------------------- leading principal coordinates ---
//
// The filter may run on z = Q^T (x - mu), Q a dp x K matrix whose columns
// approximate the K leading principal directions of the point set.  For any
// Q, |Q^T (x - y)|^2 <= rho |x - y|^2 with rho >= ||Q||_2^2, so a pair with
// d(x, y) <= eps has |z(x) - z(y)|^2 <= rho eps^2: the filter stays
// conservative with eps^2 scaled by rho (and the rounding terms below).  Q
// only decides how selective it is.  rho is the Gershgorin bound of Q^T Q
// (largest absolute row sum) evaluated in FP64.

constexpr int PCA_MAXK = 64;     // principal directions examined (at most)
constexpr int PCA_ROWS = 65536;  // covariance sample (rows, at most)

// Partial sums of (x - mu)(x - mu)^T over the sample rows j * stride; block
// b takes sample rows in chunks of 32 starting at 32 b; thread t owns an
// 8 x 8 block of the dp x dp matrix (dp <= 128).
__global__ void __launch_bounds__(256)
k_cov_partial(const float *__restrict__ x, int n, int dp, int stride, Centre C,
              double *__restrict__ part)
{
    __shared__ float xs[32][128 + 1];
    const int t = threadIdx.x;
    const int bi = t / 16, bj = t % 16;
    const bool mine = 8 * bi < dp && 8 * bj < dp;
    float acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            acc[i][j] = 0.f;
    const long long m = ((long long)n + stride - 1) / stride;
    __syncthreads();
    for (long long j0 = (long long)blockIdx.x * 32; j0 < m;
         j0 += (long long)gridDim.x * 32) {
        for (int e = t; e < 32 * dp; e += blockDim.x) {
            const int r = e / dp, c = e % dp;
            const long long j = j0 + r;
            xs[r][c] = j < m ? x[(size_t)(j * stride) * dp + c] - C.mu(C.cloud(j * stride), c)
                             : 0.f;
        }
        __syncthreads();
        if (mine) {
            for (int r = 0; r < 32; ++r) {
                float a[8], b[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    a[k] = 8 * bi + k < dp ? xs[r][8 * bi + k] : 0.f;
                    b[k] = 8 * bj + k < dp ? xs[r][8 * bj + k] : 0.f;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
            }
        }
        __syncthreads();
    }
    if (mine)
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
                const int r = 8 * bi + i, c = 8 * bj + j;
                if (r < dp && c < dp)
                    part[(size_t)blockIdx.x * dp * dp + (size_t)r * dp + c] = acc[i][j];
            }
}

// C = inv_m * (sum of the nparts partial matrices): eight partial sums per
// element keep eight loads in flight.
__global__ void k_cov_reduce(const double *__restrict__ part, int nparts, int dd,
                             double inv_m, double *__restrict__ C)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < dd;
         e += gridDim.x * blockDim.x) {
        double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int b = 0;
        for (; b + 8 <= nparts; b += 8)
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] += part[(size_t)(b + u) * dd + e];
        for (; b < nparts; ++b)
            v[0] += part[(size_t)b * dd + e];
        C[e] = (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * inv_m;
    }
}

__device__ __forceinline__ double block_sum256(double v, double *red)
{
    v = wave_sum(v);
    const int t = threadIdx.x;
    __syncthreads();
    if ((t & (WAVE - 1)) == 0)
        red[t / WAVE] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Largest v over a work-group of 256 threads (v >= 0), in every thread.
__device__ __forceinline__ float block_max256(float v, float *red)
{
    v = wave_max(v);
    const int t = threadIdx.x;
    __syncthreads();
    if ((t & (WAVE - 1)) == 0)
        red[t / WAVE] = v;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__device__ __forceinline__ double pm_one(int j, int c, int salt)
{
    unsigned h = (unsigned)j * 0x9E3779B1u ^ (unsigned)c * 0x85EBCA77u ^
                 (unsigned)salt * 0xC2B2AE3Du;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (h & 1u) ? 1.0 : -1.0;
}

// Trace of the covariance C (dp x dp, FP64), one work-group.
__global__ void __launch_bounds__(256)
k_pca_trace(const double *__restrict__ C, int dp, double *__restrict__ tr)
{
    __shared__ double red[4];
    double v = 0.0;
    for (int c = threadIdx.x; c < dp; c += 256)
        v += C[(size_t)c * dp + c];
    v = block_sum256(v, red);
    if (threadIdx.x == 0)
        *tr = v;
}

// One product of the randomized range finder: Z = C Y / trace(C), Y the
// fixed +-1 start block when null; kmax x dp outputs spread over the grid.
__global__ void __launch_bounds__(256)
k_pca_power(const double *__restrict__ C, int dp, int kmax, const double *__restrict__ tr,
            const double *__restrict__ Y, double *__restrict__ Z)
{
    const double itr = *tr > 0.0 ? 1.0 / *tr : 0.0;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < kmax * dp; e += gridDim.x * 256) {
        const int j = e / dp, c = e % dp;
        double v = 0.0;
        for (int r = 0; r < dp; ++r)
            v += C[(size_t)c * dp + r] * (Y ? Y[(size_t)j * dp + r] : pm_one(j, r, 0));
        Z[e] = v * itr;
    }
}

// Leading principal directions of the covariance C (dp x dp, FP64), one
// work-group of 256 threads, from Y = the randomized range finder's block
// (three products of C with a fixed +-1 start block, scaled by 1 / trace,
// by k_pca_power): Gram-Schmidt (two passes per column; a column that
// cancels to below 1e-6 of its norm lies numerically in the span of the
// previous ones and is replaced by a fresh +-1 vector, so the columns stay
// orthonormal to rounding).  After every 16 columns the residual variance
// trace(C) - sum q_j^T C q_j is compared with the query's scale: the first
// K with 2 (trace - captured) <= beta * t2 (or K = kfix) is written to kout
// (0 if none up to kmax).  Q is returned row-major [dp][K]; info[0] = rho
// (Gershgorin bound of Q^T Q, enlarged by 1e-12 for its own rounding),
// info[1] = captured fraction.  Y (kmax * dp doubles) is overwritten.
__global__ void __launch_bounds__(256)
k_pca(const double *__restrict__ C, int dp, int kmax, int kfix, double t2, double beta,
      const double *__restrict__ trp, double *__restrict__ Y, double *__restrict__ Q,
      int *__restrict__ kout, double *__restrict__ info)
{
    __shared__ double red[4];
    __shared__ double sdot[PCA_MAXK];
    __shared__ double grow[PCA_MAXK];
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    const double tr = *trp;
    if (!(tr > 0.0)) {
        if (t == 0) {
            *kout = 0;
            info[0] = info[1] = 0.0;
        }
        return;
    }
    double cum = 0.0;
    int K = 0;
    for (int j = 0; j < kmax; ++j) {
        double *y = Y + (size_t)j * dp;
        double nn = 0.0;
        for (int attempt = 0; attempt < 4; ++attempt) {
            double n0 = 0.0;
            for (int c = t; c < dp; c += 256)
                n0 += y[c] * y[c];
            n0 = block_sum256(n0, red);
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = wv; i < j; i += 4) {
                    double d = 0.0;
                    for (int c = lane; c < dp; c += WAVE)
                        d += Y[(size_t)i * dp + c] * y[c];
                    d = wave_sum(d);
                    if (lane == 0)
                        sdot[i] = d;
                }
                __syncthreads();
                for (int c = t; c < dp; c += 256) {
                    double v = y[c];
                    for (int i = 0; i < j; ++i)
                        v -= sdot[i] * Y[(size_t)i * dp + c];
                    y[c] = v;
                }
                __syncthreads();
            }
            nn = 0.0;
            for (int c = t; c < dp; c += 256)
                nn += y[c] * y[c];
            nn = block_sum256(nn, red);
            if (nn > 1e-12 * n0 && nn > 1e-280)
                break;
            for (int c = t; c < dp; c += 256)
                y[c] = pm_one(j, c, attempt + 1);
            __syncthreads();
            nn = 0.0;
        }
        const double inv = nn > 1e-280 ? 1.0 / sqrt(nn) : 0.0;
        for (int c = t; c < dp; c += 256)
            y[c] *= inv;
        __syncthreads();
        double cap = 0.0;
        for (int c = t; c < dp; c += 256) {
            double v = 0.0;
            for (int r = 0; r < dp; ++r)
                v += C[(size_t)c * dp + r] * y[r];
            cap += y[c] * v;
        }
        cum += block_sum256(cap, red);
        if ((j + 1) % 16 == 0 && (kfix ? j + 1 == kfix : 2.0 * (tr - cum) <= beta * t2)) {
            K = j + 1;
            break;
        }
    }
    // rho >= ||Q||_2^2: largest absolute row sum of Q^T Q
    for (int a = t; a < K; a += 256)
        grow[a] = 0.0;
    __syncthreads();
    for (int e = t; e < K * K; e += 256) {
        const int a = e / K, b = e % K;
        double g = 0.0;
        for (int c = 0; c < dp; ++c)
            g += Y[(size_t)a * dp + c] * Y[(size_t)b * dp + c];
        atomicAdd(&grow[a], fabs(g));
    }
    __syncthreads();
    for (int e = t; e < K * dp; e += 256) {
        const int c = e / K, k = e % K;
        Q[e] = Y[(size_t)k * dp + c];
    }
    if (t == 0) {
        double rho = 0.0;
        for (int a = 0; a < K; ++a)
            rho = fmax(rho, grow[a]);
        *kout = K;
        info[0] = rho * (1.0 + 1e-12);
        info[1] = cum / tr;
    }
}

// z = Q^T (x - mu) in FP64, stored as FP32 rows [n][K] (tree order).  One
// thread per row and 16 outputs at a time; Q (and mu of a single cloud)
// staged in LDS 64 coordinates at a time; each output sums its products in
// coordinate order.
constexpr int PJ_K = 16, PJ_C = 64;
__global__ void __launch_bounds__(256)
k_project(const float *__restrict__ x, int n, int dp, Centre C,
          const double *__restrict__ Q, int K, float *__restrict__ z,
          unsigned *__restrict__ zmax)
{
    __shared__ double Qs[PJ_C][PJ_K];
    __shared__ double Ms[PJ_C];
    float zm = 0.f;  // largest |z| this thread wrote
    // blocks stride over row blocks (the same trip count in every thread)
    for (long long base = (long long)blockIdx.x * blockDim.x; base < n;
         base += (long long)gridDim.x * blockDim.x) {
    const long long i = base + threadIdx.x;
    const bool row = i < n;
    const int cl = row ? C.cloud(i) : 0;
    const float *xr = x + (size_t)(row ? i : 0) * dp;
    for (int kc = 0; kc < K; kc += PJ_K) {
        double acc[PJ_K];
#pragma unroll
        for (int k = 0; k < PJ_K; ++k)
            acc[k] = 0.0;
        for (int c0 = 0; c0 < dp; c0 += PJ_C) {
            const int nc = min(PJ_C, dp - c0);
            __syncthreads();  // the previous slice is consumed
            for (int e = threadIdx.x; e < PJ_C * PJ_K; e += blockDim.x) {
                const int c = e / PJ_K, k = e % PJ_K;
                Qs[c][k] = c < nc && kc + k < K ? Q[(size_t)(c0 + c) * K + kc + k] : 0.0;
            }
            if (!C.pcl)
                for (int c = threadIdx.x; c < nc; c += blockDim.x)
                    Ms[c] = (double)C.sums[c0 + c] * (double)C.inv[0];
            __syncthreads();
            if (row) {
                for (int c = 0; c < nc; c += 4) {
                    const float4 v = *(const float4 *)(xr + c0 + c);
                    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double mu =
                            C.pcl ? (double)C.sums[(size_t)cl * dp + c0 + c + u] *
                                        (double)C.inv[cl]
                                  : Ms[c + u];
                        const double d = (double)vv[u] - mu;
#pragma unroll
                        for (int k = 0; k < PJ_K; ++k)
                            acc[k] += Qs[c + u][k] * d;
                    }
                }
            }
        }
        if (row)
#pragma unroll
            for (int k = 0; k < PJ_K; ++k)
                if (kc + k < K) {
                    const float zf = (float)acc[k];
                    z[(size_t)i * K + kc + k] = zf;
                    zm = fmaxf(zm, fabsf(zf));
                }
    }
    }
    // the largest |z| (the FP16 filter's scale), one atomic per wave
    zm = wave_max(zm);
    if (zmax && (threadIdx.x & (WAVE - 1)) == 0)
        atomicMax(zmax, __float_as_uint(zm));
}

__global__ void k_absmax(const float *__restrict__ x, int n, int dp, Centre C,
                         unsigned *__restrict__ mx)
{
    float m = 0.f;
    const int64_t tot = (int64_t)n * dp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[e] - C.mu(C.cloud(e / dp), (int)(e % dp))));
    // one atomic per wave; the grid is capped so that few waves contend
    m = wave_max(m);
    if ((threadIdx.x & (WAVE - 1)) == 0)
        atomicMax(mx, __float_as_uint(m));
}

// Sum over points of |x - mu|^2 (mu per cloud) and the largest |x - mu|.
// Thread t takes float4 t, t + T, ... of the rows' flattened coordinates
// (dp is a multiple of 4), so a wave reads 1 KB of consecutive rows per
// load; FP32 sums per thread, FP64 across the work-group (256 threads),
// one atomic per work-group (atomics on one address serialise).
__global__ void k_sqdev(const float *__restrict__ x, int n, int dp, Centre C,
                        double *__restrict__ out, unsigned *__restrict__ amax)
{
    const unsigned long long q4 = (unsigned long long)(dp >> 2);
    const unsigned long long tot = (unsigned long long)n * q4;
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    float ss = 0.f, m = 0.f;
    for (unsigned long long f = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         f < tot; f += (unsigned long long)gridDim.x * blockDim.x) {
        // 32-bit division while the flattened index fits
        const unsigned long long i = tot <= 0xFFFFFFFFull ? (unsigned)f / (unsigned)q4 : f / q4;
        const int k = 4 * (int)(f - i * q4);
        const int cl = C.cloud((long long)i);
        const float4 v = x4[f];
        const float d0 = v.x - C.mu(cl, k), d1 = v.y - C.mu(cl, k + 1),
                    d2 = v.z - C.mu(cl, k + 2), d3 = v.w - C.mu(cl, k + 3);
        ss = fmaf(d0, d0, ss);
        ss = fmaf(d1, d1, ss);
        ss = fmaf(d2, d2, ss);
        ss = fmaf(d3, d3, ss);
        m = fmaxf(m, fmaxf(fmaxf(fabsf(d0), fabsf(d1)), fmaxf(fabsf(d2), fabsf(d3))));
    }
    __shared__ double red[4];
    __shared__ float redf[4];
    const double acc = block_sum256((double)ss, red);
    m = block_max256(m, redf);
    if (threadIdx.x == 0 && acc != 0.0)
        atomicAdd(out, acc);
    if (threadIdx.x == 0 && amax)
        atomicMax(amax, __float_as_uint(m));
}

// Hamming codes as signed bytes for the integer Gram: bit b of a code
// becomes byte b, +1 if set and -1 if not.  Over K = 64 W bits the product
// of two such rows is s.t = K - 2 d_H, so d_H <= k exactly when
// s.t >= K - 2k: one integer threshold, no per-point terms.
__global__ void k_quant_ham(const uint64_t *__restrict__ h, int n, int W,
                            int8_t *__restrict__ q)
{
    const int kq = 64 * W;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
         e < (long long)n * kq; e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / kq;
        const int k = (int)(e - i * kq);
        const int bit = (int)((h[i * W + (k >> 6)] >> (k & 63)) & 1ull);
        q[e] = (int8_t)(2 * bit - 1);
    }
}

// ---------------------------------------------------- interaction lists ---

// Canonical orientation (smaller pack id first) and routing: pairs of
// ordinary packs go to the MFMA path (key = B pack, value = group), pairs
// touching an oversized pack go to the plain FP32 tiles.
__global__ void k_route(const int2 *__restrict__ inter, long long ninter,
                        const int32_t *__restrict__ q_pb,
                        const int32_t *__restrict__ q_pe, int nn, int pack,
                        uint32_t kinf, uint32_t ginf,
                        uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                        unsigned long long *__restrict__ cnt,
                        int2 *__restrict__ rest)
{
    // Pair i of the list keeps slot i of (key, val): its B pack and group,
    // or (kinf, ginf) when it goes to rest instead (both sentinels sort
    // after every real key, so the real pairs come first).  Only the rare
    // pairs with a pack larger than the tile reserve slots in rest, one
    // reservation per wave (whole waves iterate, so the ballots see every
    // lane).
    const int lane = threadIdx.x & (WAVE - 1);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const long long lim = (ninter + WAVE - 1) / WAVE * WAVE;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += (long long)gridDim.x * blockDim.x) {
        const bool valid = i < ninter;
        int a = 0, b = 0;
        bool big = false;
        if (valid) {
            const int2 p = inter[i];
            a = min(p.x, p.y);
            b = max(p.x, p.y);
            big = (q_pe[a] - q_pb[a] > pack) || (q_pe[b] - q_pb[b] > pack);
        }
        const uint64_t mb = __ballot(valid && big);
        if (mb) {
            unsigned long long ob = 0;
            if (lane == 0)
                ob = atomicAdd(&cnt[1], (unsigned long long)__popcll(mb));
            ob = __shfl(ob, 0, WAVE);
            if (valid && big)
                rest[ob + __popcll(mb & lt)] = make_int2(a, b);
        }
        if (valid) {
            key[i] = big ? kinf : (uint32_t)(b - nn);
            val[i] = big ? ginf : (uint32_t)((a - nn) / GW);
        }
    }
}

// Any pack with more than `pack` points (duplicate groups)?
__global__ void k_max_pack(const int32_t *__restrict__ pb, const int32_t *__restrict__ pe,
                           int npk, int pack, int32_t *__restrict__ big)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npk;
         i += gridDim.x * blockDim.x)
        if (pe[i] - pb[i] > pack)
            *big = 1;
}

// Packs of GP consecutive tree positions (the last one shorter) for the
// closed-form work list over a single cloud: the tree's packs hold up to GP
// points (60 on average at C2), so screening them leaves a tenth of the
// matrix slots empty, while any partition of one cloud covers every pair.
__global__ void k_uniform_packs(int n, int np, int32_t *__restrict__ pb,
                                int32_t *__restrict__ pe)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += gridDim.x * blockDim.x) {
        pb[i] = i * GP;
        pe[i] = min(i * GP + GP, n);
    }
}

// Unit table of the closed-form work list from per-run tables.  Run k
// covers B packs [k R, h_k), h_k = min((k + 1) R, npk); its units are
// U[k] .. U[k+1] - 1, unit U[k] + g pairing group g with packs
// max(k R, GW g) .. h_k - 1, and its entries start at E[k] plus the lengths
// of the run's earlier units (a closed form: the first a = min(g,
// floor(k R / GW) + 1) groups take the whole run, a later group g' takes
// h_k - GW g').
__global__ void k_dense_plan(const long long *__restrict__ U, const long long *__restrict__ E,
                             int nrun, int R, int npk, int nu, int32_t *__restrict__ ubeg,
                             int32_t *__restrict__ ug, int32_t *__restrict__ ulo)
{
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < nu;
         u += gridDim.x * blockDim.x) {
        int lo = 0, hi = nrun;  // U[lo] <= u < U[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (U[mid] <= u)
                lo = mid;
            else
                hi = mid;
        }
        const long long k = lo, g = u - U[lo];
        const long long kR = k * R, h = min((k + 1) * R, (long long)npk);
        const long long a = min(g, kR / GW + 1);
        const long long len = a * (h - kR) + (g - a) * h - GW * ((a + g - 1) * (g - a) / 2);
        ubeg[u] = (int32_t)(E[lo] + len);
        ug[u] = (int32_t)g;
        ulo[u] = (int32_t)max(kR, GW * g);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ubeg[nu] = (int32_t)E[nrun];
}

// Closed-form work list: unit u pairs group ug[u] with the consecutive B
// packs ulo[u], ulo[u] + 1, ... (entries ubeg[u] .. ubeg[u+1]); one wave
// per unit.
__global__ void k_dense_units(const int32_t *__restrict__ ubeg,
                              const int32_t *__restrict__ ug,
                              const int32_t *__restrict__ ulo, int nu,
                              int32_t *__restrict__ lg, int32_t *__restrict__ lb)
{
    const int lane = threadIdx.x & (WAVE - 1), wpb = blockDim.x / WAVE;
    for (int u = blockIdx.x * wpb + threadIdx.x / WAVE; u < nu; u += gridDim.x * wpb)
        for (int e = ubeg[u] + lane; e < ubeg[u + 1]; e += WAVE) {
            lg[e] = ug[u];
            lb[e] = ulo[u] + (e - ubeg[u]);
        }
}

// After sorting by (group, B): mark the first of each distinct pair.
__global__ void k_uniq_flags(const uint32_t *__restrict__ g,
                             const uint32_t *__restrict__ b, long long m,
                             int32_t *__restrict__ flag)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x)
        flag[i] = (i == 0 || g[i] != g[i - 1] || b[i] != b[i - 1]) ? 1 : 0;
}

__global__ void k_uniq_write(const uint32_t *__restrict__ g,
                             const uint32_t *__restrict__ b, long long m,
                             const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ pos,
                             int32_t *__restrict__ lg, int32_t *__restrict__ lb)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (long long)gridDim.x * blockDim.x)
        if (flag[i]) {
            lg[pos[i]] = (int32_t)g[i];
            lb[pos[i]] = (int32_t)b[i];
        }
}

// Work units: runs of at most RUN consecutive list entries of one group.
__global__ void k_group_first(const int32_t *__restrict__ lg, int m,
                              int32_t *__restrict__ gfirst)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += gridDim.x * blockDim.x)
        if (i == 0 || lg[i] != lg[i - 1])
            gfirst[lg[i]] = i;
}

__global__ void k_units(const int32_t *__restrict__ lg, int m, int run,
                        const int32_t *__restrict__ gfirst,
                        int32_t *__restrict__ flag)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += gridDim.x * blockDim.x)
        flag[i] = ((i - gfirst[lg[i]]) % run) == 0 ? 1 : 0;
}

__global__ void k_units_write(const int32_t *__restrict__ flag,
                              const int32_t *__restrict__ pos, int m,
                              int32_t *__restrict__ ubeg)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += gridDim.x * blockDim.x)
        if (flag[i])
            ubeg[pos[i]] = i;
}

// ------------------------------------------------------------ the tile ---

constexpr int GT = 64 * GW;      // one wave per pack of a group

template <int PREC>
struct GramCfg;
template <>
struct GramCfg<FNN_PREC_BF16> {
    static constexpr int KSTEP = 16;  // k per MFMA
    static constexpr int EB = 2;      // bytes per element
};
template <>
struct GramCfg<FNN_PREC_FP16> {
    static constexpr int KSTEP = 16;
    static constexpr int EB = 2;
};
template <>
struct GramCfg<FNN_PREC_FP8> {
    static constexpr int KSTEP = 64;
    static constexpr int EB = 1;
};
template <>
struct GramCfg<FNN_PREC_I8> {
    static constexpr int KSTEP = 32;  // code bits (one signed byte each) per MFMA
    static constexpr int EB = 1;
};

// The 16-bit formats share the operand layout of the 32 x 32 x 16 products
// (eight elements per lane); only the instruction differs.
constexpr bool is16(int prec) { return prec == FNN_PREC_BF16 || prec == FNN_PREC_FP16; }
template <int PREC>
__device__ __forceinline__ f32x16 mfma16(const int4 &a, const int4 &b, const f32x16 &c)
{
    if constexpr (PREC == FNN_PREC_FP16) {
        f16x8 x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, c, 0, 0, 0);
    } else {
        bf16x8 x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
    }
}

typedef __attribute__((ext_vector_type(4))) int i32x4;
typedef __attribute__((ext_vector_type(16))) int i32x16;

// OR of v over the wave, in every lane (DPP within rows of 16 lanes, then
// row broadcasts; no LDS round trips).
__device__ __forceinline__ unsigned wave_or_u32(unsigned v)
{
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad [1,0,3,2]
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad [2,3,0,1]
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // half mirror
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row mirror
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row bcast 15
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row bcast 31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Valid-row masks of a lane's accumulator positions: bit i is set when
// r0(i) = 32 (i / 16) + 8 ((i % 16) / 4) + i % 4 is below rl, entry rl + 4
// for rl = -4 .. 64.
struct RowMaskTable {
    unsigned m[69];
};
constexpr RowMaskTable make_rowmask()
{
    RowMaskTable t{};
    for (int k = 0; k < 69; ++k) {
        unsigned v = 0;
        for (int i = 0; i < 32; ++i) {
            const int r0 = (i >> 4) * 32 + 8 * ((i & 15) >> 2) + (i & 3);
            if (r0 < k - 4)
                v |= 1u << i;
        }
        t.m[k] = v;
    }
    return t;
}
__constant__ RowMaskTable c_rowmask = make_rowmask();

// Marks this wave's unused reserved survivor slots [cpos, cend) (-1, -1).
__device__ __forceinline__ void pad_surv(const GramArgs &G, unsigned long long cpos,
                                         unsigned long long cend)
{
    const int lane = threadIdx.x & (WAVE - 1);
    for (unsigned long long q = cpos + lane; q < cend; q += WAVE)
        if ((long long)q < G.surv_cap)
            G.surv[q] = make_int2(-1, -1);
}

// End of one 64-row x 32-column block (column block cb) of a wave's tile:
// the pairs that pass the filter (all valid pairs with their pass flag when
// validating) go to the survivor list through the wave's reserved slots
// [cpos, cend); the exact integer filter also counts degrees; npairs counts
// the screened pairs.  mx is the lane's largest accumulator (scaled) and ay
// its column term.
template <int PREC, typename V, typename ACC>
__device__ __forceinline__ void block_finish(const GramArgs &G, const ACC (&accb)[2], V ay,
                                             V mx, int cb, int na, int nb, bool self,
                                             int pa, int pb, unsigned long long &cpos,
                                             unsigned long long &cend,
                                             unsigned long long &npairs,
                                             const unsigned *rmS)
{
    const int lane = threadIdx.x & (WAVE - 1), l32 = lane & 31, hi = lane >> 5;
    const uint64_t ltmask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (cb * 32 >= nb)
        return;
    // rows r < na against columns c0 .. c0+nc-1 (r < c if self)
    if (lane == 0) {
        const long long nc = min(32, nb - cb * 32), c0 = cb * 32;
        if (!self) {
            npairs += (unsigned long long)(na * nc);
        } else {
            // sum_{c=c0}^{c0+nc-1} min(na, c)
            const long long lo = c0, hi2 = c0 + nc;  // [lo, hi2)
            const long long mid = max(lo, min(hi2, (long long)na));
            npairs += (unsigned long long)((mid - lo) * (lo + mid - 1) / 2 + (hi2 - mid) * na);
        }
    }
    // this column block may hold no survivor at all
    if (!self && !G.validate && !__any(mx >= ay))
        return;
    const int col = cb * 32 + l32;
    // Accumulator position i = 16 rb + q holds row r0(i) + 4 hi of column
    // col in every lane, r0(i) = 32 rb + 8 (q / 4) + q % 4.  Bit i of om says
    // whether that pair is valid (row < na, and row < col on a self tile:
    // r0(i) < rl, looked up per tile), bit i of pm whether it also passes.
    const int rl = (col < nb ? (self ? min(na, col) : na) : 0) - 4 * hi;
    const unsigned om = rmS[min(max(rl + 4, 0), 68)];
    // Fails as sign bits: gq < ay exactly when gq - ay is negative (integer
    // codes: no overflow; floats: x - y rounds to +0 when x == y), shifted
    // in from the top position down, one funnel shift per position.  (A
    // float tie -0 against +0 counts as a fail; the real filters keep a
    // positive slack above every true edge, so a tie is never one.)
    unsigned nm = 0;
#pragma unroll
    for (int i = 31; i >= 0; --i) {
        const int rb = i >> 4, q = i & 15;
        unsigned d;
        if constexpr (PREC == FNN_PREC_I8)
            d = (unsigned)((int)accb[rb][q] - (int)ay);
        else if constexpr (PREC == FNN_PREC_FP8)
            d = __float_as_uint(__fsub_rn(__fmul_rn(accb[rb][q], G.gscale), ay));
        else
            d = __float_as_uint(__fsub_rn((float)accb[rb][q], ay));
        nm = __builtin_amdgcn_alignbit(nm, d, 31);
    }
    const unsigned pm = ~nm & om;
    // ---- survivors: appended for the exact decision kernel ---------------
    // Emitted: the passes, or (validating) every valid pair with its pass
    // flag.  One ballot per position that some lane has set gives the pairs
    // of rows r0 (lanes 0..31) and r0 + 4 (lanes 32..63).
    const unsigned todo = G.validate ? om : pm;
    unsigned any = wave_or_u32(todo);
    int cdeg = 0;  // exact integer filter: edges of this lane's column
    while (any) {
        const int i = __ffs(any) - 1;
        any &= any - 1;
        const bool emit = (todo >> i) & 1u;
        const uint64_t m = __ballot(emit);
        const int r0 = (i >> 4) * 32 + 8 * ((i & 15) >> 2) + (i & 3);
        const int cnt = __popcll(m);
        if (cpos + (unsigned long long)cnt > cend) {
            pad_surv(G, cpos, cend);
            unsigned long long b0 = 0;
            if (lane == 0)
                b0 = atomicAdd(G.nsurv, (unsigned long long)SURV_CHUNK);
            cpos = __shfl(b0, 0, WAVE);
            cend = cpos + SURV_CHUNK;
        }
        const unsigned long long o = cpos + __popcll(m & ltmask);
        if (emit && (long long)o < G.surv_cap)
            G.surv[o] = make_int2(pa + r0 + 4 * hi,
                                  (pb + col) | (int)(((pm >> i) & 1u) << 31));
        cpos += (unsigned long long)cnt;
        if constexpr (PREC == FNN_PREC_I8) {
            if (G.degp) {
                // row degrees from the two halves of the ballot
                const int lo = __popcll(m & 0xFFFFFFFFull);
                const int hi2 = __popcll(m >> 32);
                if (lane == 0 && lo)
                    atomicAdd(&G.degp[pa + r0], lo);
                if (lane == 32 && hi2)
                    atomicAdd(&G.degp[pa + r0 + 4], hi2);
                cdeg += emit;
            }
        }
    }
    if constexpr (PREC == FNN_PREC_I8) {
        // column degrees: lanes l and l + 32 hold the two row halves
        // of column l
        cdeg += __shfl_xor(cdeg, 32, WAVE);
        if (G.degp && hi == 0 && cdeg)
            atomicAdd(&G.degp[pb + col], cdeg);
    }
}

// End of one 64 x 64 tile of a wave (both column blocks).
template <int PREC, typename V, typename ACC>
__device__ __forceinline__ void tile_finish(const GramArgs &G, const ACC (&acc)[2][2],
                                            const V (&ayc)[2], const V (&mx)[2], int na,
                                            int nb, bool self, int pa, int pb,
                                            unsigned long long &cpos,
                                            unsigned long long &cend,
                                            unsigned long long &npairs,
                                            const unsigned *rmS)
{
    if (!__any(mx[0] >= ayc[0] || mx[1] >= ayc[1]) && !self && !G.validate) {
        // no survivor: only the pair count
        if ((threadIdx.x & (WAVE - 1)) == 0) {
            const long long nc = min(64, nb);
            npairs += (unsigned long long)(na * nc);
        }
        return;
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
        block_finish<PREC>(G, acc[cb], ayc[cb], mx[cb], cb, na, nb, self, pa, pb, cpos, cend,
                           npairs, rmS);
}

__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ int vmax(int a, int b) { return max(a, b); }

template <int M, int PREC, int NKS>
__global__ void __launch_bounds__(GT, GRAM_WAVES_PER_SIMD)
k_gram(Pts P, GramArgs G, TileOut out)
{
    using C = GramCfg<PREC>;
    constexpr int KS = C::KSTEP;
    constexpr int BPE = C::EB;
    constexpr int kq = NKS * KS;               // padded k (elements)
    constexpr int nks = NKS;                   // MFMA k-steps
    constexpr int rowb = kq * BPE;             // bytes per quantised row
    constexpr int ldb = rowb + 16;             // LDS row stride (bytes)
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *Bs = smem;                  // [GP][ldb]
    // filter terms (integers on the Hamming path, where the test is exact)
    using V = typename std::conditional<PREC == FNN_PREC_I8, int, float>::type;
    using ACC = typename std::conditional<PREC == FNN_PREC_I8, i32x16, f32x16>::type;
    V *ayS = (V *)(smem + GP * ldb);           // [GP]
    V *axS = ayS + GP;                         // [GW][GP]
    __shared__ int eB[UNIT_MAX], eP[UNIT_MAX], eN[UNIT_MAX], eC[UNIT_MAX];
    __shared__ unsigned rmS[69];               // row-mask table
    for (int i = threadIdx.x; i < 69; i += GT)
        rmS[i] = c_rowmask.m[i];

    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    const int l32 = lane & 31, hi = lane >> 5;
    // products carry the FP8 scale; gscale and its inverse are powers of 2
    const float ginv = is16(PREC) ? 1.f : 1.f / G.gscale;
    unsigned long long npairs = 0;
    const uint64_t ltmask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // this wave's reserved survivor slots [cpos, cend) (wave-uniform); slots
    // it leaves unused are marked (-1, -1) for the consumers to skip
    unsigned long long cpos = 0, cend = 0;

    // XCD-aware order: the dispatcher hands consecutive work-groups to the 8
    // XCDs in turn, so physical block b runs on XCD b % 8.  The grid is a
    // multiple of 8 work-groups, all resident; XCD x takes the x-th of 8
    // contiguous slices of the unit order (units that share B tiles are
    // adjacent in that order and then meet in one XCD's L2) and its
    // work-groups stride through it.
    const int bpx = (int)gridDim.x / 8, jb = (int)blockIdx.x / 8;
    const int per = (G.nunits + 7) / 8;
    const int ub = min(G.nunits, (int)(blockIdx.x % 8) * per);
    const int ue = min(G.nunits, ub + per);
    for (int u = ub + jb; u < ue; u += bpx) {
        const int e0 = G.ubeg[u], e1 = min(G.ubeg[u + 1], e0 + UNIT_MAX);
        if (G.ubeg[u + 1] - e0 > UNIT_MAX && t == 0)
            atomicOr(out.err, ERR_INDEX);  // the list builders never do this
        const int g = G.lg[e0];
        const int a = G.nn + GW * g + w;       // this wave's pack
        // packs larger than GP (duplicate groups) are tiled by the plain path
        const bool has_a = (GW * g + w) < G.npacks && G.q_pe[a] - G.q_pb[a] <= GP;
        const int pa = has_a ? G.q_pb[a] : 0;
        const int na = has_a ? G.q_pe[a] - pa : 0;

        // ---- this wave's A rows into registers (two 32-row blocks) ------
        i32x8 Areg[2][4];                      // up to 4 k-steps of 8 dwords
        // BF16: one k-step is 16 bytes per lane (4 dwords); FP8: 32 bytes.
        // Registers hold the whole padded k range (kq <= 128 supported).
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                Areg[rb][ks] = (i32x8){0, 0, 0, 0, 0, 0, 0, 0};
        if (has_a) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const int r = rb * 32 + l32;
                if (r < na) {
                    const unsigned char *src =
                        (const unsigned char *)G.q + (size_t)(pa + r) * rowb;
                    if constexpr (is16(PREC) || PREC == FNN_PREC_I8) {
                        // k-step ks: bytes ks*32 + hi*16 .. +16 (16-bit
                        // elements ks*16 + hi*8 .. +8, or Hamming bits
                        // ks*32 + hi*16 .. +16 as bytes)
                        #pragma unroll
                        for (int ks = 0; ks < nks; ++ks) {
                            const int4 v = *(const int4 *)(src + (ks * 16 + hi * 8) * 2);
                            const int slot = ks >> 1, half = ks & 1;
                            Areg[rb][slot][half * 4 + 0] = v.x;
                            Areg[rb][slot][half * 4 + 1] = v.y;
                            Areg[rb][slot][half * 4 + 2] = v.z;
                            Areg[rb][slot][half * 4 + 3] = v.w;
                        }
                    } else {
                        #pragma unroll
                        for (int ks = 0; ks < nks; ++ks) {
                            const int4 v0 = *(const int4 *)(src + ks * 64 + hi * 32);
                            const int4 v1 = *(const int4 *)(src + ks * 64 + hi * 32 + 16);
                            Areg[rb][ks] = (i32x8){v0.x, v0.y, v0.z, v0.w,
                                                   v1.x, v1.y, v1.z, v1.w};
                        }
                    }
                }
            }
        }
        // row terms of the filter, ax = (hx - eps2') / 2, per row of this
        // wave's pack (LDS; a lane's 4 consecutive accumulator rows are one
        // aligned float4); in a batch of clouds eps2' is this pack's cloud's (packs of one
        // group may come from different clouds; pairs across clouds are
        // skipped below)
        const int ca = (G.pcl && has_a) ? G.pcl[pa] : -1;
        const float e2 = ca >= 0 ? G.ct[ca].e2f : G.e2f;
        // stored as the accumulators' start value -ax (scaled units); on
        // the Hamming path 2k - K with k = floor(eps), K = code bits, and
        // the pass test s.t + 2k - K >= 0 is exact
        for (int r = lane; r < GP; r += WAVE) {
            if constexpr (PREC == FNN_PREC_I8)
                axS[w * GP + r] = (r < na) ? 2 * (int)e2 - kq : -(1 << 29);
            else
                axS[w * GP + r] = (r < na) ? -0.5f * (G.hx[pa + r] - e2) * ginv : -FLT_MAX;
        }

        // B tiles are software-pipelined: the rows of entry e+1 are loaded
        // into registers while entry e is on the matrix cores.
        constexpr int CPR = rowb / 16;                      // 16-byte chunks per row
        constexpr int NCH = (GP * CPR + GT - 1) / GT;       // chunks per thread
        int4 pre[NCH];
        V pre_ay = PREC == FNN_PREC_I8 ? (V)(1 << 29) : (V)FLT_MAX;
        // this unit's B packs (id, first point, size, cloud) in LDS: the
        // entry loop then never waits on a chain of dependent global loads
        for (int i = t; i < e1 - e0; i += GT) {
            const int bb = G.nn + G.lb[e0 + i];
            const int pbb = G.q_pb[bb];
            eB[i] = bb;
            eP[i] = pbb;
            eN[i] = G.q_pe[bb] - pbb;
            eC[i] = G.pcl ? G.pcl[pbb] : -1;
        }
        __syncthreads();
        auto load_b = [&](int e) {
            const int pbb = eP[e - e0];
            const int nbb = eN[e - e0];
#pragma unroll
            for (int i = 0; i < NCH; ++i) {
                const int c = t + i * GT;
                const int r = c / CPR, o = (c % CPR) * 16;
                pre[i] = make_int4(0, 0, 0, 0);
                if (c < GP * CPR && r < nbb)
                    pre[i] = *(const int4 *)((const unsigned char *)G.q +
                                             (size_t)(pbb + r) * rowb + o);
            }
            if (t < GP) {
                if constexpr (PREC == FNN_PREC_I8)
                    pre_ay = (t < nbb) ? (V)0 : (V)(1 << 29);
                else
                    pre_ay = (t < nbb) ? (V)(0.5f * G.hx[pbb + t]) : (V)FLT_MAX;
            }
        };
        load_b(e0);
        for (int e = e0; e < e1; ++e) {
            const int b = eB[e - e0];
            const int pb = eP[e - e0];
            const int nb = eN[e - e0];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NCH; ++i) {
                const int c = t + i * GT;
                if (c < GP * CPR)
                    *(int4 *)(Bs + (c / CPR) * ldb + (c % CPR) * 16) = pre[i];
            }
            if (t < GP)
                ayS[t] = pre_ay;
            __syncthreads();
            if (e + 1 < e1)
                load_b(e + 1);
            if (!has_a || b < a)
                continue;                      // pair handled elsewhere
            if (ca >= 0 && (eC[e - e0] == ca) == (bool)G.cross)
                continue;  // pairs never cross clouds (a bichromatic query: always do)
            const bool self = (b == a);
            // both 32-column blocks at once: four independent accumulator
            // chains [cb][rb] per k-step.  The accumulators start at -ax (in
            // the scaled units of the products), so they end at g~ - ax.
            ACC acc[2][2];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    using V4 = typename std::conditional<PREC == FNN_PREC_I8, int4, float4>::type;
                    const V4 a4 = *reinterpret_cast<const V4 *>(
                        axS + w * GP + rb * 32 + 8 * q4 + 4 * hi);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        acc[cb][rb][4 * q4 + 0] = a4.x;
                        acc[cb][rb][4 * q4 + 1] = a4.y;
                        acc[cb][rb][4 * q4 + 2] = a4.z;
                        acc[cb][rb][4 * q4 + 3] = a4.w;
                    }
                }
            const unsigned char *brow0 = Bs + l32 * ldb;
            const unsigned char *brow1 = Bs + (32 + l32) * ldb;
            // all of this step's B fragments, read before the matrix-core
            // chain so no k-step waits on LDS
            constexpr bool B16 = is16(PREC) || PREC == FNN_PREC_I8;
            int4 bfrag[B16 ? nks : 1][2];
            if constexpr (B16) {
#pragma unroll
                for (int ks = 0; ks < nks; ++ks) {
                    const int off = (ks * 16 + hi * 8) * 2;
                    bfrag[ks][0] = *(const int4 *)(brow0 + off);
                    bfrag[ks][1] = *(const int4 *)(brow1 + off);
                }
            }
#pragma unroll
            for (int ks = 0; ks < nks; ++ks) {
                if constexpr (PREC == FNN_PREC_I8) {
                    // 16 bytes per lane and k-step, the BF16 byte layout
                    const int slot = ks >> 1, half = ks & 1;
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        i32x4 bb;
                        __builtin_memcpy(&bb, &bfrag[ks][cb], 16);
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb) {
                            const i32x4 aa = (i32x4){Areg[rb][slot][half * 4 + 0],
                                                     Areg[rb][slot][half * 4 + 1],
                                                     Areg[rb][slot][half * 4 + 2],
                                                     Areg[rb][slot][half * 4 + 3]};
                            acc[cb][rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                aa, bb, acc[cb][rb], 0, 0, 0);
                        }
                    }
                } else if constexpr (is16(PREC)) {
                    const int4 bv[2] = {bfrag[ks][0], bfrag[ks][1]};
                    const int slot = ks >> 1, half = ks & 1;
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb) {
                            const int4 av = make_int4(Areg[rb][slot][half * 4 + 0],
                                                      Areg[rb][slot][half * 4 + 1],
                                                      Areg[rb][slot][half * 4 + 2],
                                                      Areg[rb][slot][half * 4 + 3]);
                            acc[cb][rb] = mfma16<PREC>(av, bv[cb], acc[cb][rb]);
                        }
                    }
                } else {
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        const unsigned char *brow = cb ? brow1 : brow0;
                        const int4 b0 = *(const int4 *)(brow + ks * 64 + hi * 32);
                        const int4 b1 = *(const int4 *)(brow + ks * 64 + hi * 32 + 16);
                        const i32x8 bb = (i32x8){b0.x, b0.y, b0.z, b0.w,
                                                 b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb)
                            acc[cb][rb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                Areg[rb][ks], bb, acc[cb][rb], 0, 0, 0, 127, 0, 127);
                    }
                }
            }
            // ---- filter ---------------------------------------------------
            // A pair passes when g~ - ax >= ay.  Fast test per lane: the
            // largest g~ - ax over its 32 rows against its column's ay, for
            // both column blocks (rows past na carry ax = FLT_MAX, columns
            // past nb carry ay = FLT_MAX, so neither can pass).  Only when
            // some lane may hold a survivor (rare), on a self pair, or when
            // validating does the wave build per-pair masks.
            V ayc[2], mx[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                ayc[cb] = ayS[cb * 32 + l32];
                mx[cb] = acc[cb][0][0];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        mx[cb] = vmax(mx[cb], acc[cb][rb][q]);
                if constexpr (PREC == FNN_PREC_FP8)
                    mx[cb] *= G.gscale;
            }
            tile_finish<PREC>(G, acc, ayc, mx, na, nb, self, pa, pb, cpos, cend, npairs, rmS);
        }
        __syncthreads();
    }
    pad_surv(G, cpos, cend);
    if (lane == 0 && npairs)
        atomicAdd(&out.cnt[2], npairs);
}

// The first active lane's value (here always lane 0: called with every lane
// active), held in scalar registers.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

constexpr int SURV_BUF = 256;  // survivors buffered per wave in LDS
// Fourth word of a raw buffer resource on gfx9-family GPUs (32-bit data,
// no swizzle; loads past the record count return zero)
constexpr int BUF_RSRC_W3 = 0x00020000;

// Appends a wave's n buffered survivors to the list: one atomic for their
// slots, then coalesced stores.  Called with every lane of the wave active.
__device__ __forceinline__ void surv_flush(const GramArgs &G, const int2 *sb, unsigned n)
{
    const int lane = threadIdx.x & (WAVE - 1);
    // LDS writes of other lanes are read below: keep them in order
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long b0 = 0;
    if (lane == 0 && n)
        b0 = atomicAdd(G.nsurv, (unsigned long long)n);
    b0 = uniform_u64(b0);
    for (unsigned i = lane; i < n; i += WAVE) {
        const unsigned long long q = b0 + i;
        if ((long long)q < G.surv_cap)
            G.surv[q] = sb[i];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// End of one 32-row x 64-column block of the narrow kernel: rows
// 32 rb + r (r < 32) of the wave's pack against the entry's columns c < 64.
// Position q of acc[cb] in a lane holds row 32 rb + 8 (q / 4) + q % 4 + 4 hi
// of column 32 cb + l32; acc[cb] starts at -ax of its row, ay[cb] is the
// lane's column term (FLT_MAX past nb) and hm[cb] the lanes whose largest
// sum of that block reaches it; ba is the B pack's index minus the A
// pack's (0: a self block).  The pairs that pass go to the wave's LDS
// buffer sb (*fill entries held), which goes to the list when it would
// overflow.  Blocks of two different packs (not validating) take one ballot
// per row position and write each position's pairs row first; self blocks
// and validation (every valid pair with its pass flag) build per-lane pass
// and validity masks and write each lane's pairs column first, next to
// each other; more pairs than the buffer holds (only when validating) go to
// the list directly.
__device__ __forceinline__ void half_finish(const GramArgs &G, const f32x16 (&acc)[2],
                                            const float (&ay)[2], const uint64_t (&hm)[2],
                                            int rb, int na, int nb, int ba, int pa,
                                            int pb, unsigned *fillS, int2 *sb,
                                            const unsigned *rmS)
{
    const int lane = threadIdx.x & (WAVE - 1), l32 = lane & 31, hi = lane >> 5;
    // keep the entry-dependent row and column arithmetic here: without this
    // the compiler computes it ahead of the vote, on every half
    asm volatile("" : "+v"(na), "+v"(nb), "+v"(pa), "+v"(pb));
    const bool self = ba == 0;
    unsigned fill = (unsigned)__builtin_amdgcn_readfirstlane((int)*fillS);
    const uint64_t ltmask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (!G.validate && !self) {
        // Two different packs: rows past na start at -FLT_MAX and columns
        // past nb carry the term FLT_MAX, so every pair that reaches its
        // column term is valid.  One ballot per row position; the lanes of
        // a position write their pairs row first (the lanes of one half
        // share the row), next to each other.
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            if (hm[cb] == 0)
                continue;
            const int colp = (pb + cb * 32 + l32) | (int)0x80000000u;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const bool ps = acc[cb][q] >= ay[cb];
                const uint64_t m = __ballot(ps);
                if (m == 0)
                    continue;
                const unsigned cnt = (unsigned)__popcll(m);
                if (fill + cnt > (unsigned)SURV_BUF) {
                    surv_flush(G, sb, fill);
                    fill = 0;
                }
                if (ps)
                    sb[fill + (unsigned)__popcll(m & ltmask)] =
                        make_int2(pa + 32 * rb + 8 * (q >> 2) + (q & 3) + 4 * hi, colp);
                fill += cnt;
            }
        }
        if (lane == 0)
            *fillS = fill;
        return;
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        if (!G.validate && hm[cb] == 0)
            continue;  // no lane reaches its column term in this block
        // valid rows of column col: below rl (na, or min(na, col) on a
        // self pair; none past nb), counted from this lane's first row
        // 32 rb + 4 hi; the low 16 bits of table entry rl + 4 mark the
        // positions q whose row offset 8 (q / 4) + q % 4 is below rl
        const int col = cb * 32 + l32;
        const int rl = (col < nb ? (self ? min(na, col) : na) : 0) - 32 * rb - 4 * hi;
        const unsigned om = rmS[min(max(rl + 4, 0), 68)] & 0xFFFFu;
        // fails as sign bits of acc - ay (see block_finish), top position
        // first
        unsigned nm = 0;
#pragma unroll
        for (int q = 15; q >= 0; --q)
            nm = __builtin_amdgcn_alignbit(
                nm, __float_as_uint(__fsub_rn(acc[cb][q], ay[cb])), 31);
        const unsigned pm = ~nm & om;
        unsigned todo = G.validate ? om : pm;
        // the lane's count (at most 16: five bits), its exclusive prefix
        // over the wave and the wave's total, from one ballot per bit
        const unsigned c = __popc(todo);
        unsigned pre = 0, tot = 0;
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const uint64_t m = __ballot((c >> b) & 1u);
            pre += (unsigned)__popcll(m & ltmask) << b;
            tot += (unsigned)__popcll(m) << b;
        }
        if (tot == 0)
            continue;
        if (fill + tot > (unsigned)SURV_BUF) {
            surv_flush(G, sb, fill);
            fill = 0;
        }
        const int colp = pb + col;
        if (tot > (unsigned)SURV_BUF) {
            // straight to the list (validation only)
            unsigned long long b0 = 0;
            if (lane == 0)
                b0 = atomicAdd(G.nsurv, (unsigned long long)tot);
            unsigned long long o = uniform_u64(b0) + pre;
            while (todo) {
                const int q = __ffs(todo) - 1;
                todo &= todo - 1;
                const int r = 32 * rb + 8 * (q >> 2) + (q & 3) + 4 * hi;
                if ((long long)o < G.surv_cap)
                    G.surv[o] = make_int2(colp, (pa + r) | (int)(((pm >> q) & 1u) << 31));
                ++o;
            }
            continue;
        }
        unsigned o = fill + pre;
        while (todo) {
            const int q = __ffs(todo) - 1;
            todo &= todo - 1;
            const int r = 32 * rb + 8 * (q >> 2) + (q & 3) + 4 * hi;
            sb[o++] = make_int2(colp, (pa + r) | (int)(((pm >> q) & 1u) << 31));
        }
        fill += tot;
    }
    if (lane == 0)
        *fillS = fill;
}

// Filter for narrow 16-bit rows (kq <= 32: the leading principal
// coordinates).  Same work units as k_gram, but no LDS staging and no
// barrier in the entry loop: each wave reads its B fragments (16 bytes per
// lane, k-step and column block) from the per-pack copies into registers
// two entries ahead, and takes an entry as two 32-row halves, each against
// both 32-column blocks.  A wave that emits survivors then never holds up
// the other waves of its work-group; the four waves of a group read the
// same B rows at about the same time, so most of those reads hit L1.
template <int M, int PREC, int NKS>
__global__ void __launch_bounds__(GT, 4)  // waves / SIMD that fit unspilled
k_gram_direct(Pts P, GramArgs G, TileOut out)
{
    static_assert(NKS >= 1 && NKS <= 2, "narrow rows only");
    constexpr int rowb = NKS * 32;  // bytes per quantised row
    __shared__ int eB[UNIT_MAX], eP[UNIT_MAX], eN[UNIT_MAX], eC[UNIT_MAX];
    __shared__ __align__(16) float axS[GW][GP];  // accumulator start -ax per row
    __shared__ unsigned rmS[69];                 // row-mask table
    for (int i = threadIdx.x; i < 69; i += GT)
        rmS[i] = c_rowmask.m[i];
    const int t = threadIdx.x, lane = t & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(t / WAVE);  // wave-uniform
    const bool uloop = G.upk && !G.validate;  // the uniform-pack entry loop
    const int l32 = lane & 31, hi = lane >> 5;
    const unsigned char *Q = (const unsigned char *)G.q;
    __shared__ unsigned fillS[GW];                     // each wave's buffered survivors
    __shared__ __align__(16) int2 survS[GW][SURV_BUF];  // and the buffer
    if (lane == 0)
        fillS[w] = 0u;
    // XCD slices of the unit order, as in k_gram
    const int bpx = (int)gridDim.x / 8, jb = (int)blockIdx.x / 8;
    const int per = (G.nunits + 7) / 8;
    const int ub = min(G.nunits, (int)(blockIdx.x % 8) * per);
    const int ue = min(G.nunits, ub + per);
    for (int u = ub + jb; u < ue; u += bpx) {
        const int e0 = G.ubeg[u], e1 = min(G.ubeg[u + 1], e0 + UNIT_MAX);
        if (G.ubeg[u + 1] - e0 > UNIT_MAX && t == 0)
            atomicOr(out.err, ERR_INDEX);  // the list builders never do this
        const int g = G.lg[e0];
        const int a = G.nn + GW * g + w;
        const bool has_a = (GW * g + w) < G.npacks && G.q_pe[a] - G.q_pb[a] <= GP;
        const int pa = has_a ? G.q_pb[a] : 0;
        const int na = has_a ? G.q_pe[a] - pa : 0;
        // uniform packs: entry e of the unit is B pack ub0 + e - e0
        const int ub0 = uloop ? __builtin_amdgcn_readfirstlane(G.lb[e0]) : 0;
        // A fragments: rows 32 rb + l32, bytes 32 ks + 16 hi
        int4 Af[2][NKS];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const int r = rb * 32 + l32;
                int4 v = make_int4(0, 0, 0, 0);
                if (r < na)
                    v = *(const int4 *)(Q + (size_t)(pa + r) * rowb + ks * 32 + hi * 16);
                Af[rb][ks] = v;
            }
        // accumulator start values -ax of the wave's rows, through LDS: each
        // row half's 16 per lane are the addend of both of its products
        const int ca = (G.pcl && has_a) ? G.pcl[pa] : -1;
        const float e2 = ca >= 0 ? G.ct[ca].e2f : G.e2f;
        for (int r = lane; r < GP; r += WAVE)
            axS[w][r] = r < na ? -0.5f * (G.hx[pa + r] - e2) : -FLT_MAX;
        // (the uniform-pack loop derives the entries' fields from their index)
        for (int i = uloop ? e1 - e0 : t; i < e1 - e0; i += GT) {
            const int bb = G.nn + G.lb[e0 + i];
            const int pbb = G.q_pb[bb];
            eB[i] = bb;
            eP[i] = pbb;
            eN[i] = G.q_pe[bb] - pbb;
            eC[i] = G.pcl ? G.pcl[pbb] : -1;
        }
        __syncthreads();
        // lane (l32, hi) of row half rb takes rows 32 rb + 8 (q / 4) + 4 hi +
        // q % 4, the layout of the accumulators it starts.  With one k-step
        // they stay in registers for the whole unit; with two, the second
        // step's fragments take those registers and each half re-reads them
        auto load_sv = [&](int rb) {
            f32x16 v;
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const float4 a4 = *reinterpret_cast<const float4 *>(
                    &axS[w][rb * 32 + 8 * q4 + 4 * hi]);
                v[4 * q4 + 0] = a4.x;
                v[4 * q4 + 1] = a4.y;
                v[4 * q4 + 2] = a4.z;
                v[4 * q4 + 3] = a4.w;
            }
            return v;
        };
        f32x16 svr[2];
        if constexpr (NKS == 1) {
            svr[0] = load_sv(0);
            svr[1] = load_sv(1);
        }
        // B fragments and column norms of one entry (columns 32 cb + l32), in
        // two register sets: entry e uses set e % 2, whose load was issued
        // two entries earlier (no copy of a register with a load in flight)
        int4 BA[2][NKS], BB[2][NKS];
        float ayA[2], ayB[2];
        // B side from the per-pack copies: pack k's 64 rows (zero past the
        // pack) and column terms (FLT_MAX past the pack) at a scalar base,
        // so every lane loads at a fixed offset and an entry costs no vector
        // arithmetic; the loads of one entry are a fixed count, so the next
        // entry's stay in flight while this one computes.
        // record counts in bytes, below 2^32 (gram_pad_packs checks), as
        // the resource's unsigned 32-bit word
        const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<void *>(G.qp), (short)0,
            (int)(unsigned)((unsigned long long)G.npacks * GP * rowb), BUF_RSRC_W3);
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(G.ayp), (short)0,
            (int)(unsigned)((unsigned long long)G.npacks * GP * 4), BUF_RSRC_W3);
        // Entry loops: with uniform packs and no validation (U) entry e is B
        // pack ub0 + e - e0 and the loop starts at the wave's own pack (no B
        // pack before it, no other cloud), so an entry needs no field reads
        // and no tests; otherwise the fields come from LDS and each entry is
        // tested.
        auto load_b = [&](auto uc, int e, int4 (&B)[2][NKS], float (&ay)[2]) __attribute__((always_inline)) {
            constexpr bool U = decltype(uc)::value;
            // buffer loads: the pack's offset in a scalar register, the
            // lane's offset fixed (32 bits: gram_pad_packs checks that the
            // copies fit), so an entry costs no vector arithmetic
            unsigned pk;
            if constexpr (U)
                pk = (unsigned)(ub0 + (e - e0));
            else
                pk = (unsigned)(__builtin_amdgcn_readfirstlane(eB[e - e0]) - G.nn);
            const int sq = (int)(pk * (unsigned)(GP * rowb)), sa = (int)(pk * (unsigned)(GP * 4));
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int c = cb * 32 + l32;
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks)
                    B[cb][ks] = __builtin_bit_cast(
                        int4, __builtin_amdgcn_raw_buffer_load_b128(rq, c * rowb + ks * 32 + hi * 16,
                                                                    sq, 0));
                // used (and waited for) only when processed
                ay[cb] = __builtin_bit_cast(float,
                                            __builtin_amdgcn_raw_buffer_load_b32(ra, c * 4, sa, 0));
            }
        };
        auto step = [&](auto uc, int e, int4 (&B)[2][NKS], float (&ay)[2]) __attribute__((always_inline)) {
            constexpr bool U = decltype(uc)::value;
            // the entry's fields are the same in every lane
            int b, pb, nb;
            bool skip;
            if constexpr (U) {
                b = ub0 + (e - e0);
                pb = b * GP;
                nb = min(GP, G.upk - pb);
                skip = false;
            } else {
                b = __builtin_amdgcn_readfirstlane(eB[e - e0]);
                pb = __builtin_amdgcn_readfirstlane(eP[e - e0]);
                nb = __builtin_amdgcn_readfirstlane(eN[e - e0]);
                const int cb_cl = __builtin_amdgcn_readfirstlane(eC[e - e0]);
                skip = !has_a || b < a || (ca >= 0 && (cb_cl == ca) == (bool)G.cross);
            }
            if (!skip) {
                const float ayc[2] = {ay[0], ay[1]};
                // one 32-row half at a time against both column blocks: the
                // half's 16 start values feed both products.  Rows past na
                // start at -FLT_MAX and columns past nb have the column term
                // FLT_MAX, so a partial pack needs no branch: its missing
                // pairs never pass
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    f32x16 acc[2], sv;
                    if constexpr (NKS == 1) {
                        sv = svr[rb];
                    } else {
                        asm volatile("" ::: "memory");  // re-read (no registers held)
                        sv = load_sv(rb);
                    }
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int ks = 0; ks < NKS; ++ks) {
                            acc[cb] = mfma16<PREC>(Af[rb][ks], B[cb][ks],
                                                   ks == 0 ? sv : acc[cb]);
                        }
                    // fast test: the lanes whose largest sum of a column
                    // block reaches their column term, one vote for the
                    // whole half
                    uint64_t hm[2];
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        float mx = -FLT_MAX;
#pragma unroll
                        for (int q = 0; q < 16; ++q)
                            mx = fmaxf(mx, acc[cb][q]);
                        hm[cb] = __ballot(mx >= ayc[cb]);
                    }
                    if ((hm[0] | hm[1]) != 0 || (!U && G.validate))
                        half_finish(G, acc, ayc, hm, rb, na, nb, b - a, pa, pb, &fillS[w], survS[w],
                                    rmS);
                }
            }
            // issued on every path (past the end: the last entry again),
            // so the count of loads in flight never depends on the branch
            load_b(uc, min(e + 2, e1 - 1), B, ay);
        };
        auto run = [&](auto uc, int es) __attribute__((always_inline)) {
            load_b(uc, es, BA, ayA);
            // one entry's loads after the other's: the loop's waits count
            // them in this order
            asm volatile("" ::: "memory");
            load_b(uc, min(es + 1, e1 - 1), BB, ayB);
            for (int e = es; e < e1; e += 2) {
                step(uc, e, BA, ayA);
                if (e + 1 < e1)
                    step(uc, e + 1, BB, ayB);
                else
                    load_b(uc, e1 - 1, BB, ayB);  // same loads in flight on both paths
            }
        };
        if (uloop) {
            // entries before the wave's own pack pair it with earlier packs
            const int es = has_a ? e0 + max(0, a - ub0) : e1;
            if (es < e1)
                run(std::true_type{}, es);
        } else {
            run(std::false_type{}, e0);
        }
        __syncthreads();  // eB.. are rewritten by the next unit
    }
    surv_flush(G, survS[w], (unsigned)__builtin_amdgcn_readfirstlane((int)fillS[w]));
}

// Pairs the narrow kernel screens (its entry loop does not count them): for
// every list entry (group g, pack B) and every pack A = 4 g + w of the group
// that the kernel does not skip, na nb pairs (na (na - 1) / 2 when A = B).
__global__ void k_gram_pairs(GramArgs G, TileOut out)
{
    unsigned long long sum = 0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < G.nlist;
         e += (long long)gridDim.x * blockDim.x) {
        const int g = G.lg[e];
        const int b = G.nn + G.lb[e];
        const int pbb = G.q_pb[b];
        const long long nb = G.q_pe[b] - pbb;
        const int cb_cl = G.pcl ? G.pcl[pbb] : -1;
        for (int w = 0; w < GW; ++w) {
            const int a = G.nn + GW * g + w;
            if ((GW * g + w) >= G.npacks)
                break;
            const long long na = G.q_pe[a] - G.q_pb[a];
            if (na > GP || b < a)
                continue;
            const int ca = G.pcl ? G.pcl[G.q_pb[a]] : -1;
            if (ca >= 0 && (cb_cl == ca) == (bool)G.cross)
                continue;
            sum += b == a ? (unsigned long long)(na * (na - 1) / 2)
                          : (unsigned long long)(na * nb);
        }
    }
    sum = wave_sum(sum);
    if ((threadIdx.x & (WAVE - 1)) == 0 && sum)
        atomicAdd(&out.cnt[2], sum);
}

// FP32 key of every lane's pair (pi, pj), summed exactly as sqdiff_seq sums
// it (one FMA per coordinate, coordinates in index order, zero padding
// adding nothing), so the distances equal the FP32 tiles' bit for bit.  The
// wave stages its 64 pairs' rows through LDS 32 coordinates at a time:
// each load instruction then reads 128-byte row segments of 8 rows instead
// of 64 scattered lines, and the next segment is in flight while this one
// is summed.  sA, sB: the wave's LDS rows (64 x SV_LDR floats each).
constexpr int SV_CH = 32;            // coordinates per staged segment
constexpr int SV_LDR = SV_CH + 4;    // floats per staged row (bank spread)
constexpr int SV_F = SV_CH / 4;      // float4 per row segment
template <int M>
__device__ __forceinline__ float key32_staged(const Pts &P, int pi, int pj, float *sA,
                                              float *sB)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const float *X = M == M_L2 ? P.x : P.xn;
    const int dp = P.dp, p4 = 4 * (lane % SV_F);
    // this lane stages float4 p4 / 4 of the rows of pairs lane / F + 16 j
    const float *ra[SV_F], *rbp[SV_F];
    int so[SV_F];
#pragma unroll
    for (int j = 0; j < SV_F; ++j) {
        const int r = lane / SV_F + (WAVE / SV_F) * j;
        ra[j] = X + (size_t)__shfl(pi, r, WAVE) * dp + p4;
        rbp[j] = X + (size_t)__shfl(pj, r, WAVE) * dp + p4;
        so[j] = r * SV_LDR + p4;
    }
    float4 va[SV_F], vb[SV_F];
    auto fetch = [&](int c0) {
        const bool in = c0 + p4 < dp;
#pragma unroll
        for (int j = 0; j < SV_F; ++j) {
            va[j] = in ? *(const float4 *)(ra[j] + c0) : make_float4(0.f, 0.f, 0.f, 0.f);
            vb[j] = in ? *(const float4 *)(rbp[j] + c0) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    fetch(0);
    float s = 0.f;
    for (int c0 = 0; c0 < dp; c0 += SV_CH) {
#pragma unroll
        for (int j = 0; j < SV_F; ++j) {
            *(float4 *)(sA + so[j]) = va[j];
            *(float4 *)(sB + so[j]) = vb[j];
        }
        if (c0 + SV_CH < dp)
            fetch(c0 + SV_CH);
        // one wave's LDS accesses complete in order: only the compiler must
        // keep the reads after the writes (and the next writes after them)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int k = 0; k < SV_CH; k += 4) {
            const float4 u = *(const float4 *)(sA + lane * SV_LDR + k);
            const float4 v = *(const float4 *)(sB + lane * SV_LDR + k);
            const float d0 = u.x - v.x, d1 = u.y - v.y, d2 = u.z - v.z, d3 = u.w - v.w;
            s = fmaf(d0, d0, s);
            s = fmaf(d1, d1, s);
            s = fmaf(d2, d2, s);
            s = fmaf(d3, d3, s);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    return s;
}

// Counter value of `key` per lane (key < 0: none): one atomic add per run of
// equal keys among the wave's active lanes (lanes with key < 0 in between do
// not end a run), and the lanes of a run take consecutive values from its
// start.  The filters write a row's survivors within a column block next to
// each other, so runs are the common case.  Called by every lane of the wave
// that is still in its loop; returns the lane's value where key >= 0 (a
// CSR slot for row cursors, a rank in the row for degree counters).
template <class T>
__device__ __forceinline__ T claim_run(T *ctr, int key)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const bool act = key >= 0;
    const uint64_t A = __ballot(act);
    const uint64_t below = A & ((1ull << lane) - 1);  // lane < 64: no overflow
    const int p = below ? 63 - __builtin_clzll(below) : lane;
    const int pk = __shfl(key, p, WAVE);  // key of the previous active lane
    const bool cont = act && below != 0 && pk == key;
    const uint64_t Hd = A & ~__ballot(cont);  // run heads
    const uint64_t upto = lane == WAVE - 1 ? ~0ull : ((2ull << lane) - 1);
    const uint64_t hb = Hd & upto;
    const int h = hb ? 63 - __builtin_clzll(hb) : 0;
    const uint64_t from_h = ~((1ull << h) - 1);
    T base = 0;
    if (act && h == lane) {
        const uint64_t nxt = Hd & ~upto;  // next head above
        const uint64_t run = nxt ? (nxt & (0 - nxt)) - 1 : ~0ull;
        base = atomicAdd(&ctr[key], (T)__popcll(A & from_h & run));
    }
    const T off = (T)(__popcll(A & from_h & upto) - 1);
    if constexpr (sizeof(T) == 8) {
        const unsigned blo = __shfl((unsigned)base, h, WAVE);
        const unsigned bhi = __shfl((unsigned)((unsigned long long)base >> 32), h, WAVE);
        return (T)(((unsigned long long)bhi << 32) | blo) + off;
    } else {
        return __shfl(base, h, WAVE) + off;
    }
}

// Exact decision of every survivor: direct-difference FP32 key, FP64 inside
// the rounding band; survivor i's edge (input ids, distance) goes to slot i
// of an unordered list, (-1, -1) when it is none, and to the row degrees.
// A grid of resident work-groups strides over the list.
template <int M>
__global__ void __launch_bounds__(256)
k_survive(Pts P, GramArgs G, long long ns, int2 *__restrict__ edges,
          float *__restrict__ edist, TileOut out)
{
    const int lane = threadIdx.x & (WAVE - 1);
    unsigned long long nrc = 0, npass = 0, nmis = 0;
    unsigned maxerr = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    // the loop runs a whole number of waves so that ballots see every lane
    const long long lim = (ns + WAVE - 1) / WAVE * WAVE;
    __shared__ __align__(16) float sAB[M == M_HAM ? 1 : 2 * 4 * WAVE * SV_LDR];
    float *sA = sAB + (M == M_HAM ? 0 : (threadIdx.x / WAVE) * 2 * WAVE * SV_LDR);
    float *sB = sA + WAVE * SV_LDR;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += stride) {
        bool edge = false;
        float dd = 0.f;
        int oi = 0, oj = 0;
        int2 rk = make_int2(0, 0);   // the edge's ranks in its two rows
        int2 e = make_int2(-1, -1);  // (-1, -1): an unused slot
        if (i < ns)
            e = G.surv[i];
        const bool live = e.x >= 0;
        // every lane takes part in the staged key (a dead lane sums row 0
        // against itself)
        float ks = 0.f;
        if constexpr (M != M_HAM)
            ks = key32_staged<M>(P, live ? e.x : 0, live ? e.y & 0x7FFFFFFF : 0, sA, sB);
        if (live) {
            const int pi = e.x, pj = e.y & 0x7FFFFFFF;
            const bool passed = (e.y >> 31) & 1;
            npass += passed;
            const Thr E = G.pcl ? G.ct[G.pcl[pi]].E : G.E;
            float k;
            if constexpr (M == M_HAM)
                k = key32<M>(P, pi, pj);
            else
                k = ks;
            if constexpr (M == M_HAM) {
                edge = k <= E.lo;  // integer distance, exact
            } else if (k < E.lo) {
                edge = true;
            } else if (k > E.hi) {
                edge = false;
            } else {
                ++nrc;
                if constexpr (M == M_L2)
                    edge = l2_sq64(P.x + (size_t)pi * P.dp, P.x + (size_t)pj * P.dp,
                                   P.dim) <= E.p64;
                else
                    edge = ang_within64(P.x + (size_t)pi * P.dp,
                                        P.x + (size_t)pj * P.dp, P.dim, E.p64);
            }
            if (edge) {
                if (!passed)
                    ++nmis;  // validate: the filter would have lost this edge
                dd = edge_dist<M>(P, pi, pj, k, G.fp64_dist);
                if (M != M_HAM && G.validate) {
                    float ref;
                    if constexpr (M == M_L2)
                        ref = (float)sqrt(l2_sq64(P.x + (size_t)pi * P.dp,
                                                  P.x + (size_t)pj * P.dp, P.dim));
                    else if constexpr (M == M_HAM)
                        ref = dd;
                    else
                        ref = (float)ang_dist64(P.x + (size_t)pi * P.dp,
                                                P.x + (size_t)pj * P.dp, P.dim);
                    const float re = ref > 0.f ? fabsf(dd - ref) / ref : fabsf(dd);
                    maxerr = max(maxerr, __float_as_uint(re));
                }
                oi = G.perm[pi];
                oj = G.perm[pj];
                if (G.erank) {
                    rk.y = atomicAdd(&out.deg[oj], 1);
                } else {
                    atomicAdd(&out.deg[oi], 1);
                    atomicAdd(&out.deg[oj], 1);
                }
            }
        }
        // the first endpoint's rank: the list holds a row's survivors of a
        // block in runs, so one returning atomic serves a run
        if (G.erank)
            rk.x = claim_run(out.deg, edge ? oi : -1);
        // the survivor's own slot: an edge, or a hole (-1, -1) that the
        // scatter skips (no shared counter to contend on)
        if (i < ns) {
            edges[i] = edge ? make_int2(oi, oj) : make_int2(-1, -1);
            edist[i] = dd;
            if (G.erank)
                G.erank[i] = rk;
        }
    }
    nrc = wave_sum(nrc);
    npass = wave_sum(npass);
    nmis = wave_sum(nmis);
    maxerr = wave_max(maxerr);
    if (lane == 0) {
        if (nrc)
            atomicAdd(&out.cnt[1], nrc);
        if (npass)
            atomicAdd(&out.cnt[3], npass);
        if (nmis)
            atomicAdd(&out.cnt[4], nmis);
        if (maxerr)
            atomicMax((unsigned *)&out.cnt[5], maxerr);
    }
}

// Writes an edge list (input ids, distance; entries (-1, -1) are skipped)
// into the CSR: each entry into the slots of both endpoints when the list
// holds every edge once, else (every edge listed in both directions) into
// its first endpoint's row only.
__global__ void k_edges_scatter(const int2 *__restrict__ edges,
                                const float *__restrict__ edist, long long ne,
                                bool both, TileOut out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = edges[i];
        const unsigned long long s1 = claim_run(out.cursor, e.x);
        if (e.x < 0)
            continue;  // a survivor that is no edge
        const float d = edist[i];
        if (!both) {
            if (s1 < out.nnz) {
                out.col[s1] = e.y;
                out.dist[s1] = d;
            } else {
                atomicOr(out.err, ERR_INDEX);
            }
            continue;
        }
        const unsigned long long s2 = atomicAdd(&out.cursor[e.y], 1ull);
        if (s1 < out.nnz && s2 < out.nnz) {
            out.col[s1] = e.y;
            out.dist[s1] = d;
            out.col[s2] = e.x;
            out.dist[s2] = d;
        } else {
            atomicOr(out.err, ERR_INDEX);
        }
    }
}

__global__ void k_edges_place(const int2 *__restrict__ edges,
                              const float *__restrict__ edist,
                              const int2 *__restrict__ erank, long long ne,
                              const int64_t *__restrict__ row_ptr, TileOut out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = edges[i];
        if (e.x < 0)
            continue;  // a survivor that is no edge
        const int2 r = erank[i];
        const float d = edist[i];
        const int64_t a0 = row_ptr[e.x], a1 = row_ptr[e.x + 1];
        const int64_t b0 = row_ptr[e.y], b1 = row_ptr[e.y + 1];
        const int64_t s1 = a0 + r.x, s2 = b0 + r.y;
        if (r.x >= 0 && r.y >= 0 && s1 < a1 && s2 < b1) {
            out.col[s1] = e.y;
            out.dist[s1] = d;
            out.col[s2] = e.x;
            out.dist[s2] = d;
        } else {
            atomicOr(out.err, ERR_INDEX);
        }
    }
}

void edges_place(const int2 *edges, const float *edist, const int2 *erank, long long ne,
                 const int64_t *row_ptr, const TileOut &o, hipStream_t s)
{
    if (ne <= 0)
        return;
    FNN_LAUNCH(k_edges_place, dim3(grid_cap(ne, 256, 65536)), dim3(256), 0, s, edges, edist,
               erank, ne, row_ptr, o);
}

void survivors_launch(int metric, const Pts &P, const GramArgs &G,
                      long long nsurv, int2 *edges, float *edist,
                      const TileOut &o,
                      hipStream_t s)
{
    if (nsurv <= 0)
        return;
    // resident work-groups only: each wave's counters reach the shared
    // totals once
    static std::atomic<int> resident{0};
    int rb = resident.load();
    if (rb == 0) {
        FNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &rb, reinterpret_cast<const void *>(&k_survive<M_L2>), 256, 0));
        rb = std::max(1, rb);
        resident.store(rb);
    }
    const dim3 g((unsigned)std::min<long long>(grid_for(nsurv, 256),
                                               (long long)rb * num_cus()));
    if (metric == M_L2)
        FNN_LAUNCH((k_survive<M_L2>), g, dim3(256), 0, s, P, G, nsurv, edges,
                   edist, o);
    else if (metric == M_HAM)
        FNN_LAUNCH((k_survive<M_HAM>), g, dim3(256), 0, s, P, G, nsurv, edges,
                   edist, o);
    else
        FNN_LAUNCH((k_survive<M_ANG>), g, dim3(256), 0, s, P, G, nsurv, edges,
                   edist, o);
}

void edges_scatter(const int2 *edges, const float *edist, long long ne, bool both,
                   const TileOut &o, hipStream_t s)
{
    if (ne <= 0)
        return;
    FNN_LAUNCH(k_edges_scatter, dim3(grid_for(ne, 256)), dim3(256), 0, s, edges,
               edist, ne, both, o);
}

// Edges of the exact integer filter (tree positions, passed flag in bit 31
// of .y) into the CSR: distance from the codes, positions mapped to input
// ids.
__global__ void k_edges_scatter_ham(const int2 *__restrict__ surv, long long ne,
                                    const uint64_t *__restrict__ h, int W,
                                    const int32_t *__restrict__ perm, TileOut out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = surv[i];
        const int oi = e.x < 0 ? -1 : perm[e.x];
        const unsigned long long s1 = claim_run(out.cursor, oi);
        if (e.x < 0)
            continue;  // an unused slot
        const int pi = e.x, pj = e.y & 0x7FFFFFFF;
        const float d = (float)ham_words(h + (size_t)pi * W, h + (size_t)pj * W, W);
        const int oj = perm[pj];
        const unsigned long long s2 = atomicAdd(&out.cursor[oj], 1ull);
        if (s1 < out.nnz && s2 < out.nnz) {
            out.col[s1] = oj;
            out.dist[s1] = d;
            out.col[s2] = oi;
            out.dist[s2] = d;
        } else {
            atomicOr(out.err, ERR_INDEX);
        }
    }
}

void edges_scatter_ham(const int2 *surv, long long ne, const Pts &P,
                       const int32_t *perm, const TileOut &o, hipStream_t s)
{
    if (ne <= 0)
        return;
    FNN_LAUNCH(k_edges_scatter_ham, dim3(grid_cap(ne, 256, 4096)), dim3(256), 0, s, surv,
               ne, P.h, P.dp, perm, o);
}

__global__ void k_deg_from_positions(const int32_t *__restrict__ degp,
                                     const int32_t *__restrict__ perm, int n,
                                     int32_t *__restrict__ deg,
                                     unsigned long long *__restrict__ dsum)
{
    unsigned long long t = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += gridDim.x * blockDim.x) {
        deg[perm[p]] += degp[p];
        t += (unsigned long long)degp[p];
    }
    t = wave_sum(t);
    if ((threadIdx.x & (WAVE - 1)) == 0 && t)
        atomicAdd(dsum, t);
}

void degrees_from_positions(const int32_t *degp, const int32_t *perm, int n,
                            int32_t *deg, unsigned long long *dsum, hipStream_t s)
{
    if (n <= 0)
        return;
    FNN_LAUNCH(k_deg_from_positions, dim3(grid_cap(n, 256, 2048)), dim3(256), 0, s,
               degp, perm, n, deg, dsum);
}

template <int M, int PREC, int NKS>
static void launch_gram_k(bool fill_pass, const Pts &P, const GramArgs &G,
                          const TileOut &o, hipStream_t s)
{
    const int rowb = NKS * GramCfg<PREC>::KSTEP * GramCfg<PREC>::EB;
    const size_t sh = (size_t)GP * (rowb + 16) + sizeof(float) * GP * (GW + 1);
    // every work-group resident at once (a multiple of 8: one share per XCD)
    static std::atomic<int> resident{0};  // work-groups per CU (this instance)
    int rb = resident.load();
    if (rb == 0) {
        FNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &rb, reinterpret_cast<const void *>(&k_gram<M, PREC, NKS>), GT, sh));
        rb = std::max(1, rb);
        resident.store(rb);
    }
    const long long want = std::max<long long>(8, (long long)rb * num_cus() / 8 * 8);
    const long long need = ((long long)G.nunits + 7) / 8 * 8;
    const dim3 grid((unsigned)std::max<long long>(8, std::min(want, need)));
    (void)fill_pass;
    FNN_LAUNCH((k_gram<M, PREC, NKS>), grid, dim3(GT), sh, s, P, G, o);
}

template <int M, int PREC, int NKS>
static void launch_gram_direct(const Pts &P, const GramArgs &G, const TileOut &o,
                               hipStream_t s)
{
    static std::atomic<int> resident{0};  // work-groups per CU (this instance)
    int rb = resident.load();
    if (rb == 0) {
        FNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &rb, reinterpret_cast<const void *>(&k_gram_direct<M, PREC, NKS>), GT, 0));
        rb = std::max(1, rb);
        resident.store(rb);
    }
    const long long want = std::max<long long>(8, (long long)rb * num_cus() / 8 * 8);
    const long long need = ((long long)G.nunits + 7) / 8 * 8;
    const dim3 grid((unsigned)std::max<long long>(8, std::min(want, need)));
    FNN_LAUNCH((k_gram_direct<M, PREC, NKS>), grid, dim3(GT), 0, s, P, G, o);
    if (G.dense_pairs >= 0)
        fill(o.cnt + 2, (unsigned long long)G.dense_pairs, 1, s);
    else
        FNN_LAUNCH(k_gram_pairs, dim3(grid_cap(G.nlist, 256, 4096)), dim3(256), 0, s, G, o);
}

template <int M, int PREC>
static void launch_gram(bool fill_pass, const Pts &P, const GramArgs &G,
                        const TileOut &o, hipStream_t s)
{
    if (G.nunits <= 0)
        return;
    const int nks = G.kq / GramCfg<PREC>::KSTEP;
    if constexpr (PREC == FNN_PREC_I8) {
        switch (nks) {
        case 2: launch_gram_k<M, PREC, 2>(fill_pass, P, G, o, s); break;
        case 4: launch_gram_k<M, PREC, 4>(fill_pass, P, G, o, s); break;
        case 6: launch_gram_k<M, PREC, 6>(fill_pass, P, G, o, s); break;
        default: launch_gram_k<M, PREC, 8>(fill_pass, P, G, o, s); break;
        }
    } else if constexpr (is16(PREC)) {
        // the narrow kernel reads the per-pack copies (made when it applies)
        const bool narrow_fits = G.qp != nullptr;
        switch (nks) {
        case 1:
            if (narrow_fits)
                launch_gram_direct<M, PREC, 1>(P, G, o, s);
            else
                launch_gram_k<M, PREC, 1>(fill_pass, P, G, o, s);
            break;
        case 2:
            if (narrow_fits)
                launch_gram_direct<M, PREC, 2>(P, G, o, s);
            else
                launch_gram_k<M, PREC, 2>(fill_pass, P, G, o, s);
            break;
        case 3: launch_gram_k<M, PREC, 3>(fill_pass, P, G, o, s); break;
        case 4: launch_gram_k<M, PREC, 4>(fill_pass, P, G, o, s); break;
        case 5: launch_gram_k<M, PREC, 5>(fill_pass, P, G, o, s); break;
        case 6: launch_gram_k<M, PREC, 6>(fill_pass, P, G, o, s); break;
        case 7: launch_gram_k<M, PREC, 7>(fill_pass, P, G, o, s); break;
        default: launch_gram_k<M, PREC, 8>(fill_pass, P, G, o, s); break;
        }
    } else {
        if (nks == 1)
            launch_gram_k<M, PREC, 1>(fill_pass, P, G, o, s);
        else
            launch_gram_k<M, PREC, 2>(fill_pass, P, G, o, s);
    }
}

// Per-pack copies for the narrow kernel: row r of pack k at k * GP + r (the
// pack's row when r < its size, else zero) and its column term 0.5 hx (else
// FLT_MAX, which no accumulator reaches).
__global__ void k_pad_packs(const int32_t *__restrict__ pb, const int32_t *__restrict__ pe,
                            int npk, const unsigned char *__restrict__ q,
                            const float *__restrict__ hx, int rowb,
                            unsigned char *__restrict__ qp, float *__restrict__ ayp)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
         e < (long long)npk * GP; e += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(e / GP), r = (int)(e % GP);
        const int b = pb[k];
        const bool in = r < pe[k] - b;
        for (int c = 0; c < rowb; c += 16)
            *(int4 *)(qp + e * rowb + c) =
                in ? *(const int4 *)(q + (size_t)(b + r) * rowb + c) : make_int4(0, 0, 0, 0);
        ayp[e] = in ? 0.5f * hx[b + r] : FLT_MAX;
    }
}

void gram_pad_packs(int metric, int prec, GramArgs &G, Scratch &S)
{
    G.qp = nullptr;
    G.ayp = nullptr;
    const int nks = G.kq / GramCfg<FNN_PREC_BF16>::KSTEP;
    if (metric == M_HAM || !is16(prec) || nks < 1 || nks > 2 || G.npacks <= 0)
        return;
    const long long rowb = 32ll * nks;
    if ((long long)G.npacks * GP * rowb >= (1ll << 32))
        return;  // the staged kernel takes larger sets
    unsigned char *qp = (unsigned char *)S.raw((size_t)G.npacks * GP * rowb + 64);
    float *ayp = S.get<float>((size_t)G.npacks * GP);
    FNN_LAUNCH(k_pad_packs, dim3(grid_for((int64_t)G.npacks * GP, 256)), dim3(256), 0,
               S.stream(), G.q_pb + G.nn, G.q_pe + G.nn, G.npacks,
               (const unsigned char *)G.q, G.hx, (int)rowb, qp, ayp);
    G.qp = qp;
    G.ayp = ayp;
}

void gram_launch(int metric, int prec, bool fill_pass, const Pts &P,
                 const GramArgs &G, const TileOut &o, hipStream_t s)
{
    if (metric == M_HAM) {
        launch_gram<M_HAM, FNN_PREC_I8>(fill_pass, P, G, o, s);
    } else if (metric == M_L2) {
        if (prec == FNN_PREC_BF16)
            launch_gram<M_L2, FNN_PREC_BF16>(fill_pass, P, G, o, s);
        else if (prec == FNN_PREC_FP16)
            launch_gram<M_L2, FNN_PREC_FP16>(fill_pass, P, G, o, s);
        else
            launch_gram<M_L2, FNN_PREC_FP8>(fill_pass, P, G, o, s);
    } else {
        if (prec == FNN_PREC_BF16)
            launch_gram<M_ANG, FNN_PREC_BF16>(fill_pass, P, G, o, s);
        else if (prec == FNN_PREC_FP16)
            launch_gram<M_ANG, FNN_PREC_FP16>(fill_pass, P, G, o, s);
        else
            launch_gram<M_ANG, FNN_PREC_FP8>(fill_pass, P, G, o, s);
    }
}

// ------------------------------------------------------------- host side --

float gram_eps2(int metric, double eps, const Thr &E, double t2mul, double add)
{
    if (metric == M_HAM)
        return std::min(E.lo, 1048576.f);  // floor(eps); beyond any code length
    const double u32 = 1.0 / 16777216.0;
    const double T2 = gram_t2(metric, eps, E) * t2mul + add;
    return (float)(T2 * (1.0 + 320.0 * u32) + 1e-30);
}

// Hamming codes as +-1 bytes for the integer filter; no centring or
// scaling, the test is exact.
static void quantise_ham(const fnn_tree *T, int prec, Scratch &S, GramArgs &G)
{
    hipStream_t s = S.stream();
    const int n = (int)T->n, dp = T->dp;
    const int kq = dp * 64;
    if (prec != FNN_PREC_I8 || kq > 256)
        fail(FNN_EUNSUPPORTED, "integer MFMA filter supports codes of <= 256 bits");
    G.gscale = 1.f;
    G.kq = kq;
    int8_t *qb = (int8_t *)S.raw((size_t)n * kq + 64);
    G.q = qb;
    G.hx = nullptr;  // no per-point terms
    FNN_LAUNCH(k_quant_ham, dim3(grid_cap((int64_t)n * kq, 256, 16384)), dim3(256), 0,
               s, T->h, n, dp, qb);
}

// Leading principal coordinates of X for the filter (see k_pca): returns K
// (0: the filter runs on X itself) and, when K > 0, z [n][K] FP32, rho and
// the captured variance fraction.  proj: -1 off, 0 the smallest multiple of
// 16 whose residual variance, doubled (a pair's expected residual squared
// distance), is at most half the squared threshold, else that many
// coordinates.  kq_full is the padded width of X in the filter's format;
// only K < kq_full helps.  t2min is the smallest squared threshold of the
// query (FP64 rounding of the projection must also stay below 5e-7 of its
// root, else K = 0).
static int project_pca(const float *X, int n, int dp, int kq_full, int proj,
                       double t2min, const Centre &CX, Scratch &S, float **z,
                       double *rho, double *captured, unsigned *zmax, float known_absmax)
{
    hipStream_t s = S.stream();
    const int kmax = std::min({PCA_MAXK, (kq_full - 1) / 16 * 16, dp / 16 * 16});
    if (proj < 0 || kmax < 16 || (proj > 0 && proj > kmax))
        return 0;
    const int stride = (int)cdiv(n, PCA_ROWS);
    const long long m = cdiv(n, stride);
    const int nparts = (int)std::min<long long>(256, cdiv(m, 32));
    const int dd = dp * dp;
    double *part = S.get<double>((size_t)nparts * dd);
    double *Cv = S.get<double>(dd);
    FNN_LAUNCH(k_cov_partial, dim3(nparts), dim3(256), 0, s, X, n, dp, stride, CX, part);
    FNN_LAUNCH(k_cov_reduce, dim3(grid_for(dd, 256)), dim3(256), 0, s, part, nparts, dd,
               1.0 / (double)m, Cv);
    double *Y = S.get<double>((size_t)kmax * dp), *Z = S.get<double>((size_t)kmax * dp);
    double *Qd = S.get<double>((size_t)kmax * dp);
    int *kout = S.get<int>(1);
    double *info = S.get<double>(3);
    double *trd = info + 2;
    FNN_LAUNCH(k_pca_trace, dim3(1), dim3(256), 0, s, Cv, dp, trd);
    const dim3 gp(grid_for((int64_t)kmax * dp, 256));
    FNN_LAUNCH(k_pca_power, gp, dim3(256), 0, s, Cv, dp, kmax, trd, (const double *)nullptr, Y);
    FNN_LAUNCH(k_pca_power, gp, dim3(256), 0, s, Cv, dp, kmax, trd, (const double *)Y, Z);
    FNN_LAUNCH(k_pca_power, gp, dim3(256), 0, s, Cv, dp, kmax, trd, (const double *)Z, Y);
    FNN_LAUNCH(k_pca, dim3(1), dim3(256), 0, s, Cv, dp, kmax, proj, t2min, 0.5, trd, Y, Qd,
               kout, info);
    const int K = read_scalar(kout, s);
    double hinfo[2];
    FNN_HIP(hipMemcpyAsync(hinfo, info, sizeof hinfo, hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    if (K <= 0)
        return 0;
    // FP64 rounding of the projection: |z~_k - z_k| <= gamma sum_c |Q_ck| |v_c|
    // <= gamma sqrt(rho) |v|, |v| <= sqrt(dp) max |x_c - mu_c|
    float am = known_absmax;  // largest |x - mu| (negative: not known yet)
    if (am < 0.f) {
        unsigned *mx = S.get<unsigned>(1);
        fill(mx, 0u, 1, s);
        FNN_LAUNCH(k_absmax, dim3(grid_cap((int64_t)n * dp, 256, 2048)), dim3(256), 0, s, X,
                   n, dp, CX, mx);
        const unsigned mb = read_scalar(mx, s);
        memcpy(&am, &mb, 4);
    }
    const double u64 = 1.1102230246251565e-16;
    const double gam = (dp + 2) * u64 / (1.0 - (dp + 2) * u64);
    const double V = std::sqrt((double)dp) * (double)am * (1.0 + 1e-6);
    const double emax = std::sqrt((double)K) * gam * std::sqrt(hinfo[0]) * V;
    if (!(2.0 * emax <= 5e-7 * std::sqrt(hinfo[0]) * std::sqrt(t2min)))
        return 0;
    *z = S.get<float>((size_t)n * K);
    if (zmax)
        fill(zmax, 0u, 1, s);
    FNN_LAUNCH(k_project, dim3(grid_for(n, 256)), dim3(256), 0, s, X, n,
               dp, CX, Qd, K, *z, zmax);
    *rho = hinfo[0];
    *captured = hinfo[1];
    return K;
}

// Clouds that get their own centre: every cloud of a batch; one for a
// single tree and for a bichromatic query (its pairs cross the clouds).
static int centre_clouds(const fnn_tree *T)
{
    return T->cross_a >= 0 ? 1 : T->ncloud;
}

// Per-cloud centres of the rows X [n][dp] (one cloud: the global mean).
static Centre make_centre(const fnn_tree *T, const float *X, int dp, const float *inv,
                          Scratch &S, bool zero = false)
{
    hipStream_t s = S.stream();
    const int n = (int)T->n, ncl = centre_clouds(T);
    const int32_t *pcl = ncl > 1 ? T->pcl : nullptr;
    float *sums = S.get<float>((size_t)ncl * dp);
    fill(sums, 0.f, (int64_t)ncl * dp, s);
    if (!zero)
        FNN_LAUNCH(k_colsum, dim3((unsigned)cdiv(n, 1024)), dim3(256), 0, s, X, n, dp, pcl,
                   sums);
    return Centre{sums, inv, pcl, dp};
}

// 1 / size of every cloud, on the device.
static float *cloud_inv_sizes(const fnn_tree *T, Scratch &S)
{
    hipStream_t s = S.stream();
    const int ncl = centre_clouds(T);
    float *inv = S.get<float>(ncl);
    std::vector<float> ih(ncl);
    for (int c = 0; c < ncl; ++c) {
        const int64_t sz = ncl == 1 ? T->n : T->cloud_off_h[c + 1] - T->cloud_off_h[c];
        ih[c] = 1.0f / (float)std::max<int64_t>(sz, 1);
    }
    FNN_HIP(hipMemcpyAsync(inv, ih.data(), sizeof(float) * ncl, hipMemcpyHostToDevice, s));
    FNN_HIP(hipStreamSynchronize(s));  // ih goes out of scope
    return inv;
}

double gram_margin_ratio(const fnn_tree *T, double t2min, int prec, Scratch &S,
                         GramPre *pre)
{
    hipStream_t s = S.stream();
    const int n = (int)T->n, dp = T->dp, d = T->dim;
    const float *X = T->metric == M_ANG ? T->xn : T->x;
    const float *inv = cloud_inv_sizes(T, S);
    const Centre CX = make_centre(T, X, dp, inv, S);
    double *acc = S.get<double>(2);  // [0] sum of |x - mu|^2, [1] largest |x - mu|
    fill(acc, 0.0, 2, s);
    FNN_LAUNCH(k_sqdev, dim3(grid_cap((int64_t)n * (dp / 4), 256 * 8, 1024)), dim3(256), 0, s, X, n,
               dp, CX, acc,
               reinterpret_cast<unsigned *>(acc + 1));
    double h[2];
    FNN_HIP(hipMemcpyAsync(h, acc, sizeof h, hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    const double mean = h[0] / std::max(n, 1);
    if (pre) {
        unsigned mb;
        memcpy(&mb, &h[1], 4);  // the low word holds the float bits
        memcpy(&pre->absmax, &mb, 4);
        pre->sums = CX.sums;
        pre->inv = inv;
        pre->have = true;
    }
    const double u32 = 1.0 / 16777216.0;
    const int kq = (int)cdiv(dp, 16) * 16;
    const double u = prec == FNN_PREC_FP16 ? 1.0 / 2048.0 : 1.0 / 256.0;
    const double c1 = 2.25 * u + (4.0 * kq + 2.0 * d + 72.0) * u32;
    return t2min > 0 ? 2.0 * c1 * mean / t2min : HUGE_VAL;
}

// Centred, shrunk BF16, FP16 or FP8 copy of the coordinates (or of their leading
// principal coordinates) and the per-point norms of the filter.
//
// With principal coordinates z~ (FP32 roundings of z = Q^T (x - mu)
// computed in FP64): |z~(x) - z~(y)| <= sqrt(rho) d(x, y) + 2 e + u'(|z~(x)|
// + |z~(y)|), e the FP64 bound above (<= 5e-7 sqrt(rho) eps) and u' =
// u32 (1 + u32).  Squaring with (a + b)^2 <= (1 + tau) a^2 + (1 + 1/tau) b^2,
// tau = 1e-6, gives |z~(x) - z~(y)|^2 <= rho eps^2 (1 + 4e-6) + 1e-7
// (|z~(x)|^2 + |z~(y)|^2): eps^2 is scaled by t2mul = rho (1 + 4e-6) and
// c1 grows by 1e-7.
static void quantise_real(const fnn_tree *T, int prec, int proj, double t2min,
                          Scratch &S, GramArgs &G, const GramPre *pre)
{
    hipStream_t s = S.stream();
    const int n = (int)T->n;
    int dp = T->dp, d = T->dim;
    const float *X = T->metric == M_ANG ? T->xn : T->x;
    if (prec == FNN_PREC_I8)
        fail(FNN_EUNSUPPORTED, "integer MFMA filter is for Hamming codes");
    const int KS = is16(prec) ? 16 : 64;
    if (cdiv(dp, KS) * KS > 128)
        fail(FNN_EUNSUPPORTED, "MFMA filter supports dim <= 128 (got %d)", d);
    // per-cloud centres (one cloud: the global mean), from the automatic
    // precision rule's pass when it ran
    const bool known = pre && pre->have;
    const float *inv = known ? pre->inv : cloud_inv_sizes(T, S);
    Centre CX = known ? Centre{pre->sums, inv, centre_clouds(T) > 1 ? T->pcl : nullptr, dp}
                      : make_centre(T, X, dp, inv, S);
    G.t2mul = 1.0;
    G.proj = 0;
    G.captured = 0.0;
    double c_extra = 0.0;
    unsigned *zmax = nullptr;  // largest |z| (float bits), from the projection
    {
        float *z = nullptr;
        double rho = 1.0, cap = 0.0;
        unsigned *zm = S.get<unsigned>(1);
        const int K = project_pca(X, n, dp, (int)cdiv(dp, KS) * KS, proj, t2min, CX, S,
                                  &z, &rho, &cap, zm, known ? pre->absmax : -1.f);
        if (K > 0) {
            zmax = zm;
            X = z;
            dp = d = K;
            G.t2mul = rho * (1.0 + 4e-6);
            G.proj = K;
            G.captured = cap;
            c_extra = 1e-7;
            // z = Q^T (x - mu) is centred already (per cloud): its own mean
            // is a rounding residue, and the filter's bound holds for any
            // centre, so z is quantised about 0
            CX = make_centre(T, X, dp, inv, S, true);
        }
    }
    const int kq = (int)cdiv(dp, KS) * KS;
    const double u32 = 1.0 / 16777216.0;
    const double u = prec == FNN_PREC_BF16   ? 1.0 / 256.0
                     : prec == FNN_PREC_FP16 ? 1.0 / 2048.0
                                             : 1.0 / 16.0;
    // FP16: the filter runs on s (x - mu), s = 2^e with the largest
    // |coordinate| in [2^14, 2^15) (no overflow), eps^2 scaled by s^2 (exact).
    // Below 2^-14 the format is subnormal: |q(v) - v| <= u |v| + eta, eta =
    // 2^-25.  Per coordinate |q(a) q(b) - a b| <= (2u + u^2)|a||b| + 2.01 eta
    // (|a| + |b|) + eta^2; summed, with |a|_1 <= sqrt(k) |a| and |a| <= (|a|^2
    // + 1) / 2, the eta part of the error of 2 g~ is at most 2.01 eta sqrt(k)
    // (|a|^2 + |b|^2) + 4.02 eta sqrt(k) + 2 k eta^2: the first term goes into
    // c1, the rest is added to the scaled eps^2.
    const double eta = prec == FNN_PREC_FP16 ? std::ldexp(1.0, -25) : 0.0;
    G.e2add = prec == FNN_PREC_FP16 ? 4.02 * eta * std::sqrt((double)kq) + 2.0 * kq * eta * eta
                                    : 0.0;
    // margin coefficient (see the header comment); the FP8 subnormal terms
    // are absorbed by the global scale that maps the largest |coordinate| to
    // at least 224.
    const double c1 = 2.25 * u + (4.0 * kq + 2.0 * d + 72.0) * u32 +
                      (prec == FNN_PREC_FP8 ? 4.0 * d / 224.0 / 512.0 : 0.0) +
                      2.01 * eta * std::sqrt((double)kq) + c_extra;
    float scale = 1.f;
    if (prec == FNN_PREC_FP16) {
        // largest |x - mu|: from the projection (z is centred about 0), else
        // one pass over the rows
        unsigned *mx = zmax;
        if (!mx) {
            mx = S.get<unsigned>(1);
            fill(mx, 0u, 1, s);
            FNN_LAUNCH(k_absmax, dim3(grid_cap((int64_t)n * dp, 256, 2048)), dim3(256), 0,
                       s, X, n, dp, CX, mx);
        }
        unsigned mb = read_scalar(mx, s);
        float m;
        memcpy(&m, &mb, 4);
        if (m > 0.f) {
            int e;
            frexpf(m, &e);  // 2^(e-1) <= m < 2^e
            scale = ldexpf(1.f, 15 - e);
        }
        G.t2mul *= (double)scale * (double)scale;
    }
    if (prec == FNN_PREC_FP8) {
        unsigned *mx = S.get<unsigned>(1);
        fill(mx, 0u, 1, s);
        FNN_LAUNCH(k_absmax, dim3(grid_cap((int64_t)n * dp, 256, 2048)), dim3(256), 0,
                   s, X, n, dp, CX, mx);
        unsigned mb = read_scalar(mx, s);
        float m;
        memcpy(&m, &mb, 4);
        if (m > 0.f) {
            int e;
            frexpf(224.0f / m, &e);  // 2^(e-1) <= 224/m < 2^e
            scale = ldexpf(1.f, e - 1);
        }
    }
    // FP8 products are scaled back by gscale; the FP16 filter works in
    // scaled units throughout (norms, eps^2)
    G.gscale = prec == FNN_PREC_FP16 ? 1.f : 1.0f / (scale * scale);
    G.kq = kq;
    void *qbuf = S.raw((size_t)n * kq * (is16(prec) ? 2 : 1) + 64);
    float *hxbuf = S.get<float>(n);
    G.q = qbuf;
    G.hx = hxbuf;
    if (prec == FNN_PREC_BF16)
        FNN_LAUNCH((k_quant<FNN_PREC_BF16>), dim3(grid_cap(n, 4, 16384)), dim3(256), 0,
                   s, X, n, dp, kq, CX, scale, (float)(1.0 - c1), qbuf, hxbuf);
    else if (prec == FNN_PREC_FP16)
        FNN_LAUNCH((k_quant<FNN_PREC_FP16>), dim3(grid_cap(n, 4, 16384)), dim3(256), 0,
                   s, X, n, dp, kq, CX, scale, (float)(1.0 - c1), qbuf, hxbuf);
    else
        FNN_LAUNCH((k_quant<FNN_PREC_FP8>), dim3(grid_cap(n, 4, 16384)), dim3(256), 0,
                   s, X, n, dp, kq, CX, scale, (float)(1.0 - c1), qbuf, hxbuf);
}

bool gram_packs_fit(const fnn_tree *T, Scratch &S)
{
    hipStream_t s = S.stream();
    const int nn = (int)T->nnodes, npk = (int)T->npacks;
    if (npk <= 0)
        return true;
    int32_t *big = S.get<int32_t>(1);
    fill(big, 0, 1, s);
    FNN_LAUNCH(k_max_pack, dim3(grid_for(npk, 256)), dim3(256), 0, s, T->q_pt_begin + nn,
               T->q_pt_end + nn, npk, GP, big);
    return read_scalar(big, s) == 0;
}

double gram_t2(int metric, double eps, const Thr &E)
{
    return metric == M_L2 ? eps * eps : 2.0 - 2.0 * E.p64;
}

// Quantised copy + per-point terms, and the MFMA work lists, for one query.
void gram_prepare(const fnn_tree *T, int prec, int proj, double eps, const Thr &E,
                  double t2min, const int2 *inter, long long ninter, Scratch &S,
                  GramArgs &G, int2 **rest, long long *nrest, const GramPre *pre)
{
    hipStream_t s = S.stream();
    G.e2add = 0.0;
    G.dense_pairs = -1;
    G.upk = 0;
    if (T->metric == M_HAM) {
        quantise_ham(T, prec, S, G);
        G.t2mul = 1.0;
        G.proj = 0;
        G.captured = 0.0;
    } else {
        quantise_real(T, prec, proj, t2min, S, G, pre);
    }
    G.e2f = gram_eps2(T->metric, eps, E, G.t2mul, G.e2add);
    G.E = E;
    G.q_pb = T->q_pt_begin;
    G.q_pe = T->q_pt_end;

    const int nn = (int)T->nnodes;
    const int npk = (int)T->npacks;
    const int RUN = UNIT_MAX;  // work unit: at most RUN list entries of one group

    // ---- near-complete interaction lists: closed-form work list ----------
    // When the traversal kept (almost) every pack pair and no pack is larger
    // than GP, the work list is every (group g, B >= 4g) pair; the few pairs
    // the traversal pruned are evaluated too, which changes no edge.
    {
        const int ngr = (npk + GW - 1) / GW;
        const long long allp = (long long)npk * (npk + 1) / 2;
        long long mu = 0;  // entries: every (group, B >= its first pack)
        for (int g = 0; g < ngr; ++g)
            mu += npk - GW * g;
        if (npk > 0 && (double)ninter >= 0.95 * (double)allp && mu < INT32_MAX) {
            int32_t *big = S.get<int32_t>(1);
            fill(big, 0, 1, s);
            FNN_LAUNCH(k_max_pack, dim3(grid_for(npk, 256)), dim3(256), 0, s,
                       T->q_pt_begin + nn, T->q_pt_end + nn, npk, GP, big);
            if (read_scalar(big, s) == 0) {
                // one cloud: full packs of consecutive tree positions in
                // place of the tree's (indexed from 0, not past the nodes)
                const bool one = T->ncloud <= 1 && T->cross_a < 0;
                int base = nn, np = npk;
                if (one) {
                    np = (int)((T->n + GP - 1) / GP);
                    int32_t *vpb = S.get<int32_t>(np), *vpe = S.get<int32_t>(np);
                    FNN_LAUNCH(k_uniform_packs, dim3(grid_for(np, 256)), dim3(256), 0, s,
                               (int)T->n, np, vpb, vpe);
                    base = 0;
                    G.q_pb = vpb;
                    G.q_pe = vpe;
                    G.upk = (int)T->n;
                    const int ng1 = (np + GW - 1) / GW;
                    mu = 0;
                    for (int g = 0; g < ng1; ++g)
                        mu += np - GW * g;
                }
                const int ngp = (np + GW - 1) / GW;
                // units ordered by B run (runs aligned to RUN packs), then by
                // group: the units of one run read the same B tiles.  The
                // host sums the per-run counts; the unit table itself is
                // filled on the device (k_dense_plan).
                const int nrun = (np + RUN - 1) / RUN;
                std::vector<long long> U(nrun + 1, 0), E(nrun + 1, 0);
                for (int k = 0; k < nrun; ++k) {
                    const long long kR = (long long)k * RUN;
                    const long long h = std::min<long long>(kR + RUN, np);
                    const long long c = std::min<long long>(ngp, (h + GW - 1) / GW);
                    const long long a = std::min<long long>(c, kR / GW + 1);
                    U[k + 1] = U[k] + c;
                    E[k + 1] = E[k] + a * (h - kR) + (c - a) * h -
                               (long long)GW * ((a + c - 1) * (c - a) / 2);
                }
                const int nu = (int)U[nrun];
                const int64_t e = E[nrun];
                int32_t *lg = S.get<int32_t>(mu + 1), *lb = S.get<int32_t>(mu + 1);
                int32_t *ubeg = S.get<int32_t>(nu + 1);
                int32_t *ug_d = S.get<int32_t>(nu), *ulo_d = S.get<int32_t>(nu);
                long long *UE = S.get<long long>(2 * (size_t)(nrun + 1));
                FNN_HIP(hipMemcpyAsync(UE, U.data(), sizeof(long long) * (nrun + 1),
                                       hipMemcpyHostToDevice, s));
                FNN_HIP(hipMemcpyAsync(UE + nrun + 1, E.data(), sizeof(long long) * (nrun + 1),
                                       hipMemcpyHostToDevice, s));
                FNN_LAUNCH(k_dense_plan, dim3(grid_for(nu, 256)), dim3(256), 0, s, UE,
                           UE + nrun + 1, nrun, RUN, np, nu, ubeg, ug_d, ulo_d);
                FNN_LAUNCH(k_dense_units, dim3(grid_cap(nu, 4, 16384)), dim3(256), 0, s,
                           ubeg, ug_d, ulo_d, nu, lg, lb);
                FNN_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
                *rest = nullptr;
                *nrest = 0;
                G.nn = base;
                G.npacks = np;
                G.lg = lg;
                G.lb = lb;
                G.ubeg = ubeg;
                G.nunits = nu;
                G.nlist = (int)e;
                // every pair of one cloud: the narrow kernel screens each once
                if (one)
                    G.dense_pairs = T->n * (T->n - 1) / 2;
                return;
            }
        }
    }

    // ---- lists: canonical pairs, routed, unique per (group, B) ----------
    uint32_t *k1 = S.get<uint32_t>(ninter + 1), *v1 = S.get<uint32_t>(ninter + 1);
    int2 *rs = S.get<int2>(ninter + 1);
    unsigned long long *cnt = S.get<unsigned long long>(2);
    fill(cnt, 0ull, 2, s);
    // sentinels past every B pack and every group (within the sort's bits)
    const uint32_t kinf = (uint32_t)npk, ginf = (uint32_t)(npk / GW + 1);
    FNN_LAUNCH(k_route, dim3(grid_for(ninter, 256)), dim3(256), 0, s, inter,
               ninter, T->q_pt_begin, T->q_pt_end, nn, GP, kinf, ginf, k1, v1, cnt, rs);
    unsigned long long hc[2];
    FNN_HIP(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    const long long m = ninter - (long long)hc[1];  // real pairs: sorted first
    *rest = rs;
    *nrest = (long long)hc[1];
    G.nn = nn;
    G.npacks = npk;
    if (m == 0) {
        G.nunits = 0;
        return;
    }
    auto bits = [](uint32_t v) {
        int b = 0;
        while (v) {
            ++b;
            v >>= 1;
        }
        return b;
    };
    uint32_t *k2 = S.get<uint32_t>(ninter), *v2 = S.get<uint32_t>(ninter);
    // sort by B, then stably by group: (group, B) order, sentinels last
    radix_sort_pairs(k1, v1, k2, v2, ninter, bits(kinf), S);
    uint32_t *gk = S.get<uint32_t>(ninter), *bv = S.get<uint32_t>(ninter);
    radix_sort_pairs(v2, k2, gk, bv, ninter, bits(ginf), S);
    int32_t *flag = S.get<int32_t>(m + 1), *pos = S.get<int32_t>(m + 2);
    FNN_LAUNCH(k_uniq_flags, dim3(grid_for(m, 256)), dim3(256), 0, s, gk, bv, m,
               flag);
    scan_i32(flag, pos, m, S);
    const int mu = read_scalar(pos + m, s);
    int32_t *lg = S.get<int32_t>(mu + 1), *lb = S.get<int32_t>(mu + 1);
    G.lg = lg;
    G.lb = lb;
    FNN_LAUNCH(k_uniq_write, dim3(grid_for(m, 256)), dim3(256), 0, s, gk, bv, m,
               flag, pos, lg, lb);
    // units of at most RUN entries of one group
    int32_t *uf = S.get<int32_t>(mu + 1), *up = S.get<int32_t>(mu + 2);
    int32_t *gfirst = S.get<int32_t>(npk / GW + 2);
    FNN_LAUNCH(k_group_first, dim3(grid_for(mu, 256)), dim3(256), 0, s, lg, mu,
               gfirst);
    FNN_LAUNCH(k_units, dim3(grid_for(mu, 256)), dim3(256), 0, s, lg, mu, RUN,
               gfirst, uf);
    scan_i32(uf, up, mu, S);
    const int nu = read_scalar(up + mu, s);
    int32_t *ubeg = S.get<int32_t>(nu + 1);
    G.ubeg = ubeg;
    FNN_LAUNCH(k_units_write, dim3(grid_for(mu, 256)), dim3(256), 0, s, uf, up,
               mu, ubeg);
    FNN_HIP(hipMemcpyAsync(ubeg + nu, &mu, sizeof(int), hipMemcpyHostToDevice, s));
    FNN_HIP(hipStreamSynchronize(s));
    G.nunits = nu;
    G.nlist = mu;
}

}  // namespace fnn
