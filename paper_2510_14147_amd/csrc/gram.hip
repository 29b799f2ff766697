// MFMA Gram filter for the Euclidean and angular leaf tiles.
//
// d(x,y)^2 = |x|^2 + |y|^2 - 2 x.y.  The inner products of a tile are taken
// on the matrix cores from BF16 (or FP8 E4M3) copies of the globally centred
// points, accumulated in FP32.  With u the unit roundoff of the input
// format, |q(x).q(y) - x.y| <= (2u + u^2)|x||y| (Cauchy-Schwarz), plus the
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
// GW waves.  Every unordered point pair is evaluated once: a wave skips B
// packs with a smaller id, and inside its own pack keeps only pairs whose
// first point precedes the second in tree order.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include <string.h>

#include "gram.h"

namespace fnn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) int i32x8;

constexpr int GP = 64;           // rows per pack (max) on the MFMA path
constexpr int GW = 4;            // packs per group = waves per work-group
constexpr int UNIT_MAX = 64;     // list entries per work unit (at most)
// two waves per SIMD: the second wave hides the first one's LDS and MFMA
// dependency stalls (one wave per SIMD with 512 registers measured 1.7x
// slower)
constexpr int GRAM_WAVES_PER_SIMD = 2;

// ---------------------------------------------------------------- prep ---

__global__ void k_colsum(const float *__restrict__ x, int n, int dp,
                         float *__restrict__ sums)
{
    // block b takes rows [b*R, (b+1)*R); thread t sums columns t, t+256..
    const int R = 1024;
    const int r0 = blockIdx.x * R, r1 = min(n, r0 + R);
    for (int c = threadIdx.x; c < dp; c += blockDim.x) {
        float s = 0.f;
        for (int r = r0; r < r1; ++r)
            s += x[(size_t)r * dp + c];
        atomicAdd(&sums[c], s);
    }
}

// Quantised rows of x - mu (tree order) and the per-point norm term.
template <int PREC>
__global__ void k_quant(const float *__restrict__ x, int n, int dp, int kq,
                        const float *__restrict__ sums, float inv_n,
                        float scale, float one_minus_c1, void *__restrict__ q,
                        float *__restrict__ hx)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int i = blockIdx.x * wpb + threadIdx.x / WAVE; i < n;
         i += gridDim.x * wpb) {
        float ss = 0.f;
        for (int k = lane; k < kq; k += WAVE) {
            float v = 0.f;
            if (k < dp) {
                v = x[(size_t)i * dp + k] - sums[k] * inv_n;
                ss = fmaf(v, v, ss);
            }
            if constexpr (PREC == FNN_PREC_BF16) {
                ((__bf16 *)q)[(size_t)i * kq + k] = (__bf16)v;
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

__global__ void k_absmax(const float *__restrict__ x, int n, int dp,
                         const float *__restrict__ sums, float inv_n,
                         unsigned *__restrict__ mx)
{
    float m = 0.f;
    const int64_t tot = (int64_t)n * dp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[e] - sums[e % dp] * inv_n));
    m = wave_max(m);
    if ((threadIdx.x & (WAVE - 1)) == 0)
        atomicMax(mx, __float_as_uint(m));
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
                        uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                        unsigned long long *__restrict__ cnt,
                        int2 *__restrict__ rest)
{
    // one reservation per wave and destination (whole waves iterate, so the
    // ballots see every lane)
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
        const uint64_t mb = __ballot(valid && big), ms = __ballot(valid && !big);
        unsigned long long ob = 0, os = 0;
        if (lane == 0) {
            if (mb)
                ob = atomicAdd(&cnt[1], (unsigned long long)__popcll(mb));
            if (ms)
                os = atomicAdd(&cnt[0], (unsigned long long)__popcll(ms));
        }
        ob = __shfl(ob, 0, WAVE);
        os = __shfl(os, 0, WAVE);
        if (valid && big) {
            rest[ob + __popcll(mb & lt)] = make_int2(a, b);
        } else if (valid) {
            const unsigned long long o = os + __popcll(ms & lt);
            key[o] = (uint32_t)(b - nn);
            val[o] = (uint32_t)((a - nn) / GW);
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
struct GramCfg<FNN_PREC_FP8> {
    static constexpr int KSTEP = 64;
    static constexpr int EB = 1;
};
template <>
struct GramCfg<FNN_PREC_I8> {
    static constexpr int KSTEP = 32;  // code bits (one signed byte each) per MFMA
    static constexpr int EB = 1;
};

typedef __attribute__((ext_vector_type(4))) int i32x4;
typedef __attribute__((ext_vector_type(16))) int i32x16;

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

    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    const int l32 = lane & 31, hi = lane >> 5;
    // products carry the FP8 scale; gscale and its inverse are powers of 2
    const float ginv = PREC == FNN_PREC_BF16 ? 1.f : 1.f / G.gscale;
    unsigned long long npairs = 0;
    const uint64_t ltmask = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    // XCD-aware order: the dispatcher hands consecutive work-groups to the 8
    // XCDs in turn, so physical block b runs on XCD b % 8.  XCD x takes the
    // contiguous slice of the unit order starting at xs (units that share B
    // tiles are adjacent in that order and then meet in one XCD's L2).
    const int nbk = gridDim.x, xq = nbk / 8, xr = nbk % 8;
    const int xcd = blockIdx.x % 8;
    const int xs = xcd * xq + min(xcd, xr);
    const int u0 = xs + (int)(blockIdx.x / 8);
    for (int u = u0; u < G.nunits; u += gridDim.x) {
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
                    if constexpr (PREC == FNN_PREC_BF16 || PREC == FNN_PREC_I8) {
                        // k-step ks: bytes ks*32 + hi*16 .. +16 (BF16
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
            if (ca >= 0 && eC[e - e0] != ca)
                continue;                      // different clouds never connect
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
            constexpr bool B16 = PREC == FNN_PREC_BF16 || PREC == FNN_PREC_I8;
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
                } else if constexpr (PREC == FNN_PREC_BF16) {
                    const int4 bv[2] = {bfrag[ks][0], bfrag[ks][1]};
                    const int slot = ks >> 1, half = ks & 1;
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        bf16x8 bb;
                        __builtin_memcpy(&bb, &bv[cb], 16);
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb) {
                            const int4 av = make_int4(Areg[rb][slot][half * 4 + 0],
                                                      Areg[rb][slot][half * 4 + 1],
                                                      Areg[rb][slot][half * 4 + 2],
                                                      Areg[rb][slot][half * 4 + 3]);
                            bf16x8 aa;
                            __builtin_memcpy(&aa, &av, 16);
                            acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                aa, bb, acc[cb][rb], 0, 0, 0);
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
            if (__any(mx[0] >= ayc[0] || mx[1] >= ayc[1]) || self || G.validate) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                if (cb * 32 >= nb)
                    break;
                const int col = cb * 32 + l32;
                const V ay = ayc[cb];
                unsigned pm = 0, om = 0;
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int row = rb * 32 + 8 * (q >> 2) + 4 * hi + (q & 3);
                        const bool ok = row < na && col < nb && (!self || row < col);
                        const V gq = PREC == FNN_PREC_FP8 ? (V)(acc[cb][rb][q] * G.gscale)
                                                          : (V)acc[cb][rb][q];
                        const bool pass = ok && (gq >= ay);
                        pm |= (unsigned)pass << (rb * 16 + q);
                        om |= (unsigned)ok << (rb * 16 + q);
                    }
                }
                // ---- survivors: appended for the exact decision kernel -----
                const unsigned todo = G.validate ? om : pm;
                const int mine = __popc(todo);
                int incl = mine;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    const int v = __shfl_up(incl, o, WAVE);
                    if (lane >= o)
                        incl += v;
                }
                const int total = __shfl(incl, WAVE - 1, WAVE);
                if (total) {
                    unsigned long long base = 0;
                    if (lane == 0)
                        base = atomicAdd(G.nsurv, (unsigned long long)total);
                    base = __shfl(base, 0, WAVE);
                    unsigned long long o = base + (unsigned long long)(incl - mine);
                    unsigned tb = todo;
                    while (tb) {
                        const int bit = __ffs(tb) - 1;
                        tb &= tb - 1;
                        const int rb = bit >> 4, q = bit & 15;
                        const int row = rb * 32 + 8 * (q >> 2) + 4 * hi + (q & 3);
                        if ((long long)o < G.surv_cap)
                            G.surv[o] = make_int2(pa + row,
                                                  (pb + col) | (int)(((pm >> bit) & 1u) << 31));
                        ++o;
                        if constexpr (PREC == FNN_PREC_I8)
                            if (G.degp)
                                atomicAdd(&G.degp[pa + row], 1);
                    }
                }
                if constexpr (PREC == FNN_PREC_I8) {
                    // exact filter, not validating: the survivors are the
                    // edges; column degrees summed over the two row halves
                    // of each column (lanes l and l + 32)
                    const int cdeg = mine + __shfl_xor(mine, 32, WAVE);
                    if (G.degp && hi == 0 && cdeg)
                        atomicAdd(&G.degp[pb + col], cdeg);
                }
            }
            }
            // pairs screened by this wave (both column blocks)
            if (lane == 0) {
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    if (cb * 32 >= nb)
                        break;
                    // rows r < na against columns c0 .. c0+nc-1 (r < c if self)
                    const long long nc = min(32, nb - cb * 32), c0 = cb * 32;
                    if (!self) {
                        npairs += (unsigned long long)(na * nc);
                    } else {
                        // sum_{c=c0}^{c0+nc-1} min(na, c)
                        const long long lo = c0, hi2 = c0 + nc;  // [lo, hi2)
                        const long long mid = max(lo, min(hi2, (long long)na));
                        npairs += (unsigned long long)((mid - lo) * (lo + mid - 1) / 2 +
                                                       (hi2 - mid) * na);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (lane == 0 && npairs)
        atomicAdd(&out.cnt[2], npairs);
}

// Exact decision of every survivor: direct-difference FP32 key, FP64 inside
// the rounding band; edges go to an unordered list (input ids, distance) and
// to the row degrees.
template <int M>
__global__ void __launch_bounds__(256)
k_survive(Pts P, GramArgs G, long long ns, int2 *__restrict__ edges,
          float *__restrict__ edist, unsigned long long *__restrict__ nedges,
          TileOut out)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const uint64_t ltm = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    unsigned long long nrc = 0, npass = 0, nmis = 0;
    unsigned maxerr = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    // the loop runs a whole number of waves so that ballots see every lane
    const long long lim = (ns + WAVE - 1) / WAVE * WAVE;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += stride) {
        bool edge = false;
        float dd = 0.f;
        int oi = 0, oj = 0;
        if (i < ns) {
            const int2 e = G.surv[i];
            const int pi = e.x, pj = e.y & 0x7FFFFFFF;
            const bool passed = (e.y >> 31) & 1;
            npass += passed;
            const Thr E = G.pcl ? G.ct[G.pcl[pi]].E : G.E;
            float k;
            if constexpr (M == M_HAM)
                k = key32<M>(P, pi, pj);
            else
                k = key32_seq<M>(P, pi, pj);
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
                atomicAdd(&out.deg[oi], 1);
                atomicAdd(&out.deg[oj], 1);
            }
        }
        const uint64_t m = __ballot(edge);
        if (m) {
            unsigned long long base = 0;
            if (lane == 0)
                base = atomicAdd(nedges, (unsigned long long)__popcll(m));
            base = __shfl(base, 0, WAVE);
            if (edge) {
                const unsigned long long o = base + __popcll(m & ltm);
                edges[o] = make_int2(oi, oj);
                edist[o] = dd;
            }
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

// Writes an unordered edge list (input ids, distance) into the CSR slots of
// both endpoints.
__global__ void k_edges_scatter(const int2 *__restrict__ edges,
                                const float *__restrict__ edist, long long ne,
                                TileOut out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = edges[i];
        const float d = edist[i];
        const unsigned long long s1 = atomicAdd(&out.cursor[e.x], 1ull);
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

void survivors_launch(int metric, const Pts &P, const GramArgs &G,
                      long long nsurv, int2 *edges, float *edist,
                      unsigned long long *nedges, const TileOut &o,
                      hipStream_t s)
{
    if (nsurv <= 0)
        return;
    const dim3 g(grid_for(nsurv, 256));
    if (metric == M_L2)
        FNN_LAUNCH((k_survive<M_L2>), g, dim3(256), 0, s, P, G, nsurv, edges,
                   edist, nedges, o);
    else if (metric == M_HAM)
        FNN_LAUNCH((k_survive<M_HAM>), g, dim3(256), 0, s, P, G, nsurv, edges,
                   edist, nedges, o);
    else
        FNN_LAUNCH((k_survive<M_ANG>), g, dim3(256), 0, s, P, G, nsurv, edges,
                   edist, nedges, o);
}

void edges_scatter(const int2 *edges, const float *edist, long long ne,
                   const TileOut &o, hipStream_t s)
{
    if (ne <= 0)
        return;
    FNN_LAUNCH(k_edges_scatter, dim3(grid_for(ne, 256)), dim3(256), 0, s, edges,
               edist, ne, o);
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
        const int pi = e.x, pj = e.y & 0x7FFFFFFF;
        const float d = (float)ham_words(h + (size_t)pi * W, h + (size_t)pj * W, W);
        const int oi = perm[pi], oj = perm[pj];
        const unsigned long long s1 = atomicAdd(&out.cursor[oi], 1ull);
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
    FNN_LAUNCH(k_edges_scatter_ham, dim3(grid_for(ne, 256)), dim3(256), 0, s, surv,
               ne, P.h, P.dp, perm, o);
}

__global__ void k_deg_from_positions(const int32_t *__restrict__ degp,
                                     const int32_t *__restrict__ perm, int n,
                                     int32_t *__restrict__ deg)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += gridDim.x * blockDim.x)
        deg[perm[p]] += degp[p];
}

void degrees_from_positions(const int32_t *degp, const int32_t *perm, int n,
                            int32_t *deg, hipStream_t s)
{
    if (n <= 0)
        return;
    FNN_LAUNCH(k_deg_from_positions, dim3(grid_cap(n, 256, 16384)), dim3(256), 0, s,
               degp, perm, n, deg);
}

template <int M, int PREC, int NKS>
static void launch_gram_k(bool fill_pass, const Pts &P, const GramArgs &G,
                          const TileOut &o, hipStream_t s)
{
    const int rowb = NKS * GramCfg<PREC>::KSTEP * GramCfg<PREC>::EB;
    const size_t sh = (size_t)GP * (rowb + 16) + sizeof(float) * GP * (GW + 1);
    const dim3 grid(grid_for(G.nunits, 1));
    (void)fill_pass;
    FNN_LAUNCH((k_gram<M, PREC, NKS>), grid, dim3(GT), sh, s, P, G, o);
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
    } else if constexpr (PREC == FNN_PREC_BF16) {
        switch (nks) {
        case 1: launch_gram_k<M, PREC, 1>(fill_pass, P, G, o, s); break;
        case 2: launch_gram_k<M, PREC, 2>(fill_pass, P, G, o, s); break;
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

void gram_launch(int metric, int prec, bool fill_pass, const Pts &P,
                 const GramArgs &G, const TileOut &o, hipStream_t s)
{
    if (metric == M_HAM) {
        launch_gram<M_HAM, FNN_PREC_I8>(fill_pass, P, G, o, s);
    } else if (metric == M_L2) {
        if (prec == FNN_PREC_BF16)
            launch_gram<M_L2, FNN_PREC_BF16>(fill_pass, P, G, o, s);
        else
            launch_gram<M_L2, FNN_PREC_FP8>(fill_pass, P, G, o, s);
    } else {
        if (prec == FNN_PREC_BF16)
            launch_gram<M_ANG, FNN_PREC_BF16>(fill_pass, P, G, o, s);
        else
            launch_gram<M_ANG, FNN_PREC_FP8>(fill_pass, P, G, o, s);
    }
}

// ------------------------------------------------------------- host side --

float gram_eps2(int metric, double eps, const Thr &E)
{
    if (metric == M_HAM)
        return std::min(E.lo, 1048576.f);  // floor(eps); beyond any code length
    const double u32 = 1.0 / 16777216.0;
    const double T2 = metric == M_L2 ? eps * eps : 2.0 - 2.0 * E.p64;
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

// Centred, shrunk BF16 or FP8 copy of the coordinates and the per-point
// norms of the filter.
static void quantise_real(const fnn_tree *T, int prec, Scratch &S, GramArgs &G)
{
    hipStream_t s = S.stream();
    const int n = (int)T->n, dp = T->dp;
    const int d = T->dim;
    const float *X = T->metric == M_ANG ? T->xn : T->x;
    if (prec == FNN_PREC_I8)
        fail(FNN_EUNSUPPORTED, "integer MFMA filter is for Hamming codes");
    const int KS = prec == FNN_PREC_BF16 ? 16 : 64;
    const int kq = (int)cdiv(dp, KS) * KS;
    if (kq > 128)
        fail(FNN_EUNSUPPORTED, "MFMA filter supports dim <= 128 (got %d)", d);
    const double u32 = 1.0 / 16777216.0;
    const double u = prec == FNN_PREC_BF16 ? 1.0 / 256.0 : 1.0 / 16.0;
    // margin coefficient (see the header comment); the FP8 subnormal terms
    // are absorbed by the global scale that maps the largest |coordinate| to
    // at least 224.
    const double c1 = 2.25 * u + (4.0 * kq + 2.0 * d + 72.0) * u32 +
                      (prec == FNN_PREC_FP8 ? 4.0 * d / 224.0 / 512.0 : 0.0);
    // mean, scale
    float *sums = S.get<float>(dp);
    fill(sums, 0.f, dp, s);
    FNN_LAUNCH(k_colsum, dim3((unsigned)cdiv(n, 1024)), dim3(256), 0, s, X, n,
               dp, sums);
    float scale = 1.f;
    if (prec == FNN_PREC_FP8) {
        unsigned *mx = S.get<unsigned>(1);
        fill(mx, 0u, 1, s);
        FNN_LAUNCH(k_absmax, dim3(grid_for((int64_t)n * dp, 256)), dim3(256), 0,
                   s, X, n, dp, sums, 1.0f / n, mx);
        unsigned mb = read_scalar(mx, s);
        float m;
        memcpy(&m, &mb, 4);
        if (m > 0.f) {
            int e;
            frexpf(224.0f / m, &e);  // 2^(e-1) <= 224/m < 2^e
            scale = ldexpf(1.f, e - 1);
        }
    }
    G.gscale = 1.0f / (scale * scale);
    G.kq = kq;
    void *qbuf = S.raw((size_t)n * kq * (prec == FNN_PREC_BF16 ? 2 : 1) + 64);
    float *hxbuf = S.get<float>(n);
    G.q = qbuf;
    G.hx = hxbuf;
    if (prec == FNN_PREC_BF16)
        FNN_LAUNCH((k_quant<FNN_PREC_BF16>), dim3(grid_cap(n, 4, 16384)), dim3(256), 0,
                   s, X, n, dp, kq, sums, 1.0f / n, scale, (float)(1.0 - c1), qbuf,
                   hxbuf);
    else
        FNN_LAUNCH((k_quant<FNN_PREC_FP8>), dim3(grid_cap(n, 4, 16384)), dim3(256), 0,
                   s, X, n, dp, kq, sums, 1.0f / n, scale, (float)(1.0 - c1), qbuf,
                   hxbuf);
}

// Quantised copy + per-point terms, and the MFMA work lists, for one query.
void gram_prepare(const fnn_tree *T, int prec, double eps, const Thr &E,
                  const int2 *inter, long long ninter, Scratch &S, GramArgs &G,
                  int2 **rest, long long *nrest)
{
    hipStream_t s = S.stream();
    if (T->metric == M_HAM)
        quantise_ham(T, prec, S, G);
    else
        quantise_real(T, prec, S, G);
    G.e2f = gram_eps2(T->metric, eps, E);
    G.E = E;

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
                // units ordered by B run (runs aligned to RUN packs), then by
                // group: the units of one run read the same B tiles
                std::vector<int32_t> ub, ug, ulo;
                int64_t e = 0;
                for (int k = 0; (int64_t)k * RUN < npk; ++k)
                    for (int g = 0; g < ngr; ++g) {
                        const int lo = std::max(k * RUN, GW * g);
                        const int hi = std::min((k + 1) * RUN, npk);
                        if (lo >= hi)
                            continue;
                        ub.push_back((int32_t)e);
                        ug.push_back(g);
                        ulo.push_back(lo);
                        e += hi - lo;
                    }
                ub.push_back((int32_t)e);
                const int nu = (int)ug.size();
                int32_t *lg = S.get<int32_t>(mu + 1), *lb = S.get<int32_t>(mu + 1);
                int32_t *ubeg = S.get<int32_t>(nu + 1);
                int32_t *ug_d = S.get<int32_t>(nu), *ulo_d = S.get<int32_t>(nu);
                FNN_HIP(hipMemcpyAsync(ubeg, ub.data(), sizeof(int32_t) * (nu + 1),
                                       hipMemcpyHostToDevice, s));
                FNN_HIP(hipMemcpyAsync(ug_d, ug.data(), sizeof(int32_t) * nu,
                                       hipMemcpyHostToDevice, s));
                FNN_HIP(hipMemcpyAsync(ulo_d, ulo.data(), sizeof(int32_t) * nu,
                                       hipMemcpyHostToDevice, s));
                FNN_LAUNCH(k_dense_units, dim3(grid_cap(nu, 4, 16384)), dim3(256), 0, s,
                           ubeg, ug_d, ulo_d, nu, lg, lb);
                FNN_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
                *rest = nullptr;
                *nrest = 0;
                G.nn = nn;
                G.npacks = npk;
                G.lg = lg;
                G.lb = lb;
                G.ubeg = ubeg;
                G.nunits = nu;
                G.nlist = (int)e;
                return;
            }
        }
    }

    // ---- lists: canonical pairs, routed, unique per (group, B) ----------
    uint32_t *k1 = S.get<uint32_t>(ninter + 1), *v1 = S.get<uint32_t>(ninter + 1);
    int2 *rs = S.get<int2>(ninter + 1);
    unsigned long long *cnt = S.get<unsigned long long>(2);
    fill(cnt, 0ull, 2, s);
    FNN_LAUNCH(k_route, dim3(grid_for(ninter, 256)), dim3(256), 0, s, inter,
               ninter, T->q_pt_begin, T->q_pt_end, nn, GP, k1, v1, cnt, rs);
    unsigned long long hc[2];
    FNN_HIP(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    const long long m = (long long)hc[0];
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
    uint32_t *k2 = S.get<uint32_t>(m), *v2 = S.get<uint32_t>(m);
    // sort by B, then stably by group: (group, B) order
    radix_sort_pairs(k1, v1, k2, v2, m, bits((uint32_t)npk), S);
    uint32_t *gk = S.get<uint32_t>(m), *bv = S.get<uint32_t>(m);
    radix_sort_pairs(v2, k2, gk, bv, m, bits((uint32_t)(npk / GW + 1)), S);
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
