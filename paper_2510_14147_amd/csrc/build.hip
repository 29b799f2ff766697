// Level-wise batched cover-tree construction (Section IV-A; Algorithm 1
// SplitVertex driven level by level as in Algorithm 2 BuildLevel), for every
// hub of a level at once.
//
// Data layout.  Points stay in input order during the build; a permutation
// perm[pos] keeps every hub's points contiguous (its segment).  Per
// position: D = FP32 key to the currently assigned centre, L = index of that
// centre within the hub's centre list (cent[hub_begin + j], input indices).
//
// One level ("round"):
//  1. net selection, repeated passes over all active hubs:
//       k_update  -- apply the centres accepted in the last pass (D <- min,
//                    L <- argmin, strict '<' so ties stay with the earlier
//                    centre), then report per 64-point chunk the farthest
//                    point not yet within 2^{l-1} of its centre;
//       k_select  -- per hub, accept up to kmax of those farthest points,
//                    farthest first, each only if it is more than 2^{l-1}
//                    from every centre accepted in the same pass.
//     A hub stops when no point is farther than 2^{l-1} from its centre.
//     Threshold decisions inside the FP32 rounding band are made in FP64.
//  2. stable segmented partition of every hub by centre (radix sort on the
//     child id), children become vertices one level down; children with
//     more than zeta points (and nonzero radius) are next level's hubs.
#include <float.h>
#include <limits.h>
#include <math.h>
#include <string.h>

#include <algorithm>

#include "tree.h"

namespace fnn {

constexpr int CH = 64;  // chunk of a hub handled by one wave

// ------------------------------------------------------------ thresholds --

static void round_out(double lo, double hi, float *flo, float *fhi)
{
    float a = (float)lo, b = (float)hi;
    if ((double)a > lo)
        a = nextafterf(a, -INFINITY);
    if ((double)b < hi)
        b = nextafterf(b, INFINITY);
    *flo = a;
    *fhi = b;
}

// Band of the FP32 key around the exact threshold key T (see common.h).
static Thr band(int metric, int dp, double T, double p64)
{
    const double u = 1.0 / 16777216.0;
    Thr t;
    t.p64 = p64;
    if (metric == M_L2) {
        double b = 2.0 * (dp + 4) * u;
        double a = (dp + 4) * 1e-37;
        round_out(T * (1.0 - b) - a, T * (1.0 + b) + a, &t.lo, &t.hi);
        if (!(t.lo < FLT_MAX))
            t.lo = FLT_MAX;
    } else {
        double dl = T * 2.0 * (3.0 * dp + 24) * u + 16.0 * u * sqrt(T) + 1e-9;
        round_out(T - dl, T + dl, &t.lo, &t.hi);
    }
    return t;
}

Thr make_thr_eps(int metric, int dp, double eps)
{
    if (metric == M_HAM || metric == M_LEV) {
        Thr t;
        double k = floor(eps);
        if (k > 1e9)
            k = 1e9;
        t.lo = t.hi = (float)k;
        t.p64 = k;
        return t;
    }
    if (metric == M_L2) {
        double E2 = eps * eps;
        return band(metric, dp, E2, E2);
    }
    double C = eps >= M_PI ? -1.0 : cos(eps);
    return band(metric, dp, 2.0 - 2.0 * C, C);
}

void make_level_table(int metric, int dp, LevelTab *tab)
{
    for (int i = 0; i < NLEV; ++i) {
        int l = i - LOFF;
        double tau = ldexp(1.0, l);
        Thr t;
        if (metric == M_HAM || metric == M_LEV) {
            double k = floor(tau);
            if (k > 1e9)
                k = 1e9;
            t.lo = t.hi = (float)k;
            t.p64 = k;
        } else if (metric == M_L2) {
            double T = ldexp(1.0, 2 * l);
            t = band(metric, dp, T, T);
        } else {
            double C = tau >= M_PI ? -1.0 : cos(tau);
            t = band(metric, dp, 2.0 - 2.0 * C, C);
        }
        tab->t[i] = t;
    }
}

// ------------------------------------------------------------- ingest ----

// Largest coordinate magnitude accepted for vector metrics: every squared
// difference sum over dim coordinates stays below 4 bound^2 dim <= 4e37,
// well inside FP32 range.
float coord_bound(int dim)
{
    return (float)std::min(1e16, sqrt(1e37 / std::max(dim, 1)));
}

// Coordinates are checked to be finite and at most `bound` in magnitude
// (so that no FP32 squared distance or squared norm can overflow: the host
// sets bound = min(1e16, sqrt(1e37 / dim))); angular rows must be non-zero.
// The unit rows of the angular metric are computed from an FP64 norm, so
// tiny rows whose FP32 squared norm would underflow are still accepted.
// Euclidean rows already a multiple of four floats wide (no padding) and
// 16-byte aligned: the same checks over flat float4 pieces, one error flag
// per wave; the build then reads the caller's rows in place (x null: no
// copy).
__global__ void k_ingest_flat(const float4 *__restrict__ in, long long n4, float bound,
                              float4 *__restrict__ x, int *err)
{
    bool bad = false, big = false;
    for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < n4;
         f += (long long)gridDim.x * blockDim.x) {
        const float4 v = in[f];
        bad |= !isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(v.w);
        big |= fabsf(v.x) > bound || fabsf(v.y) > bound || fabsf(v.z) > bound ||
               fabsf(v.w) > bound;
        if (x)
            x[f] = v;
    }
    // a non-finite coordinate reports ERR_INPUT (and no range error for it)
    const bool b = __any(bad), g = __any(big && !bad);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (b)
            atomicOr(err, ERR_INPUT);
        if (g)
            atomicOr(err, ERR_RANGE);
    }
}

__global__ void k_ingest_vec(const float *__restrict__ in, int n, int dim,
                             int dp, int angular, float bound,
                             float *__restrict__ x, float *__restrict__ xn,
                             int *err)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int i = blockIdx.x * wpb + threadIdx.x / WAVE; i < n;
         i += gridDim.x * wpb) {
    const float *r = in + (size_t)i * dim;
    float *o = x + (size_t)i * dp;
    double ss = 0.0;
    bool bad = false, big = false;
    for (int k = lane; k < dp; k += WAVE) {
        float v = k < dim ? r[k] : 0.f;
        bad |= !isfinite(v);
        big |= fabsf(v) > bound;
        ss += (double)v * (double)v;
        o[k] = v;
    }
    if (__any(bad)) {
        if (lane == 0)
            atomicOr(err, ERR_INPUT);
        continue;
    }
    if (__any(big)) {
        if (lane == 0)
            atomicOr(err, ERR_RANGE);
        continue;
    }
    if (angular) {
        ss = wave_sum(ss);
        if (!(ss > 0.0)) {
            if (lane == 0)
                atomicOr(err, ERR_INPUT);
            continue;
        }
        // unit row in FP32 (the key's error band allows for its rounding)
        const double inv = 1.0 / sqrt(ss);
        float *on = xn + (size_t)i * dp;
        for (int k = lane; k < dp; k += WAVE)
            on[k] = (float)((double)o[k] * inv);
    }
    }
}

__global__ void k_ingest_lev(const uint8_t *__restrict__ in, int n, int stride,
                             int32_t *__restrict__ len, int *__restrict__ sigma,
                             int *err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint8_t *r = in + (size_t)i * stride;
    int l = 0, mx = -1;
    while (l < stride && r[l] != 0xFF) {
        mx = max(mx, (int)r[l]);
        ++l;
    }
    len[i] = l;
    if (mx >= MAX_SIGMA)
        atomicOr(err, ERR_INPUT);
    else if (mx >= 0)
        atomicMax(sigma, mx + 1);
}

__global__ void k_peq(const uint8_t *__restrict__ s, const int32_t *__restrict__ len,
                      int n, int stride, int sigma, int W,
                      uint64_t *__restrict__ peq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint64_t *o = peq + (size_t)i * sigma * W;
    for (int k = 0; k < sigma * W; ++k)
        o[k] = 0ull;
    const uint8_t *r = s + (size_t)i * stride;
    const int l = len[i];
    for (int p = 0; p < l; ++p) {
        int c = r[p];
        if (c < sigma)
            o[c * W + (p >> 6)] |= 1ull << (p & 63);
    }
}

// --------------------------------------------------------------- root ----

template <int M>
__global__ void k_root_keys(Pts P, int32_t *__restrict__ perm,
                            float *__restrict__ D, unsigned *__restrict__ kmax)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float k = 0.f;
    if (i < P.n) {
        perm[i] = i;
        if constexpr (M == M_L2 || M == M_ANG) {
            // key32's four chains in its order, the row read eight float4
            // at a time (one thread per row: the loads, not the arithmetic,
            // set the pace)
            const float *X = M == M_L2 ? P.x : P.xn;
            const float *a = X + (size_t)i * P.dp, *b = X;
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
            for (int c = 0; c < P.dp; c += 32) {
                float4 u[8], w[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (c + 4 * q < P.dp) {
                        u[q] = *reinterpret_cast<const float4 *>(a + c + 4 * q);
                        w[q] = *reinterpret_cast<const float4 *>(b + c + 4 * q);
                    }
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (c + 4 * q < P.dp) {
                        const float d0 = u[q].x - w[q].x, d1 = u[q].y - w[q].y,
                                    d2 = u[q].z - w[q].z, d3 = u[q].w - w[q].w;
                        s0 = fmaf(d0, d0, s0);
                        s1 = fmaf(d1, d1, s1);
                        s2 = fmaf(d2, d2, s2);
                        s3 = fmaf(d3, d3, s3);
                    }
            }
            k = (s0 + s1) + (s2 + s3);
        } else {
            k = key32<M>(P, i, 0);
        }
        D[i] = k;
    }
    // one atomic per work-group of 256 (atomics on one address serialise)
    __shared__ float wm[4];
    k = wave_max(k);
    if ((threadIdx.x & (WAVE - 1)) == 0)
        wm[threadIdx.x / WAVE] = k;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(kmax, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

// Forest of independent clouds: cloud id of every position, and each point's
// key to the first point of its cloud (that cloud's root centre).
__global__ void k_cloud_ids(const int32_t *__restrict__ off, int C,
                            int32_t *__restrict__ pcl)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int c = blockIdx.x * wpb + threadIdx.x / WAVE; c < C;
         c += gridDim.x * wpb)
        for (int p = off[c] + lane; p < off[c + 1]; p += WAVE)
            pcl[p] = c;
}

template <int M>
__global__ void k_forest_keys(Pts P, const int32_t *__restrict__ off,
                              const int32_t *__restrict__ pcl,
                              int32_t *__restrict__ perm, float *__restrict__ D,
                              unsigned *__restrict__ kmax)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const long long lim = ((long long)P.n + WAVE - 1) / WAVE * WAVE;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += (long long)gridDim.x * blockDim.x) {
        const bool ok = i < P.n;
        int c = -1;
        float k = 0.f;
        if (ok) {
            c = pcl[i];
            perm[i] = (int32_t)i;
            k = key32<M>(P, (int)i, off[c]);
            D[i] = k;
        }
        // one atomic per wave when the wave lies inside one cloud
        const int c0 = __shfl(c, 0, WAVE);
        const bool same = __ballot(ok && c != c0) == 0ull;
        if (same) {
            const float m = wave_max(k);
            if (lane == 0 && c0 >= 0)
                atomicMax(&kmax[c0], __float_as_uint(m));
        } else if (ok) {
            atomicMax(&kmax[c], __float_as_uint(k));
        }
    }
}

// -------------------------------------------------------------- chunks ---

struct Hubs {
    int32_t *node, *b, *e, *lvl, *m, *ma, *act, *cb, *ce, *kof;
};

__global__ void k_hub_sizes(const int32_t *__restrict__ b,
                            const int32_t *__restrict__ e, int H,
                            int32_t *__restrict__ nch, int32_t *__restrict__ sz)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H)
        return;
    int s = e[h] - b[h];
    nch[h] = (s + CH - 1) / CH;
    sz[h] = s;
}

__global__ void k_make_chunks(Hubs hb, int H, const int32_t *__restrict__ choff,
                              const int32_t *__restrict__ itemoff,
                              int32_t *__restrict__ ch_hub,
                              int32_t *__restrict__ ch_s,
                              int32_t *__restrict__ ch_e,
                              int32_t *__restrict__ ch_k)
{
    for (int h = blockIdx.x; h < H; h += gridDim.x) {
        const int c0 = choff[h], c1 = choff[h + 1];
        const int b = hb.b[h], e = hb.e[h];
        if (threadIdx.x == 0) {
            hb.cb[h] = c0;
            hb.ce[h] = c1;
            hb.kof[h] = itemoff[h];
        }
        for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
            int s = b + (c - c0) * CH;
            ch_hub[c] = h;
            ch_s[c] = s;
            ch_e[c] = min(s + CH, e);
            ch_k[c] = itemoff[h] + (c - c0) * CH;
        }
    }
}

__global__ void __launch_bounds__(CH)
k_round_init(const int32_t *__restrict__ ch_s, const int32_t *__restrict__ ch_e,
             const int32_t *__restrict__ ch_k, int NC, int32_t *__restrict__ L,
             int32_t *__restrict__ hpos)
{
    for (int c = blockIdx.x; c < NC; c += gridDim.x) {
        const int p = ch_s[c] + threadIdx.x;
        if (p < ch_e[c]) {
            L[p] = 0;
            hpos[ch_k[c] + threadIdx.x] = p;
        }
    }
}

// ------------------------------------------------------ net selection ----

__device__ __forceinline__ bool better(float d, int id, float d2, int id2)
{
    return d > d2 || (d == d2 && id < id2);
}

constexpr int UPD_K = 32;   // centres staged per batch
constexpr int CAND_R = 8;   // most candidates reported per chunk and pass

// Candidates per chunk of a hub with nch chunks: about 2 kmax per hub when
// the hub is small, one per chunk once it has that many chunks.
__device__ __forceinline__ int cand_per_chunk(int nch, int kmax)
{
    return min(CAND_R, max(1, (2 * kmax + nch - 1) / nch));
}
constexpr int UPD_D = 128;  // largest row stride staged in LDS

constexpr int UPD_W = 4;  // queue entries (one wave each) per work-group
static_assert(CH == 64 && UPD_K % 8 == 0, "lane layout of the distance loop");

// One point per lane against a staged batch of nj (<= UPD_K) centres
// (rows ldc apart in LDS; every lane reads the same centre row, a
// broadcast): UPD_K FMA chains over the coordinates in order, then the
// running nearest over the batch in centre order (strict '<': the first
// minimum stays).  The wave's 64 point rows (point o of each lane) come
// through the wave's LDS rows stg, US_CH coordinates at a time: each load
// instruction reads whole row segments of several rows instead of 64
// scattered lines, and the next segment is in flight while this one is
// used.  Groups of eight centres past nj are skipped (a wave-uniform test);
// rows between nj and the group's end are staged data that is never
// compared.  Called with every lane of the wave active.
constexpr int US_CH = 8;              // coordinates per staged segment
constexpr int US_LDR = US_CH + 4;       // floats per staged row (bank spread)
constexpr int US_F = US_CH / 4;         // float4 per row segment
__device__ __forceinline__ void upd_lane(const float *__restrict__ X, int o, float *stg,
                                         const float *__restrict__ cen, int ldc, int dp,
                                         int jb, int nj, float &dcur, int &lcur)
{
    constexpr int NJ = UPD_K;
    const int lane = threadIdx.x & (CH - 1);
    float acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        acc[j] = 0.f;
    const int q4 = dp >> 2, p4 = 4 * (lane % US_F);
    // this lane stages float4 p4 / 4 of the rows of lanes lane / F + (64 / F) i
    const float *rs[US_F];
    int so[US_F];
#pragma unroll
    for (int i = 0; i < US_F; ++i) {
        const int r = lane / US_F + (CH / US_F) * i;
        rs[i] = X + (size_t)__shfl(o, r, CH) * dp + p4;
        so[i] = r * US_LDR + p4;
    }
    float4 va[US_F];
    auto fetch = [&](int c0) {
        const bool in = c0 + p4 < dp;
#pragma unroll
        for (int i = 0; i < US_F; ++i)
            va[i] = in ? *(const float4 *)(rs[i] + c0) : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    fetch(0);
    for (int c0 = 0; c0 < dp; c0 += US_CH) {
#pragma unroll
        for (int i = 0; i < US_F; ++i)
            *(float4 *)(stg + so[i]) = va[i];
        if (c0 + US_CH < dp)
            fetch(c0 + US_CH);
        // one wave's LDS accesses complete in order: only the compiler must
        // keep the reads after the writes (and the next writes after them)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        float4 vr[US_F];
#pragma unroll
        for (int u = 0; u < US_F; ++u)
            vr[u] = *(const float4 *)(stg + lane * US_LDR + 4 * u);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int u = 0; u < US_F; ++u) {
            const int cc4 = c0 / 4 + u;
            const float4 v = vr[u];
            if (cc4 < q4) {
#pragma unroll
                for (int g = 0; g < NJ / 8; ++g) {
                    if (8 * g < nj) {
#pragma unroll
                        for (int jj = 0; jj < 8; ++jj) {
                            const int j = 8 * g + jj;
                            const float4 cc = *reinterpret_cast<const float4 *>(
                                __builtin_assume_aligned(cen + j * ldc + 4 * cc4, 16));
                            const float d0 = v.x - cc.x, d1 = v.y - cc.y, d2 = v.z - cc.z,
                                        d3 = v.w - cc.w;
                            acc[j] = fmaf(d0, d0, acc[j]);
                            acc[j] = fmaf(d1, d1, acc[j]);
                            acc[j] = fmaf(d2, d2, acc[j]);
                            acc[j] = fmaf(d3, d3, acc[j]);
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        if (j < nj && acc[j] < dcur) {
            dcur = acc[j];
            lcur = jb + j;
        }
}

template <int M>
__global__ void __launch_bounds__(CH * UPD_W)
k_update(Pts P, const int32_t *__restrict__ ch_hub, const int32_t *__restrict__ ch_s,
         const int32_t *__restrict__ ch_e, const int32_t *__restrict__ queue,
         const int32_t *__restrict__ qlen, Hubs hb,
         const int32_t *__restrict__ cent, const int32_t *__restrict__ perm,
         float *__restrict__ D, int32_t *__restrict__ L,
         const LevelTab *__restrict__ tab, float *__restrict__ cb_D,
         int32_t *__restrict__ cb_id, int kmax, unsigned long long *__restrict__ cnt)
{
    // staged centres: UPD_K rows of the point stride (sized at launch, so
    // low-dimensional inputs keep many work-groups resident), shared by the
    // work-group's waves whose chunks belong to the same hub (a hub's chunks
    // are consecutive in the queue)
    extern __shared__ __align__(16) float cen[];
    __shared__ __align__(16) float ustg[UPD_W][CH * US_LDR];  // each wave's staged rows
    __shared__ int hub_s[UPD_W];
    const int w = threadIdx.x / CH, lane = threadIdx.x % CH;
    // the queue lists the chunks of the hubs still active (device-resident
    // length, so passes need no host round trip)
    const int nq = *qlen;
    for (int t0 = blockIdx.x * UPD_W; t0 < nq; t0 += gridDim.x * UPD_W) {
    const int t = t0 + w;
    const int c = t < nq ? queue[t] : 0;
    const int h = t < nq ? ch_hub[c] : 0;
    const bool act = t < nq && hb.act[h];
    const int s = act ? ch_s[c] : 0, e = act ? ch_e[c] : 0;
    const int p = s + lane;
    const bool valid = act && p < e;
    const int b = act ? hb.b[h] : 0;
    const int j0 = act ? hb.ma[h] : 0, j1 = act ? hb.m[h] : 0;
    float dv = -1.f;
    int id = INT_MAX;
    const int o = valid ? perm[p] : 0;
    float dcur = valid ? D[p] : 0.f;
    int lcur = valid ? L[p] : 0;
    bool staged = false;
    if constexpr (M == M_L2 || M == M_ANG) {
        // vector metrics: the pass's new centres go to LDS in batches of
        // UPD_K, once per distinct hub of the work-group, and every point
        // row is read once per batch
        staged = P.dp <= UPD_D;
        if (staged) {
            const float *X = (M == M_ANG) ? P.xn : P.x;
            const int dp = P.dp, ldc = dp + 4;  // rows 16-byte aligned
            // one point per lane (its row read once per batch), the batch's
            // centres broadcast from LDS
            __syncthreads();  // hub_s of the previous entries is consumed
            if (lane == 0)
                hub_s[w] = act && j1 > j0 ? h : -1;
            __syncthreads();
            for (int r = 0; r < UPD_W; ++r) {
                const int hr = hub_s[r];
                bool first = hr >= 0;
                for (int q = 0; q < r; ++q)
                    first = first && hub_s[q] != hr;
                if (!first)
                    continue;  // no hub, or staged in an earlier round
                const bool mine = act && h == hr;  // the same in every lane
                const int br = hb.b[hr], j0r = hb.ma[hr], j1r = hb.m[hr];
                for (int jb = j0r; jb < j1r; jb += UPD_K) {
                    const int nj = min(UPD_K, j1r - jb);
                    __syncthreads();  // the previous batch is consumed
                    {
                        // nj rows of dp / 4 float4 each, at most UPD_K * UPD_D / 4
                        // in all: every index load, then every row load, is
                        // issued before the first wait
                        constexpr int SU = UPD_K * UPD_D / 4 / (CH * UPD_W);
                        static_assert(SU * CH * UPD_W * 4 == UPD_K * UPD_D, "staging split");
                        const int q4 = dp >> 2, tot = nj * q4;
                        int ci[SU], so[SU], c4[SU];
#pragma unroll
                        for (int u = 0; u < SU; ++u) {
                            const int f = threadIdx.x + u * CH * UPD_W;
                            const int r = f < tot ? f / q4 : 0;
                            ci[u] = f < tot ? cent[br + jb + r] : -1;
                            c4[u] = 4 * (f - r * q4);
                            so[u] = r * ldc + c4[u];
                        }
                        float4 cv[SU];
#pragma unroll
                        for (int u = 0; u < SU; ++u)
                            if (ci[u] >= 0)
                                cv[u] = *reinterpret_cast<const float4 *>(
                                    X + (size_t)ci[u] * dp + c4[u]);
#pragma unroll
                        for (int u = 0; u < SU; ++u)
                            if (ci[u] >= 0)
                                *reinterpret_cast<float4 *>(cen + so[u]) = cv[u];
                    }
                    __syncthreads();
                    if (mine)
                        upd_lane(X, o, ustg[w], cen, ldc, dp, jb, nj, dcur, lcur);
                }
            }
        }
    }
    if (valid) {
        bool scanned = staged;  // the new centres already compared
        if constexpr (M == M_HAM) {
            if (!scanned && P.dp <= 4) {
                // codes of up to 256 bits: the point's words stay in
                // registers and eight centres' indices and words are
                // fetched at once (the scan order is unchanged)
                uint64_t mine[4];
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    mine[w] = w < P.dp ? P.h[(size_t)o * P.dp + w] : 0ull;
                for (int j = j0; j < j1; j += 8) {
                    int cj[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        cj[u] = j + u < j1 ? cent[b + j + u] : -1;
                    uint64_t cw[8][4];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int w = 0; w < 4; ++w)
                            cw[u][w] = cj[u] >= 0 && w < P.dp ? P.h[(size_t)cj[u] * P.dp + w]
                                                              : 0ull;
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (cj[u] >= 0) {
                            int dh = 0;
#pragma unroll
                            for (int w = 0; w < 4; ++w)
                                dh += __popcll(mine[w] ^ cw[u][w]);
                            const float k = (float)dh;
                            if (k < dcur) {
                                dcur = k;
                                lcur = j + u;
                            }
                        }
                }
                scanned = true;
            }
        }
        if (!scanned)
            for (int j = j0; j < j1; ++j) {
                float k = key32<M>(P, o, cent[b + j]);
                if (k < dcur) {
                    dcur = k;
                    lcur = j;
                }
            }
        if (j1 > j0) {
            D[p] = dcur;
            L[p] = lcur;
        }
        const Thr T = tab->t[hb.lvl[h] - 1 + LOFF];
        if (!within<M>(P, o, cent[b + lcur], dcur, T, cnt + 1)) {
            dv = dcur;
            id = o;
        }
    }
    if (act) {
        // the chunk's R farthest uncovered points, farthest first
        const int R = cand_per_chunk(hb.ce[h] - hb.cb[h], kmax);
        for (int r = 0; r < R; ++r) {
            float bd = dv;
            int bi = id;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                float d2 = __shfl_xor(bd, off, WAVE);
                int i2 = __shfl_xor(bi, off, WAVE);
                if (better(d2, i2, bd, bi)) {
                    bd = d2;
                    bi = i2;
                }
            }
            if (lane == 0) {
                cb_D[(size_t)c * CAND_R + r] = bd;
                cb_id[(size_t)c * CAND_R + r] = bi;
            }
            if (id == bi && bd >= 0.f) {  // the winner leaves the race
                dv = -1.f;
                id = INT_MAX;
            }
        }
        if (lane == 0 && j1 > j0)
            atomicAdd(cnt, (unsigned long long)(j1 - j0) * (unsigned)(e - s));
    }
    }
}

constexpr int SEL_T = 256;
constexpr int MAX_K = 256;     // candidates examined per hub and pass
constexpr int SEL_BUF = 2048;  // LDS sort buffer (candidate keys)
constexpr int SEL_W = MAX_K / 64;
constexpr int SEL_CR = 64;     // candidates whose rows are staged in LDS
// candidates read per round of the top-K stream: at most SEL_BUF - MAX_K, so
// a round always fits after a sort has cut buf to K keys
constexpr int SEL_STEP = 4 * SEL_T;
static_assert(SEL_STEP <= SEL_BUF - MAX_K, "top-K stream round too large");

// Sort key of a chunk candidate: farther first, then the smaller input id
// (0 = no candidate).
__device__ __forceinline__ unsigned long long cand_key(float d, int id)
{
    if (!(d >= 0.f))
        return 0ull;
    return ((unsigned long long)__float_as_uint(d) << 32) |
           (unsigned long long)(uint32_t)(0x7FFFFFFF - id);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m)
{
    const unsigned lo = __shfl_xor((unsigned)v, m, WAVE);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), m, WAVE);
    return ((unsigned long long)hi << 32) | lo;
}

// Bitonic sort, descending, of one wave's 512 keys held as x[j] = element
// 64 j + lane: partners 64 or more apart sit in the same lane, nearer ones
// in the same register of another lane (a shuffle).  No barrier.
__device__ __forceinline__ void wave_sort512_desc(unsigned long long (&x)[8])
{
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int k = 2; k <= 512; k <<= 1)
#pragma unroll
        for (int d = k >> 1; d > 0; d >>= 1) {
            if (d >= WAVE) {
                const int m = d / WAVE;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if ((j & m) == 0) {
                        // element 64 j + lane is the lower of the pair
                        const bool up = ((j * WAVE) & k) == 0;
                        const unsigned long long a = x[j], b = x[j | m];
                        const unsigned long long hi = a > b ? a : b, lo = a > b ? b : a;
                        x[j] = up ? hi : lo;
                        x[j | m] = up ? lo : hi;
                    }
            } else {
                const bool lower = (lane & d) == 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool up = ((j * WAVE + lane) & k) == 0;
                    const unsigned long long b = shfl_xor_u64(x[j], d);
                    const unsigned long long a = x[j];
                    const unsigned long long hi = a > b ? a : b, lo = a > b ? b : a;
                    x[j] = lower == up ? hi : lo;
                }
            }
        }
}

// buf[0..tot) (tot <= SEL_BUF = 4 x 512) to its min(K, tot) largest keys in
// descending order at buf[0..): every wave sorts a 512-key segment in
// registers and writes it back, then the four sorted segments are merged by
// rank.  out: LDS of MAX_K keys.  Called by the whole work-group.
__device__ void topk_sorted(unsigned long long *buf, int tot, int K,
                            unsigned long long *out)
{
    static_assert(SEL_BUF == 4 * 512 && SEL_T == 256, "four waves of 512 keys");
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (tot <= WAVE) {
        // a small hub: one wave sorts a key per lane (no merge)
        if (w == 0) {
            unsigned long long v = lane < tot ? buf[lane] : 0ull;
            for (int k = 2; k <= WAVE; k <<= 1)
                for (int d = k >> 1; d > 0; d >>= 1) {
                    const unsigned long long o = shfl_xor_u64(v, d);
                    const bool lower = (lane & d) == 0, up = (lane & k) == 0;
                    const unsigned long long hi = o > v ? o : v, lo = o > v ? v : o;
                    v = lower == up ? hi : lo;
                }
            if (lane < tot)
                buf[lane] = v;
        }
        __syncthreads();
        return;
    }
    if (w * 512 < tot) {  // a segment wholly past tot holds no key: no sort
        unsigned long long x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = w * 512 + j * WAVE + lane;
            x[j] = i < tot ? buf[i] : 0ull;
        }
        wave_sort512_desc(x);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            buf[w * 512 + j * WAVE + lane] = x[j];
    }
    __syncthreads();
    const int nk = min(K, tot);
    // Merge by rank: the best nk keys are among the first nk of each sorted
    // segment (whose own keys, all nonzero, lead it); a key's rank in the
    // union is its index plus the keys above it in the other segments
    // (binary search; keys are distinct), and the keys ranked below nk go
    // to out.
    int cnt[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        cnt[q] = min(nk, max(0, min(512, tot - q * 512)));
    for (int c = threadIdx.x; c < 4 * nk; c += SEL_T) {
        const int q = c / nk, i = c % nk;
        if (i >= cnt[q])
            continue;
        const unsigned long long v = buf[q * 512 + i];
        int rank = i;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            if (o == q)
                continue;
            int lo = 0, hi = cnt[o];  // keys of segment o above v: [0, lo)
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (buf[o * 512 + mid] > v)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            rank += lo;
        }
        if (rank < nk)
            out[rank] = v;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nk; r += SEL_T)
        buf[r] = out[r];
    __syncthreads();
}

// Top-K (K <= MAX_K) of the keys key(v), v in [0, nv), for the whole
// work-group: the keys stream through once; a key enters buf only when it is
// above thr, the K-th best key of the last sort (keys are distinct), and buf
// is sorted and cut to its best K only when it fills.  Returns nk <= K with
// buf[0..nk) the best keys in descending order.
template <class KeyF>
__device__ int topk_stream(long long nv, int K, KeyF key, unsigned long long *buf,
                           int *fill_s, unsigned long long *out)
{
    if (threadIdx.x == 0)
        *fill_s = 0;
    unsigned long long thr = 0ull;  // no candidate has key 0
    int nk = 0;
    __syncthreads();
    auto compact = [&]() {
        const int tot = *fill_s;
        topk_sorted(buf, tot, K, out);
        nk = min(K, tot);
        if (nk == K)
            thr = buf[K - 1];
        __syncthreads();
        if (threadIdx.x == 0)
            *fill_s = nk;
        __syncthreads();
    };
    for (long long base = 0; base < nv; base += SEL_STEP) {
#pragma unroll
        for (int r = 0; r < SEL_STEP / SEL_T; ++r) {
            const long long v = base + r * SEL_T + threadIdx.x;
            if (v < nv) {
                const unsigned long long kv = key(v);
                if (kv > thr)
                    buf[atomicAdd(fill_s, 1)] = kv;  // *fill_s <= SEL_BUF - SEL_STEP before
            }
        }
        __syncthreads();
        if (*fill_s > SEL_BUF - SEL_STEP)
            compact();
    }
    compact();
    return nk;
}

// The K largest of nv <= SEL_RANK keys (0: no candidate; the others are
// distinct), in descending order in buf[0 .. nk), by rank: every key counts
// the keys above it (a broadcast read per key of the buffer).  Returns nk.
constexpr int SEL_RANK = 512;
template <class KeyF>
__device__ int topk_rank(int nv, int K, KeyF key, unsigned long long *buf,
                         unsigned long long *out, int *cnt_s)
{
    if (threadIdx.x == 0)
        *cnt_s = 0;
    for (int v = threadIdx.x; v < nv; v += SEL_T)
        buf[v] = key(v);
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += SEL_T) {
        const unsigned long long k = buf[v];
        if (!k)
            continue;
        atomicAdd(cnt_s, 1);
        int r = 0;
        // eight reads in flight (the buffer's tail past nv is never read)
        int u = 0;
        for (; u + 8 <= nv; u += 8) {
#pragma unroll
            for (int o = 0; o < 8; ++o)
                r += buf[u + o] > k;
        }
        for (; u < nv; ++u)
            r += buf[u] > k;
        if (r < K)
            out[r] = k;
    }
    __syncthreads();
    const int nk = min(K, *cnt_s);
    for (int r = threadIdx.x; r < nk; r += SEL_T)
        buf[r] = out[r];
    __syncthreads();
    return nk;
}

// Candidate slices of a hub with many candidates (more than SEL_PRE): nsl
// slices of len candidates each (the last may be shorter); 0 when the hub
// streams its candidates whole.
constexpr int SEL_SL = 8;                // slices per hub at most
constexpr long long SEL_PRE = 2 * SEL_STEP;
__device__ __forceinline__ void sel_slices(long long ncand, int &nsl, long long &len)
{
    nsl = ncand > SEL_PRE ? (int)min<long long>(SEL_SL, (ncand + SEL_STEP - 1) / SEL_STEP) : 0;
    len = nsl ? (ncand + nsl - 1) / nsl : 0;
}

// Pre-selection for hubs with many candidates, SEL_SL work-groups per hub:
// slice s keeps its K best candidates in its own first K slots (the rest of
// those slots become "no candidate"), so k_select streams nsl x K keys
// instead of all.  The K best of the hub are among them (keys are distinct).
__global__ void __launch_bounds__(SEL_T)
k_select_pre(Hubs hb, int H, float *__restrict__ cb_D, int32_t *__restrict__ cb_id, int kmax)
{
    __shared__ unsigned long long buf[SEL_BUF], out[MAX_K];
    __shared__ int fill_s;
    const int K = min(kmax, MAX_K);
    for (long long w = blockIdx.x; w < (long long)H * SEL_SL; w += gridDim.x) {
        const int h = (int)(w / SEL_SL), sl = (int)(w % SEL_SL);
        if (!hb.act[h])
            continue;
        const int R = cand_per_chunk(hb.ce[h] - hb.cb[h], kmax);
        const long long c0 = (long long)hb.cb[h] * R, c1 = (long long)hb.ce[h] * R;
        int nsl;
        long long len;
        sel_slices(c1 - c0, nsl, len);
        if (sl >= nsl)
            continue;
        const long long qs = c0 + sl * len, qe = min(c1, qs + len);
        auto at = [&](long long q) { return (size_t)(q / R) * CAND_R + (size_t)(q % R); };
        const int nk = topk_stream(
            qe - qs, K,
            [&](long long v) { const size_t a = at(qs + v); return cand_key(cb_D[a], cb_id[a]); },
            buf, &fill_s, out);
        for (int j = threadIdx.x; j < K; j += SEL_T)
            if (qs + j < qe) {
                const size_t a = at(qs + j);
                if (j < nk) {
                    cb_D[a] = __uint_as_float((uint32_t)(buf[j] >> 32));
                    cb_id[a] = 0x7FFFFFFF - (int)(uint32_t)buf[j];
                } else {
                    cb_D[a] = -1.f;
                    cb_id[a] = INT_MAX;
                }
            }
        __syncthreads();  // buf is reused by the next slice
    }
}

// One net-selection pass for every active hub (one work-group per hub): the
// up to kmax farthest chunk candidates, in order (distance descending, id
// ascending), are accepted greedily when more than 2^{l-1} from every
// candidate accepted before them in this pass.  The pairwise conflicts of
// the candidates are evaluated in parallel, then the greedy scan runs on
// bit masks.
template <int M>
__global__ void __launch_bounds__(SEL_T)
k_select(Pts P, Hubs hb, int H, int32_t *__restrict__ cent,
         const float *__restrict__ cb_D, const int32_t *__restrict__ cb_id,
         const LevelTab *__restrict__ tab, int kmax, int32_t *__restrict__ qnext,
         int32_t *__restrict__ qnext_len, unsigned long long *__restrict__ cnt)
{
    __shared__ unsigned long long buf[SEL_BUF], out[MAX_K];
    __shared__ unsigned long long conf[MAX_K][SEL_W];
    __shared__ __align__(16) float crow[SEL_CR * (UPD_D + 4)];  // staged candidate rows
    __shared__ int acc[MAX_K];
    __shared__ int nacc_s, nk_s, qb_s, fill_s;
    const int K = min(kmax, MAX_K);
    for (int h = blockIdx.x; h < H; h += gridDim.x) {
    if (!hb.act[h])
        continue;
    const int R = cand_per_chunk(hb.ce[h] - hb.cb[h], kmax);
    const long long c0 = (long long)hb.cb[h] * R, c1 = (long long)hb.ce[h] * R;
    const int b = hb.b[h], m0 = hb.m[h];
    const Thr T = tab->t[hb.lvl[h] - 1 + LOFF];

    // ---- top-K candidates ------------------------------------------------
    // (a hub with many candidates streams its slices' pre-selected K each)
    int nsl;
    long long len;
    sel_slices(c1 - c0, nsl, len);
    const long long nv = nsl ? (long long)nsl * K : c1 - c0;
    auto ckey = [&](long long v) -> unsigned long long {
        const long long q = nsl ? c0 + (v / K) * len + (v % K) : c0 + v;
        if (q >= c1 || (nsl && (v % K) >= len))
            return 0ull;
        const size_t a = (size_t)(q / R) * CAND_R + (size_t)(q % R);
        return cand_key(cb_D[a], cb_id[a]);
    };
    int nk = nv <= SEL_RANK ? topk_rank((int)nv, K, ckey, buf, out, &fill_s)
                            : topk_stream(nv, K, ckey, buf, &fill_s, out);
    if (threadIdx.x == 0)
        nk_s = nk;
    for (int i = threadIdx.x; i < MAX_K * SEL_W; i += SEL_T)
        conf[i / SEL_W][i % SEL_W] = 0ull;
    __syncthreads();
    nk = nk_s;

    // ---- pairwise conflicts (j < i): within 2^{l-1} ----------------------
    // Vector rows of up to SEL_CR candidates are staged in LDS first (rows
    // padded by 4 floats: neighbouring rows start in different banks) and
    // tested in 2 x 2 blocks; the FP32 key is that of sqdiff_key either way.
    unsigned long long tests = 0;
    const bool lds_rows = (M == M_L2 || M == M_ANG) && P.dp <= UPD_D && nk <= SEL_CR;
    const int ldr = P.dp + 4;
    if (lds_rows) {
        const float *X = M == M_ANG ? P.xn : P.x;
        const int dp = P.dp, q4 = dp / 4;
        // float4 pieces, every load issued before the first store (at most
        // SEL_CR rows of UPD_D floats: eight pieces per thread)
        constexpr int SU = SEL_CR * UPD_D / 4 / SEL_T;
        float4 v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int e = threadIdx.x + u * SEL_T;
            if (e < nk * q4) {
                const int r = e / q4, c4 = e - r * q4;
                const int id = 0x7FFFFFFF - (int)(uint32_t)buf[r];
                v[u] = *reinterpret_cast<const float4 *>(X + (size_t)id * dp + 4 * c4);
            }
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int e = threadIdx.x + u * SEL_T;
            if (e < nk * q4) {
                const int r = e / q4, c4 = e - r * q4;
                *reinterpret_cast<float4 *>(crow + r * ldr + 4 * c4) = v[u];
            }
        }
        __syncthreads();
        // 2 x 2 blocks of the triangle (rows 2 bi, 2 bi + 1 against columns
        // 2 bj, 2 bj + 1, bj <= bi): four keys from four row reads, each
        // summed exactly as sqdiff_key sums it
        const int nb = (nk + 1) / 2;
        for (int q = threadIdx.x; q < nb * (nb + 1) / 2; q += SEL_T) {
            int bi = (int)((sqrtf(1.0f + 8.0f * (float)q) - 1.0f) * 0.5f);
            while (bi * (bi + 1) / 2 > q)
                --bi;
            while ((bi + 1) * (bi + 2) / 2 <= q)
                ++bi;
            const int bj = q - bi * (bi + 1) / 2;
            const int i0 = 2 * bi, j0 = 2 * bj;
            const float *r0 = crow + i0 * ldr, *r1 = crow + min(i0 + 1, nk - 1) * ldr;
            const float *c0 = crow + j0 * ldr, *c1 = crow + min(j0 + 1, nk - 1) * ldr;
            float4 s00 = {0.f, 0.f, 0.f, 0.f}, s01 = s00, s10 = s00, s11 = s00;
            auto acc = [](float4 &t, const float4 &x, const float4 &y) {
                const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z, d3 = x.w - y.w;
                t.x = fmaf(d0, d0, t.x);
                t.y = fmaf(d1, d1, t.y);
                t.z = fmaf(d2, d2, t.z);
                t.w = fmaf(d3, d3, t.w);
            };
            for (int k = 0; k < P.dp; k += 4) {
                const float4 a0 = *reinterpret_cast<const float4 *>(r0 + k);
                const float4 a1 = *reinterpret_cast<const float4 *>(r1 + k);
                const float4 b0 = *reinterpret_cast<const float4 *>(c0 + k);
                const float4 b1 = *reinterpret_cast<const float4 *>(c1 + k);
                acc(s00, a0, b0);
                acc(s01, a0, b1);
                acc(s10, a1, b0);
                acc(s11, a1, b1);
            }
            auto test = [&](int i, int j, const float4 &t) {
                if (i >= nk || j >= i)
                    return;
                const int a = 0x7FFFFFFF - (int)(uint32_t)buf[i];
                const int c = 0x7FFFFFFF - (int)(uint32_t)buf[j];
                ++tests;
                const float k = (t.x + t.y) + (t.z + t.w);
                if (within<M>(P, a, c, k, T, cnt + 1))
                    atomicOr(&conf[i][j >> 6], 1ull << (j & 63));
            };
            test(i0, j0, s00);
            test(i0, j0 + 1, s01);
            test(i0 + 1, j0, s10);
            test(i0 + 1, j0 + 1, s11);
        }
    } else {
        // pairs j < i enumerated over the triangle: q = i (i - 1) / 2 + j
        for (int q = threadIdx.x; q < nk * (nk - 1) / 2; q += SEL_T) {
            int i = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
            while (i * (i - 1) / 2 > q)
                --i;
            while ((i + 1) * i / 2 <= q)
                ++i;
            const int j = q - i * (i - 1) / 2;
            const int a = 0x7FFFFFFF - (int)(uint32_t)buf[i];
            const int c = 0x7FFFFFFF - (int)(uint32_t)buf[j];
            ++tests;
            if (within<M>(P, a, c, key32<M>(P, a, c), T, cnt + 1))
                atomicOr(&conf[i][j >> 6], 1ull << (j & 63));
        }
    }
    __syncthreads();

    // ---- greedy acceptance in candidate order ------------------------------
    if (nk <= WAVE) {
        // one wave: lane i holds candidate i's conflicts with the ones
        // before it, the scan runs on scalar registers, and the accepted
        // candidates take their places by a prefix count
        if (threadIdx.x < WAVE) {
            const int l = threadIdx.x;
            const unsigned long long ci = l < nk ? conf[l][0] : 0ull;
            const unsigned clo = (unsigned)ci, chi = (unsigned)(ci >> 32);
            unsigned long long am = 0ull;
            for (int i = 0; i < nk; ++i) {
                const unsigned long long c =
                    ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)chi, i) << 32) |
                    (unsigned)__builtin_amdgcn_readlane((int)clo, i);
                if ((c & am) == 0ull)
                    am |= 1ull << i;
            }
            if (l < nk && ((am >> l) & 1ull)) {
                const unsigned long long below = l == 0 ? 0ull : (~0ull >> (WAVE - l));
                acc[__popcll(am & below)] = 0x7FFFFFFF - (int)(uint32_t)buf[l];
            }
            if (l == 0)
                nacc_s = __popcll(am);
        }
    } else if (threadIdx.x == 0) {
        unsigned long long am[SEL_W];
#pragma unroll
        for (int w = 0; w < SEL_W; ++w)
            am[w] = 0ull;
        int na = 0;
        for (int i = 0; i < nk; ++i) {
            bool ok = true;
#pragma unroll
            for (int w = 0; w < SEL_W; ++w)
                ok &= (conf[i][w] & am[w]) == 0ull;
            if (ok) {
                am[i >> 6] |= 1ull << (i & 63);
                acc[na++] = 0x7FFFFFFF - (int)(uint32_t)buf[i];
            }
        }
        nacc_s = na;
    }
    __syncthreads();
    const int nacc = nacc_s;
    for (int a = threadIdx.x; a < nacc; a += SEL_T)
        cent[b + m0 + a] = acc[a];
    tests = wave_sum(tests);
    if ((threadIdx.x & (WAVE - 1)) == 0 && tests)
        atomicAdd(cnt, tests);
    if (threadIdx.x == 0) {
        hb.ma[h] = m0;
        hb.m[h] = m0 + nacc;
        if (nacc == 0)
            hb.act[h] = 0;
        else  // the hub's chunks go to the next pass's queue
            qb_s = atomicAdd(qnext_len, hb.ce[h] - hb.cb[h]);
    }
    __syncthreads();
    if (nacc > 0)
        for (int i = threadIdx.x; i < hb.ce[h] - hb.cb[h]; i += SEL_T)
            qnext[qb_s + i] = hb.cb[h] + i;
    __syncthreads();
    }
}

__global__ void k_iota(int32_t *__restrict__ q, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x)
        q[i] = i;
}

// ----------------------------------------------------------- partition ---

__global__ void __launch_bounds__(CH)
k_part_keys(const int32_t *__restrict__ ch_hub, const int32_t *__restrict__ ch_s,
            const int32_t *__restrict__ ch_e, const int32_t *__restrict__ ch_k,
            int NC, const int32_t *__restrict__ child_base,
            const int32_t *__restrict__ L, uint32_t *__restrict__ key,
            uint32_t *__restrict__ val)
{
    for (int c = blockIdx.x; c < NC; c += gridDim.x) {
        const int p = ch_s[c] + threadIdx.x;
        if (p < ch_e[c]) {
            const int k = ch_k[c] + threadIdx.x;
            key[k] = (uint32_t)(child_base[ch_hub[c]] + L[p]);
            val[k] = (uint32_t)p;
        }
    }
}

__global__ void k_part_gather(const uint32_t *__restrict__ src, int NH,
                              const int32_t *__restrict__ perm,
                              const float *__restrict__ D,
                              int32_t *__restrict__ tperm, float *__restrict__ tD)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NH)
        return;
    const int s = (int)src[k];
    tperm[k] = perm[s];
    tD[k] = D[s];
}

__global__ void k_part_store(const uint32_t *__restrict__ skey, int NH,
                             const int32_t *__restrict__ hpos,
                             const int32_t *__restrict__ tperm,
                             const float *__restrict__ tD,
                             int32_t *__restrict__ perm, float *__restrict__ D,
                             int32_t *__restrict__ cfirst,
                             int32_t *__restrict__ clast,
                             unsigned *__restrict__ ckmax)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = k < NH;
    uint32_t key = valid ? skey[k] : 0xFFFFFFFFu;
    float d = 0.f;
    if (valid) {
        const int p = hpos[k];
        perm[p] = tperm[k];
        d = tD[k];
        D[p] = d;
        if (k == 0 || skey[k - 1] != key)
            cfirst[key] = p;
        if (k == NH - 1 || skey[k + 1] != key)
            clast[key] = p;
    }
    // maximum aggregated over a wave whose points all belong to one child,
    // then over the work-group's waves of one child (the first rounds have
    // few large children: their atomics on one address would serialise)
    __shared__ uint32_t wkey[4];
    __shared__ float wmax[4];
    const int w = threadIdx.x / WAVE;
    const uint32_t k0 = __shfl(key, 0, WAVE);
    const bool same = __all(key == k0);
    const float m = same ? wave_max(d) : 0.f;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        wkey[w] = same ? k0 : 0xFFFFFFFFu;
        wmax[w] = m;
    }
    if (!same && valid)
        atomicMax(&ckmax[key], __float_as_uint(d));
    __syncthreads();
    if (threadIdx.x == 0) {
        // runs of equal keys among the waves: one atomic per run
        for (int a = 0; a < 4;) {
            int b = a + 1;
            float mm = wmax[a];
            while (b < 4 && wkey[b] == wkey[a]) {
                mm = fmaxf(mm, wmax[b]);
                ++b;
            }
            if (wkey[a] != 0xFFFFFFFFu)
                atomicMax(&ckmax[wkey[a]], __float_as_uint(mm));
            a = b;
        }
    }
}

struct NodeArrays {
    int32_t *center, *level, *cbeg, *ccnt, *pb, *pe;
    float *radius;
};

__global__ void k_children(Hubs hb, int H, int metric, int dp, int zeta,
                           int node_base, const int32_t *__restrict__ child_base,
                           const int32_t *__restrict__ cent,
                           const int32_t *__restrict__ cfirst,
                           const int32_t *__restrict__ clast,
                           const unsigned *__restrict__ ckmax, NodeArrays nd,
                           int32_t *__restrict__ hubflag)
{
    for (int h = blockIdx.x; h < H; h += gridDim.x) {
    const int b = hb.b[h], m = hb.m[h], lv = hb.lvl[h];
    const int cb = child_base[h];
    if (threadIdx.x == 0) {
        const int v = hb.node[h];
        nd.cbeg[v] = node_base + cb;
        nd.ccnt[v] = m;
    }
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const int g = cb + j;
        const int v = node_base + g;
        const int pb = cfirst[g], pe = clast[g] + 1;
        const float km = __uint_as_float(ckmax[g]);
        const float r = radius_from_key(metric, dp, km);
        int l = lv - 1;
        if (r > 0.f)
            l = min(level_of(r), lv - 1);
        nd.center[v] = cent[b + j];
        nd.radius[v] = r;
        nd.level[v] = l;
        nd.pb[v] = pb;
        nd.pe[v] = pe;
        nd.cbeg[v] = 0;
        nd.ccnt[v] = 0;
        hubflag[g] = (pe - pb > zeta && km > 0.f) ? 1 : 0;
    }
    }
}

__global__ void k_next_hubs(int C, int node_base,
                            const int32_t *__restrict__ flag,
                            const int32_t *__restrict__ fscan, NodeArrays nd,
                            Hubs nh, int32_t *__restrict__ cent)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= C || !flag[g])
        return;
    const int q = fscan[g];
    const int v = node_base + g;
    nh.node[q] = v;
    nh.b[q] = nd.pb[v];
    nh.e[q] = nd.pe[v];
    nh.lvl[q] = nd.level[v];
    nh.m[q] = 1;
    nh.ma[q] = 1;
    nh.act[q] = 1;
    cent[nd.pb[v]] = nd.center[v];
}

// Forest: cloud roots are the children 1..C of the virtual vertex 0, each
// centred on the first point of its cloud at its own top level (the smallest
// l with 2^l >= its radius).
__global__ void k_forest_roots(int C, const int32_t *__restrict__ off,
                               const unsigned *__restrict__ kmax, int metric,
                               int dp, int zeta, NodeArrays nd,
                               int32_t *__restrict__ hubflag)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C;
         c += gridDim.x * blockDim.x) {
        const int v = 1 + c;
        const int pb = off[c], pe = off[c + 1];
        const float km = __uint_as_float(kmax[c]);
        const float r = radius_from_key(metric, dp, km);
        const int l = r > 0.f ? level_of(r) : 0;
        nd.center[v] = pb;
        nd.radius[v] = r;
        nd.level[v] = l;
        nd.pb[v] = pb;
        nd.pe[v] = pe;
        nd.cbeg[v] = 0;
        nd.ccnt[v] = 0;
        hubflag[c] = (pe - pb > zeta && km > 0.f) ? 1 : 0;
        atomicMax(&nd.level[0], l + 1);
    }
}

// ------------------------------------------------------------ finalize ---

__global__ void k_inverse(const int32_t *__restrict__ perm, int n,
                          int32_t *__restrict__ inv)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n)
        inv[perm[p]] = p;
}

__global__ void k_center_pos(const int32_t *__restrict__ center,
                             const int32_t *__restrict__ inv, int nn,
                             int32_t *__restrict__ cpos)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < nn)
        cpos[v] = inv[center[v]];
}

// out row p = in row perm[p].  Rows of a multiple of 16 bytes (16-byte
// aligned arrays) move as int4
// chunks of the flattened output (a wave writes 1 KB of consecutive rows
// per store); other rows one element per lane, a wave per row.
template <class T>
__global__ void k_gather_rows(const T *__restrict__ in, const int32_t *__restrict__ perm,
                              int n, int stride, T *__restrict__ out)
{
    const size_t rowb = (size_t)stride * sizeof(T);
    if (rowb % 16 == 0 && (((uintptr_t)in | (uintptr_t)out) & 15) == 0) {
        const unsigned long long q = rowb / 16;
        const unsigned long long tot = (unsigned long long)n * q;
        const int4 *in4 = reinterpret_cast<const int4 *>(in);
        int4 *out4 = reinterpret_cast<int4 *>(out);
        for (unsigned long long f = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
             f < tot; f += (unsigned long long)gridDim.x * blockDim.x) {
            // 32-bit division while the flattened index fits
            const unsigned long long p =
                tot <= 0xFFFFFFFFull ? (unsigned)f / (unsigned)q : f / q;
            out4[f] = in4[(size_t)perm[p] * q + (f - p * q)];
        }
        return;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int p = blockIdx.x * wpb + threadIdx.x / WAVE; p < n;
         p += gridDim.x * wpb) {
        const T *r = in + (size_t)perm[p] * stride;
        T *o = out + (size_t)p * stride;
        for (int k = lane; k < stride; k += WAVE)
            o[k] = r[k];
    }
}

// ---- query tree: packs of consecutive sibling leaf blocks ----------------

// One wave per vertex: its children are read 64 at a time (one per lane,
// coalesced), and the next-fit walk over them (a run of consecutive leaf
// blocks grows while its points fit in P; a non-leaf child ends the run)
// runs on scalar registers, one child per step, marking the children that
// open a pack.  Every query-tree kid (a non-leaf child or a new pack) then
// takes its slot from a prefix count over the lanes.
struct QtChunk {
    uint64_t open;  // lanes whose child opens a new pack
    uint64_t kid;   // lanes whose child is a query-tree kid (non-leaf or open)
};
__device__ __forceinline__ QtChunk qt_walk(int cnt, bool leaf, int sz, int P, int &run)
{
    const uint64_t leafm = __ballot(leaf);
    uint64_t open = 0;
    for (int j = 0; j < cnt; ++j) {
        if (!((leafm >> j) & 1ull)) {
            run = -1;
            continue;
        }
        const int s = __builtin_amdgcn_readlane(sz, j);
        if (run >= 0 && run + s <= P) {
            run += s;
        } else {
            open |= 1ull << j;
            run = s;
        }
    }
    const uint64_t valid = cnt >= WAVE ? ~0ull : ((1ull << cnt) - 1);
    return QtChunk{open, (~leafm & valid) | open};
}

__global__ void k_qt_count(int nn, const int32_t *__restrict__ ccnt,
                           const int32_t *__restrict__ cbeg,
                           const int32_t *__restrict__ pb,
                           const int32_t *__restrict__ pe, int P, int solo,
                           int32_t *__restrict__ npk, int32_t *__restrict__ nqk)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int v = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x / WAVE) +
                                                      threadIdx.x / WAVE));
    if (v >= nn)
        return;
    const int cc = ccnt[v];
    // leaf children of the forest's virtual root (one per cloud) never share
    // a pack: packs stay inside one cloud
    if (v == solo)
        P = 0;
    int packs = 0, kids = 0, run = -1;
    const int c0 = cc > 0 ? cbeg[v] : 0;
    for (int a0 = 0; a0 < cc; a0 += WAVE) {
        const int cnt = min(WAVE, cc - a0);
        const int u = c0 + a0 + lane;
        const bool in = lane < cnt;
        const bool leaf = in && ccnt[u] == 0;
        const int sz = in ? pe[u] - pb[u] : 0;
        const QtChunk q = qt_walk(cnt, leaf, sz, P, run);
        packs += __popcll(q.open);
        kids += __popcll(q.kid);
    }
    if (lane == 0) {
        npk[v] = packs;
        nqk[v] = kids;
    }
}

__global__ void k_qt_fill(int nn, const int32_t *__restrict__ ccnt,
                          const int32_t *__restrict__ cbeg,
                          const int32_t *__restrict__ pb,
                          const int32_t *__restrict__ pe,
                          const int32_t *__restrict__ cpos,
                          const float *__restrict__ radius, int P, int solo,
                          const int32_t *__restrict__ pkoff,
                          const int32_t *__restrict__ kidoff,
                          int32_t *__restrict__ q_cpos, float *__restrict__ q_rad,
                          int32_t *__restrict__ q_pb, int32_t *__restrict__ q_pe,
                          int32_t *__restrict__ q_kbeg,
                          int32_t *__restrict__ q_kcnt,
                          int32_t *__restrict__ q_kids)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int v = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x / WAVE) +
                                                      threadIdx.x / WAVE));
    if (v >= nn)
        return;
    const int cc = ccnt[v];
    // internal vertices keep their own attributes; leaf blocks are not
    // query-tree vertices (they live inside packs)
    if (lane == 0) {
        q_cpos[v] = cpos[v];
        q_rad[v] = radius[v];
        q_pb[v] = pb[v];
        q_pe[v] = pe[v];
        q_kbeg[v] = kidoff[v];
        q_kcnt[v] = kidoff[v + 1] - kidoff[v];
    }
    if (cc == 0)
        return;
    if (v == solo)
        P = 0;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (WAVE - lane));  // lanes < lane
    int pk0 = nn + pkoff[v] - 1;  // id of the current pack
    int kd0 = kidoff[v];
    int run = -1;
    const int c0 = cbeg[v];
    for (int a0 = 0; a0 < cc; a0 += WAVE) {
        const int cnt = min(WAVE, cc - a0);
        const int u = c0 + a0 + lane;
        const bool in = lane < cnt;
        const bool leaf = in && ccnt[u] == 0;
        const int pbk = in ? pb[u] : 0, pek = in ? pe[u] : 0;
        const QtChunk q = qt_walk(cnt, leaf, pek - pbk, P, run);
        // this lane's pack (the last one opened at or before it) and slot
        const int pk = pk0 + __popcll(q.open & (below | (1ull << lane)));
        const int kd = kd0 + __popcll(q.kid & below);
        if (in && !leaf)
            q_kids[kd] = u;
        if ((q.open >> lane) & 1ull) {
            q_kids[kd] = pk;
            q_cpos[pk] = cpos[u];
            q_pb[pk] = pbk;
            q_kbeg[pk] = 0;
            q_kcnt[pk] = 0;
            q_rad[pk] = 0.f;
        }
        // the pack's end: written by its last leaf in this chunk (a run
        // that goes on in the next chunk is written again there, after this
        // store has completed)
        const bool last =
            lane == cnt - 1 || (lane < WAVE - 1 && ((q.kid >> (lane + 1)) & 1ull));
        if (leaf && last)
            q_pe[pk] = pek;
        pk0 += __popcll(q.open);
        kd0 += __popcll(q.kid);
        if (a0 + WAVE < cc)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
}

// Radius of each pack: the largest key from its centre to its points.
template <int M>
__global__ void k_pack_radius(Pts P, int first, int npk,
                              const int32_t *__restrict__ q_cpos,
                              const int32_t *__restrict__ q_pb,
                              const int32_t *__restrict__ q_pe, int dp,
                              float *__restrict__ q_rad)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int k = blockIdx.x * wpb + threadIdx.x / WAVE; k < npk;
         k += gridDim.x * wpb) {
        const int q = first + k;
        const int c = q_cpos[q];
        float m = 0.f;
        for (int p = q_pb[q] + lane; p < q_pe[q]; p += WAVE)
            m = fmaxf(m, key32<M>(P, c, p));
        m = wave_max(m);
        if (lane == 0)
            q_rad[q] = radius_from_key(M, dp, m);
    }
}

// -------------------------------------------------------------- driver ---

static int bitlen(uint32_t v)
{
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Ingest (input order): rows validated (finite, within coord_bound; no zero
// angular row; string symbols < MAX_SIGMA) and padded, plus the per-metric
// preprocessing (unit rows, string lengths and match masks).  Sets T->sigma
// and T->W for strings.  The returned view reads the caller's rows for
// Hamming and Levenshtein.
template <int M>
static Pts ingest_impl(fnn_tree *T, const void *points, Scratch &S)
{
    hipStream_t st = S.stream();
    const int n = (int)T->n;
    int *err = S.get<int>(1);
    fill(err, 0, 1, st);
    Pts P{};
    P.metric = M;
    P.n = n;
    P.dim = T->dim;
    P.dp = T->dp;
    float *x_in = nullptr, *xn_in = nullptr;
    if (M == M_L2 || M == M_ANG) {
        if (M == M_L2 && T->dim == T->dp && ((uintptr_t)points & 15) == 0) {
            // unpadded, aligned rows: checked, then read in place (the
            // caller's rows stay unchanged during the call)
            const long long n4 = (long long)n * T->dp / 4;
            FNN_LAUNCH(k_ingest_flat, dim3(grid_cap(n4, 256 * 8, 8192)), dim3(256), 0, st,
                       (const float4 *)points, n4, coord_bound(T->dim), (float4 *)nullptr,
                       err);
            P.x = (const float *)points;
        } else {
            x_in = S.get<float>((size_t)n * T->dp);
            if (M == M_ANG)
                xn_in = S.get<float>((size_t)n * T->dp);
            FNN_LAUNCH(k_ingest_vec, dim3(grid_cap(n, 4, 16384)), dim3(256), 0, st,
                       (const float *)points, n, T->dim, T->dp,
                       M == M_ANG ? 1 : 0, coord_bound(T->dim), x_in, xn_in, err);
            P.x = x_in;
            P.xn = xn_in;
        }
    } else if (M == M_HAM) {
        P.h = (const uint64_t *)points;
    } else {
        int32_t *len_in = S.get<int32_t>(n);
        int *sig = S.get<int>(1);
        fill(sig, 1, 1, st);
        FNN_LAUNCH(k_ingest_lev, dim3(cdiv(n, 256)), dim3(256), 0, st,
                           (const uint8_t *)points, n, T->dim, len_in, sig, err);
        int e = read_scalar(err, st);
        if (e)
            fail(FNN_EINVAL, "Levenshtein input has a symbol >= %d", MAX_SIGMA);
        T->sigma = read_scalar(sig, st);
        T->W = (T->dim + 63) / 64;
        uint64_t *peq_in = S.get<uint64_t>((size_t)n * T->sigma * T->W);
        FNN_LAUNCH(k_peq, dim3(cdiv(n, 256)), dim3(256), 0, st,
                           (const uint8_t *)points, len_in, n, T->dim, T->sigma,
                           T->W, peq_in);
        P.s = (const uint8_t *)points;
        P.len = len_in;
        P.peq = peq_in;
        P.sigma = T->sigma;
        P.W = T->W;
    }
    {
        int e = read_scalar(err, st);
        if (e & ERR_INPUT)
            fail(FNN_EINVAL, M == M_ANG ? "input has a NaN/Inf coordinate or a zero row"
                                        : "input has a NaN/Inf coordinate");
        if (e & ERR_RANGE)
            fail(FNN_EUNSUPPORTED,
                 "input has a coordinate of magnitude above %g (FP32 squared "
                 "distances could overflow)", (double)coord_bound(T->dim));
    }

    return P;
}

Pts ingest_input(fnn_tree *T, const void *points, Scratch &S)
{
    switch (T->metric) {
    case M_L2:
        return ingest_impl<M_L2>(T, points, S);
    case M_ANG:
        return ingest_impl<M_ANG>(T, points, S);
    case M_HAM:
        return ingest_impl<M_HAM>(T, points, S);
    default:
        return ingest_impl<M_LEV>(T, points, S);
    }
}

template <int M>
static void build_impl(fnn_tree *T, const void *points, Scratch &S)
{
    hipStream_t st = S.stream();
    const int n = (int)T->n;
    int *err = S.get<int>(1);
    fill(err, 0, 1, st);
    unsigned long long *cnt = S.get<unsigned long long>(4);
    fill(cnt, 0ull, 4, st);

    hipEvent_t ev0, ev1;
    FNN_HIP(hipEventCreate(&ev0));
    FNN_HIP(hipEventCreate(&ev1));
    FNN_HIP(hipEventRecord(ev0, st));

    // ---- ingest (input order) -------------------------------------------
    Pts P = ingest_impl<M>(T, points, S);

    LevelTab htab;
    make_level_table(M, T->dp, &htab);
    LevelTab *tab = S.get<LevelTab>(1);
    FNN_HIP(hipMemcpyAsync(tab, &htab, sizeof(LevelTab), hipMemcpyHostToDevice,
                           st));

    // ---- node arrays (at most 2n - 1 vertices) ------------------------------
    const size_t cap = 2 * (size_t)n + 2 + (size_t)T->ncloud;
    NodeArrays nd;
    nd.center = S.get<int32_t>(cap);
    nd.level = S.get<int32_t>(cap);
    nd.cbeg = S.get<int32_t>(cap);
    nd.ccnt = S.get<int32_t>(cap);
    nd.pb = S.get<int32_t>(cap);
    nd.pe = S.get<int32_t>(cap);
    nd.radius = S.get<float>(cap);

    int32_t *perm = S.get<int32_t>(n);
    float *D = S.get<float>(n);
    int32_t *L = S.get<int32_t>(n);
    int32_t *cent = S.get<int32_t>(n);
    int32_t *hpos = S.get<int32_t>(n);
    int32_t *tperm = S.get<int32_t>(n);
    float *tD = S.get<float>(n);
    uint32_t *key = S.get<uint32_t>(n), *val = S.get<uint32_t>(n);
    uint32_t *skey = S.get<uint32_t>(n), *sval = S.get<uint32_t>(n);
    int32_t *cfirst = S.get<int32_t>(n), *clast = S.get<int32_t>(n);
    unsigned *ckmax = S.get<unsigned>(n + 1);
    int32_t *hubflag = S.get<int32_t>(n + 1), *fscan = S.get<int32_t>(n + 2);
    const int maxch = (int)cdiv(n, CH) + n / 2 + 2;  // chunks over all hubs
    int32_t *ch_hub = S.get<int32_t>(maxch), *ch_s = S.get<int32_t>(maxch),
            *ch_e = S.get<int32_t>(maxch), *ch_k = S.get<int32_t>(maxch);
    float *cb_D = S.get<float>((size_t)maxch * CAND_R);
    int32_t *cb_id = S.get<int32_t>((size_t)maxch * CAND_R);
    int32_t *qa = S.get<int32_t>(maxch), *qb = S.get<int32_t>(maxch);
    int32_t *qlen = S.get<int32_t>(2);
    // net-selection passes per graph replay (even: the live queue returns
    // to qa); 1 = one eager pass per host check
    const int GP = T->opt.graph_passes <= 1 ? 1 : (T->opt.graph_passes + 1) / 2 * 2;

    auto alloc_hubs = [&](int cnt_) {
        Hubs hb;
        hb.node = S.get<int32_t>(cnt_);
        hb.b = S.get<int32_t>(cnt_);
        hb.e = S.get<int32_t>(cnt_);
        hb.lvl = S.get<int32_t>(cnt_);
        hb.m = S.get<int32_t>(cnt_);
        hb.ma = S.get<int32_t>(cnt_);
        hb.act = S.get<int32_t>(cnt_);
        hb.cb = S.get<int32_t>(cnt_);
        hb.ce = S.get<int32_t>(cnt_);
        hb.kof = S.get<int32_t>(cnt_);
        return hb;
    };
    const int hub_cap = n / 2 + 2;  // every hub holds more than zeta >= 1 points
    Hubs hubs = alloc_hubs(hub_cap), nhubs = alloc_hubs(hub_cap);
    int32_t *nch = S.get<int32_t>(hub_cap + 1), *hsz = S.get<int32_t>(hub_cap + 1);
    int32_t *choff = S.get<int32_t>(hub_cap + 2), *itemoff = S.get<int32_t>(hub_cap + 2);
    int32_t *child_base = S.get<int32_t>(hub_cap + 2);

    int H = 0;
    int64_t node_count = 1;
    // host staging values stay alive until the synchronisation below
    int32_t zero = 0;
    const int NCL = T->ncloud;
    std::vector<int32_t> offh;
    int32_t v0[5] = {0, 1, NCL, 0, n};
    const float inf = INFINITY;
    int32_t h0[7] = {0, 0, 0, 0, 0, n, 0};
    int32_t one[10] = {0, 0, n, 0, 1, 1, 1, 0, 0, 0};
    float r0 = 0.f;
    if (NCL > 1) {
        // ---- forest: one root per cloud, all clouds share every launch ---
        offh.resize(NCL + 1);
        for (int c = 0; c <= NCL; ++c)
            offh[c] = (int32_t)T->cloud_off_h[c];
        int32_t *off = S.get<int32_t>(NCL + 1);
        FNN_HIP(hipMemcpyAsync(off, offh.data(), sizeof(int32_t) * (NCL + 1),
                               hipMemcpyHostToDevice, st));
        T->pcl = (int32_t *)T->own(sizeof(int32_t) * n);
        FNN_LAUNCH(k_cloud_ids, dim3(grid_for(NCL, 4)), dim3(256), 0, st, off,
                   NCL, T->pcl);
        unsigned *ck = S.get<unsigned>(NCL);
        fill(ck, 0u, NCL, st);
        FNN_LAUNCH((k_forest_keys<M>), dim3(grid_for(n, 256)), dim3(256), 0, st,
                   P, off, T->pcl, perm, D, ck);
        fill(nd.level, INT_MIN, 1, st);
        int32_t *cflag = S.get<int32_t>(NCL + 1), *cscan = S.get<int32_t>(NCL + 2);
        FNN_LAUNCH(k_forest_roots, dim3(grid_for(NCL, 256)), dim3(256), 0, st,
                   NCL, off, ck, M, T->dp, T->opt.zeta, nd, cflag);
        // vertex 0: the virtual root (never part of a query pair)
        FNN_HIP(hipMemcpyAsync(nd.center, &v0[0], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.cbeg, &v0[1], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.ccnt, &v0[2], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.pb, &v0[3], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.pe, &v0[4], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.radius, &inf, 4, hipMemcpyHostToDevice, st));
        scan_i32(cflag, cscan, NCL, S);
        H = read_scalar(cscan + NCL, st);
        if (H > hub_cap)
            fail(FNN_EINTERNAL, "hub capacity exceeded");
        FNN_LAUNCH(k_next_hubs, dim3(cdiv(NCL, 256)), dim3(256), 0, st, NCL, 1,
                   cflag, cscan, nd, hubs, cent);
        node_count = 1 + NCL;
    } else {
        // ---- root: D[p] = d(p, p_0) (Algorithm 1's pre-initialised D) -----
        unsigned *rk = S.get<unsigned>(1);
        fill(rk, 0u, 1, st);
        FNN_LAUNCH((k_root_keys<M>), dim3(cdiv(n, 256)), dim3(256), 0, st,
                           P, perm, D, rk);
        const unsigned r0bits = read_scalar(rk, st);
        float r0key;
        memcpy(&r0key, &r0bits, sizeof r0key);
        r0 = radius_from_key(M, T->dp, r0key);
        const int l0 = r0 > 0.f ? level_of(r0) : 0;
        h0[1] = l0;
        one[3] = l0;
        // root vertex: centre 0, all points
        FNN_HIP(hipMemcpyAsync(nd.center, &h0[0], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.level, &h0[1], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.cbeg, &h0[2], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.ccnt, &h0[3], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.pb, &h0[4], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.pe, &h0[5], 4, hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(nd.radius, &r0, 4, hipMemcpyHostToDevice, st));
        if (n > T->opt.zeta && r0key > 0.f) {
            int32_t *dst[10] = {hubs.node, hubs.b, hubs.e, hubs.lvl, hubs.m,
                                hubs.ma, hubs.act, hubs.cb, hubs.ce, hubs.kof};
            for (int i = 0; i < 10; ++i)
                FNN_HIP(hipMemcpyAsync(dst[i], &one[i], 4, hipMemcpyHostToDevice, st));
            FNN_HIP(hipMemcpyAsync(cent, &zero, 4, hipMemcpyHostToDevice, st));
            H = 1;
        }
    }
    FNN_HIP(hipStreamSynchronize(st));

    int rounds = 0, passes = 0;
    while (H > 0) {
        ++rounds;
        // chunk table of this level's hubs
        FNN_LAUNCH(k_hub_sizes, dim3(cdiv(H, 256)), dim3(256), 0, st,
                           hubs.b, hubs.e, H, nch, hsz);
        scan_i32(nch, choff, H, S);
        scan_i32(hsz, itemoff, H, S);
        int32_t tot[2];
        FNN_HIP(hipMemcpyAsync(&tot[0], choff + H, 4, hipMemcpyDeviceToHost, st));
        FNN_HIP(hipMemcpyAsync(&tot[1], itemoff + H, 4, hipMemcpyDeviceToHost, st));
        FNN_HIP(hipStreamSynchronize(st));
        const int NC = tot[0], NH = tot[1];
        if (NC > maxch || NH > n)
            fail(FNN_EINTERNAL, "chunk table overflow (%d > %d)", NC, maxch);
        FNN_LAUNCH(k_make_chunks, dim3(grid_cap(H, 1, 8192)), dim3(64), 0, st, hubs, H,
                           choff, itemoff, ch_hub, ch_s, ch_e, ch_k);
        FNN_LAUNCH(k_round_init, dim3(grid_cap(NC, 1, 16384)), dim3(CH), 0, st, ch_s,
                   ch_e, ch_k, NC, L, hpos);

        // ---- net selection passes ----------------------------------------
        // Pass p: k_update over the queue of active chunks, k_select writes
        // the next queue.  Once every hub is done both kernels do nothing,
        // so passes can run ahead of the host: G passes are recorded into a
        // graph once per level and replayed until the queue is empty.
        FNN_LAUNCH(k_iota, dim3(grid_for(NC, 256)), dim3(256), 0, st, qa, NC);
        fill(qlen, NC, 1, st);
        const unsigned gu = grid_cap(NC, UPD_W, 4096);
        const size_t upd_lds =
            (M == M_L2 || M == M_ANG) && T->dp <= UPD_D ? sizeof(float) * UPD_K * (T->dp + 4)
                                                        : 16;
        auto pass = [&](hipStream_t s, int k) {
            int32_t *qc = k ? qb : qa, *qx = k ? qa : qb;
            fill(qlen + (1 - k), 0, 1, s);
            FNN_LAUNCH((k_update<M>), dim3(gu), dim3(CH * UPD_W), upd_lds, s, P, ch_hub, ch_s,
                       ch_e, qc, qlen + k, hubs, cent, perm, D, L, tab, cb_D,
                       cb_id, T->opt.kmax, cnt);
            FNN_LAUNCH(k_select_pre, dim3(grid_cap((int64_t)H * SEL_SL, 1, 8192)),
                       dim3(SEL_T), 0, s, hubs, H, cb_D, cb_id, T->opt.kmax);
            FNN_LAUNCH((k_select<M>), dim3(grid_cap(H, 1, 4096)), dim3(SEL_T), 0, s, P,
                       hubs, H, cent, cb_D, cb_id, tab, T->opt.kmax, qx,
                       qlen + (1 - k), cnt);
        };
        if (GP <= 1) {
            for (int k = 0;; k ^= 1) {
                pass(st, k);
                ++passes;
                if (read_scalar(qlen + (1 - k), st) == 0)
                    break;
            }
        } else {
            GraphRun gr;
            gr.begin();
            for (int k = 0; k < GP; ++k)
                pass(gr.cs, k & 1);
            gr.end();
            for (;;) {
                gr.launch(st);
                passes += GP;
                if (read_scalar(qlen, st) == 0)
                    break;
            }
        }

        // ---- partition into children ---------------------------------------
        scan_i32(hubs.m, child_base, H, S);
        const int C = read_scalar(child_base + H, st);
        if (node_count + C > (int64_t)cap)
            fail(FNN_EINTERNAL, "vertex capacity exceeded");
        FNN_LAUNCH(k_part_keys, dim3(grid_cap(NC, 1, 16384)), dim3(CH), 0, st, ch_hub,
                   ch_s, ch_e, ch_k, NC, child_base, L, key, val);
        radix_sort_pairs(key, val, skey, sval, NH, bitlen((uint32_t)C), S);
        FNN_LAUNCH(k_part_gather, dim3(cdiv(NH, 256)), dim3(256), 0, st,
                           sval, NH, perm, D, tperm, tD);
        fill(ckmax, 0u, C, st);
        FNN_LAUNCH(k_part_store, dim3(cdiv(NH, 256)), dim3(256), 0, st,
                           skey, NH, hpos, tperm, tD, perm, D, cfirst, clast,
                           ckmax);
        FNN_LAUNCH(k_children, dim3(grid_cap(H, 1, 8192)), dim3(64), 0, st, hubs, H, M,
                           T->dp, T->opt.zeta, (int)node_count, child_base, cent,
                           cfirst, clast, ckmax, nd, hubflag);
        scan_i32(hubflag, fscan, C, S);
        const int Hn = read_scalar(fscan + C, st);
        if (Hn > hub_cap)
            fail(FNN_EINTERNAL, "hub capacity exceeded");
        FNN_LAUNCH(k_next_hubs, dim3(cdiv(C, 256)), dim3(256), 0, st, C,
                           (int)node_count, hubflag, fscan, nd, nhubs, cent);
        node_count += C;
        std::swap(hubs, nhubs);
        H = Hn;
    }

    // ---- finalize: tree order, vertex centre positions ------------------
    const int nn = (int)node_count;
    T->nnodes = nn;
    T->perm = (int32_t *)T->own(sizeof(int32_t) * n);
    FNN_HIP(hipMemcpyAsync(T->perm, perm, sizeof(int32_t) * n,
                           hipMemcpyDeviceToDevice, st));
    int32_t *inv = S.get<int32_t>(n);
    FNN_LAUNCH(k_inverse, dim3(cdiv(n, 256)), dim3(256), 0, st, perm, n,
                       inv);
    {
        const size_t vb = sizeof(int32_t) * (size_t)nn;
        const size_t sizes[8] = {vb, vb, vb, vb, vb, vb, vb, vb};
        void *v[8];
        T->own_many(sizes, v);
        T->center = (int32_t *)v[0];
        T->center_pos = (int32_t *)v[1];
        T->radius = (float *)v[2];
        T->level = (int32_t *)v[3];
        T->child_begin = (int32_t *)v[4];
        T->child_count = (int32_t *)v[5];
        T->pt_begin = (int32_t *)v[6];
        T->pt_end = (int32_t *)v[7];
    }
    auto cp = [&](void *dst, const void *src, size_t b) {
        FNN_HIP(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, st));
    };
    cp(T->center, nd.center, 4 * (size_t)nn);
    cp(T->radius, nd.radius, 4 * (size_t)nn);
    cp(T->level, nd.level, 4 * (size_t)nn);
    cp(T->child_begin, nd.cbeg, 4 * (size_t)nn);
    cp(T->child_count, nd.ccnt, 4 * (size_t)nn);
    cp(T->pt_begin, nd.pb, 4 * (size_t)nn);
    cp(T->pt_end, nd.pe, 4 * (size_t)nn);
    FNN_LAUNCH(k_center_pos, dim3(cdiv(nn, 256)), dim3(256), 0, st,
                       nd.center, inv, nn, T->center_pos);

    // point data in tree order
    Pts Q = P;
    if (M == M_L2 || M == M_ANG) {
        T->x = (float *)T->own(sizeof(float) * (size_t)n * T->dp);
        FNN_LAUNCH((k_gather_rows<float>), dim3(grid_cap(n, 4, 16384)), dim3(256), 0,
                           st, P.x, perm, n, T->dp, T->x);
        Q.x = T->x;
        if (M == M_ANG) {
            T->xn = (float *)T->own(sizeof(float) * (size_t)n * T->dp);
            FNN_LAUNCH((k_gather_rows<float>), dim3(grid_cap(n, 4, 16384)),
                               dim3(256), 0, st, P.xn, perm, n, T->dp, T->xn);
            Q.xn = T->xn;
        }
    } else if (M == M_HAM) {
        T->h = (uint64_t *)T->own(sizeof(uint64_t) * (size_t)n * T->dp);
        FNN_LAUNCH((k_gather_rows<uint64_t>), dim3(grid_cap(n, 4, 16384)),
                           dim3(256), 0, st, P.h, perm, n, T->dp, T->h);
        Q.h = T->h;
    } else {
        T->s = (uint8_t *)T->own((size_t)n * T->dp);
        T->len = (int32_t *)T->own(sizeof(int32_t) * n);
        T->peq = (uint64_t *)T->own(sizeof(uint64_t) * (size_t)n * T->sigma * T->W);
        FNN_LAUNCH((k_gather_rows<uint8_t>), dim3(grid_cap(n, 4, 16384)), dim3(256),
                           0, st, P.s, perm, n, T->dp, T->s);
        FNN_LAUNCH((k_gather_rows<int32_t>), dim3(grid_cap(n, 4, 16384)), dim3(256),
                           0, st, P.len, perm, n, 1, T->len);
        FNN_LAUNCH((k_gather_rows<uint64_t>), dim3(grid_cap(n, 4, 16384)),
                           dim3(256), 0, st, P.peq, perm, n, T->sigma * T->W,
                           T->peq);
        Q.s = T->s;
        Q.len = T->len;
        Q.peq = T->peq;
    }

    // ---- query tree with packs ------------------------------------------
    const int PK = T->opt.pack;
    const int solo = NCL > 1 ? 0 : -1;
    int32_t *npk = S.get<int32_t>(nn + 1), *nqk = S.get<int32_t>(nn + 1);
    int32_t *pkoff = S.get<int32_t>(nn + 2), *kidoff = S.get<int32_t>(nn + 2);
    FNN_LAUNCH(k_qt_count, dim3(cdiv(nn, 256 / WAVE)), dim3(256), 0, st, nn,
                       nd.ccnt, nd.cbeg, nd.pb, nd.pe, PK, solo, npk, nqk);
    scan_i32(npk, pkoff, nn, S);
    scan_i32(nqk, kidoff, nn, S);
    int32_t tots[2];
    FNN_HIP(hipMemcpyAsync(&tots[0], pkoff + nn, 4, hipMemcpyDeviceToHost, st));
    FNN_HIP(hipMemcpyAsync(&tots[1], kidoff + nn, 4, hipMemcpyDeviceToHost, st));
    FNN_HIP(hipStreamSynchronize(st));
    int npacks = tots[0], nkids = tots[1];
    const bool root_leaf = (nn == 1);
    if (root_leaf)
        npacks = 1;
    const int nq = nn + npacks;
    T->npacks = npacks;
    T->nq = nq;
    {
        const size_t qb = sizeof(int32_t) * (size_t)nq;
        const size_t sizes[7] = {qb, qb, qb, qb, qb, qb, sizeof(int32_t) * ((size_t)nkids + 1)};
        void *v[7];
        T->own_many(sizes, v);
        T->q_center_pos = (int32_t *)v[0];
        T->q_radius = (float *)v[1];
        T->q_pt_begin = (int32_t *)v[2];
        T->q_pt_end = (int32_t *)v[3];
        T->q_kbeg = (int32_t *)v[4];
        T->q_kcnt = (int32_t *)v[5];
        T->q_kids = (int32_t *)v[6];
    }
    FNN_LAUNCH(k_qt_fill, dim3(cdiv(nn, 256 / WAVE)), dim3(256), 0, st, nn,
                       nd.ccnt, nd.cbeg, nd.pb, nd.pe, T->center_pos, nd.radius, PK,
                       solo, pkoff, kidoff, T->q_center_pos, T->q_radius, T->q_pt_begin,
                       T->q_pt_end, T->q_kbeg, T->q_kcnt, T->q_kids);
    int32_t vals[5] = {0, n, 0, 0, 0};
    if (root_leaf) {
        // the whole set is one leaf block: one pack, the query tree's root
        FNN_HIP(hipMemcpyAsync(T->q_center_pos + nn, T->center_pos, 4,
                               hipMemcpyDeviceToDevice, st));
        FNN_HIP(hipMemcpyAsync(T->q_pt_begin + nn, &vals[0], 4,
                               hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(T->q_pt_end + nn, &vals[1], 4,
                               hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(T->q_kbeg + nn, &vals[2], 4,
                               hipMemcpyHostToDevice, st));
        FNN_HIP(hipMemcpyAsync(T->q_kcnt + nn, &vals[3], 4,
                               hipMemcpyHostToDevice, st));
        T->qroot = nn;
    } else {
        T->qroot = 0;
    }
    if (npacks > 0)
        FNN_LAUNCH((k_pack_radius<M>), dim3(grid_for(npacks, 4)), dim3(256),
                           0, st, Q, nn, npacks, T->q_center_pos, T->q_pt_begin,
                           T->q_pt_end, T->dp, T->q_radius);

    FNN_HIP(hipEventRecord(ev1, st));
    unsigned long long hc[4];
    FNN_HIP(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, st));
    FNN_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    FNN_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    {
        int e = read_scalar(err, st);
        if (e & ERR_INDEX)
            fail(FNN_EINTERNAL, "build index check failed");
    }

    fnn_stats &s = T->stats;
    s.n = n;
    s.nodes = nn;
    s.packs = npacks;
    s.rounds = rounds;
    s.netsel_passes = passes;
    s.build_dist_evals = (int64_t)(hc[0] + n);
    s.fp64_rechecks = (int64_t)hc[1];
    s.build_ms = ms;
    s.total_ms = ms;
    T->depth = rounds;
}

// ------------------------------------------------- two-tree forest ------
//
// A bichromatic query (foreign points against a tree) runs as the self-join
// of a two-cloud forest restricted to pairs across the clouds: vertex 0 is a
// virtual root, the data tree A and the query tree B keep their shapes, and
// the traversal starts from the pair of their query-tree roots.  Only the
// arrays the query reads are assembled: points (tree order, A then B),
// perm (B's input indices shifted by nA), the query tree and the cloud
// tables.  Internal-vertex ids: 0 virtual, then A's (id v -> 1 + v), then
// B's (v -> 1 + nnA + v); packs: A's, then B's, after all internal ids.

__global__ void k_pair_qtree(int nq_src, int nn_src, int vbase, int pbase, int pos_off,
                             int kid_off, const int32_t *__restrict__ cpos,
                             const float *__restrict__ rad, const int32_t *__restrict__ pb,
                             const int32_t *__restrict__ pe, const int32_t *__restrict__ kbeg,
                             const int32_t *__restrict__ kcnt, int32_t *__restrict__ ocpos,
                             float *__restrict__ orad, int32_t *__restrict__ opb,
                             int32_t *__restrict__ ope, int32_t *__restrict__ okbeg,
                             int32_t *__restrict__ okcnt)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nq_src;
         v += gridDim.x * blockDim.x) {
        const int d = v < nn_src ? vbase + v : pbase + (v - nn_src);
        ocpos[d] = cpos[v] + pos_off;
        orad[d] = rad[v];
        opb[d] = pb[v] + pos_off;
        ope[d] = pe[v] + pos_off;
        okbeg[d] = kbeg[v] + kid_off;
        okcnt[d] = kcnt[v];
    }
}

__global__ void k_pair_kids(int nk, int nn_src, int vbase, int pbase,
                            const int32_t *__restrict__ kids, int32_t *__restrict__ okids)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nk;
         i += gridDim.x * blockDim.x) {
        const int v = kids[i];
        okids[i] = v < nn_src ? vbase + v : pbase + (v - nn_src);
    }
}

__global__ void k_add_i32(const int32_t *__restrict__ src, int n, int add,
                          int32_t *__restrict__ dst)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = src[i] + add;
}

static int total_kids(const fnn_tree *T, hipStream_t s)
{
    std::vector<int32_t> kb(T->nq), kc(T->nq);
    FNN_HIP(hipMemcpyAsync(kb.data(), T->q_kbeg, sizeof(int32_t) * T->nq,
                           hipMemcpyDeviceToHost, s));
    FNN_HIP(hipMemcpyAsync(kc.data(), T->q_kcnt, sizeof(int32_t) * T->nq,
                           hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    int64_t m = 0;
    for (int64_t v = 0; v < T->nq; ++v)
        if (kc[v] > 0)
            m = std::max<int64_t>(m, (int64_t)kb[v] + kc[v]);
    return (int)m;
}

// Match-mask table of n strings widened from sigma_in to sigma_out symbols
// (a symbol a string does not hold has an empty mask).
__global__ void k_widen_peq(const uint64_t *__restrict__ in, int n, int sig_in, int W,
                            int sig_out, uint64_t *__restrict__ out)
{
    const long long tot = (long long)n * sig_out * W;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / ((long long)sig_out * W);
        const int r = (int)(e % ((long long)sig_out * W));
        const int c = r / W, w = r % W;
        out[e] = c < sig_in ? in[(i * sig_in + c) * W + w] : 0ull;
    }
}

fnn_tree *forest_pair(const fnn_tree *A, const fnn_tree *B, Scratch &S)
{
    hipStream_t s = S.stream();
    if (A->metric != B->metric || A->dp != B->dp || A->dim != B->dim || A->W != B->W)
        fail(FNN_EINVAL, "query rows do not match the tree's metric and dimension "
             "(metric %d / %d, dim %d / %d)", A->metric, B->metric, A->dim, B->dim);
    if (A->ncloud != 1 || B->ncloud != 1)
        fail(FNN_EUNSUPPORTED, "bichromatic queries need single-cloud trees");
    if ((int64_t)A->n + B->n >= INT32_MAX)
        fail(FNN_EUNSUPPORTED, "too many points");
    fnn_tree *F = new fnn_tree();
    try {
        const int nA = (int)A->n, nB = (int)B->n, n = nA + nB;
        F->metric = A->metric;
        F->n = n;
        F->dim = A->dim;
        F->dp = A->dp;
        F->W = A->W;
        // strings: one alphabet for both sets (each built its table for its
        // own largest symbol)
        F->sigma = std::max(A->sigma, B->sigma);
        F->opt = A->opt;
        auto cat = [&](const void *a, const void *b, size_t row_bytes) -> void * {
            if (!a)
                return nullptr;
            char *d = (char *)F->own(row_bytes * (size_t)n);
            FNN_HIP(hipMemcpyAsync(d, a, row_bytes * nA, hipMemcpyDeviceToDevice, s));
            FNN_HIP(hipMemcpyAsync(d + row_bytes * nA, b, row_bytes * nB,
                                   hipMemcpyDeviceToDevice, s));
            return d;
        };
        F->x = (float *)cat(A->x, B->x, sizeof(float) * A->dp);
        F->xn = (float *)cat(A->xn, B->xn, sizeof(float) * A->dp);
        F->h = (uint64_t *)cat(A->h, B->h, sizeof(uint64_t) * A->dp);
        F->s = (uint8_t *)cat(A->s, B->s, (size_t)A->dp);
        F->len = (int32_t *)cat(A->len, B->len, sizeof(int32_t));
        if (A->peq) {
            const int sg = F->sigma, W = A->W;
            F->peq = (uint64_t *)F->own(sizeof(uint64_t) * (size_t)n * sg * W);
            FNN_LAUNCH(k_widen_peq, dim3(grid_cap((int64_t)nA * sg * W, 256, 8192)),
                       dim3(256), 0, s, A->peq, nA, A->sigma, W, sg, F->peq);
            FNN_LAUNCH(k_widen_peq, dim3(grid_cap((int64_t)nB * sg * W, 256, 8192)),
                       dim3(256), 0, s, B->peq, nB, B->sigma, W, sg,
                       F->peq + (size_t)nA * sg * W);
        }
        F->perm = (int32_t *)F->own(sizeof(int32_t) * n);
        FNN_HIP(hipMemcpyAsync(F->perm, A->perm, sizeof(int32_t) * nA,
                               hipMemcpyDeviceToDevice, s));
        FNN_LAUNCH(k_add_i32, dim3(grid_cap(nB, 256, 4096)), dim3(256), 0, s, B->perm, nB, nA,
                   F->perm + nA);

        // query tree
        const int nnA = (int)A->nnodes, nnB = (int)B->nnodes;
        const int npA = (int)A->npacks, npB = (int)B->npacks;
        const int nn = 1 + nnA + nnB;
        const int nq = nn + npA + npB;
        const int kA = total_kids(A, s), kB = total_kids(B, s);
        F->nnodes = nn;
        F->npacks = npA + npB;
        F->nq = nq;
        F->qroot = 0;
        F->q_center_pos = (int32_t *)F->own(sizeof(int32_t) * nq);
        F->q_radius = (float *)F->own(sizeof(float) * nq);
        F->q_pt_begin = (int32_t *)F->own(sizeof(int32_t) * nq);
        F->q_pt_end = (int32_t *)F->own(sizeof(int32_t) * nq);
        F->q_kbeg = (int32_t *)F->own(sizeof(int32_t) * nq);
        F->q_kcnt = (int32_t *)F->own(sizeof(int32_t) * nq);
        F->q_kids = (int32_t *)F->own(sizeof(int32_t) * (kA + kB + 2));
        FNN_LAUNCH(k_pair_qtree, dim3(grid_cap(A->nq, 256, 4096)), dim3(256), 0, s,
                   (int)A->nq, nnA, 1, nn, 0, 0, A->q_center_pos, A->q_radius,
                   A->q_pt_begin, A->q_pt_end, A->q_kbeg, A->q_kcnt, F->q_center_pos,
                   F->q_radius, F->q_pt_begin, F->q_pt_end, F->q_kbeg, F->q_kcnt);
        FNN_LAUNCH(k_pair_qtree, dim3(grid_cap(B->nq, 256, 4096)), dim3(256), 0, s,
                   (int)B->nq, nnB, 1 + nnA, nn + npA, nA, kA, B->q_center_pos, B->q_radius,
                   B->q_pt_begin, B->q_pt_end, B->q_kbeg, B->q_kcnt, F->q_center_pos,
                   F->q_radius, F->q_pt_begin, F->q_pt_end, F->q_kbeg, F->q_kcnt);
        if (kA > 0)
            FNN_LAUNCH(k_pair_kids, dim3(grid_cap(kA, 256, 4096)), dim3(256), 0, s, kA, nnA,
                       1, nn, A->q_kids, F->q_kids);
        if (kB > 0)
            FNN_LAUNCH(k_pair_kids, dim3(grid_cap(kB, 256, 4096)), dim3(256), 0, s, kB, nnB,
                       1 + nnA, nn + npA, B->q_kids, F->q_kids + kA);
        // the virtual root: the two query-tree roots as its children
        const int ra = A->qroot < nnA ? 1 + A->qroot : nn + (A->qroot - nnA);
        const int rb = B->qroot < nnB ? 1 + nnA + B->qroot : nn + npA + (B->qroot - nnB);
        const int32_t kids2[2] = {ra, rb};
        const int32_t root_i[5] = {0, 0, n, kA + kB, 2};  // cpos, pb, pe, kbeg, kcnt
        const float inf = INFINITY;
        FNN_HIP(hipMemcpyAsync(F->q_kids + kA + kB, kids2, sizeof kids2,
                               hipMemcpyHostToDevice, s));
        FNN_HIP(hipMemcpyAsync(F->q_center_pos, &root_i[0], 4, hipMemcpyHostToDevice, s));
        FNN_HIP(hipMemcpyAsync(F->q_pt_begin, &root_i[1], 4, hipMemcpyHostToDevice, s));
        FNN_HIP(hipMemcpyAsync(F->q_pt_end, &root_i[2], 4, hipMemcpyHostToDevice, s));
        FNN_HIP(hipMemcpyAsync(F->q_kbeg, &root_i[3], 4, hipMemcpyHostToDevice, s));
        FNN_HIP(hipMemcpyAsync(F->q_kcnt, &root_i[4], 4, hipMemcpyHostToDevice, s));
        FNN_HIP(hipMemcpyAsync(F->q_radius, &inf, 4, hipMemcpyHostToDevice, s));
        F->cross_a = ra;
        F->cross_b = rb;

        // clouds: A's positions [0, nA), B's [nA, n)
        F->ncloud = 2;
        F->cloud_off_h = {0, (int64_t)nA, (int64_t)n};
        F->cloud_src = {0, 1};
        F->ncloud_in = 2;
        F->pcl = (int32_t *)F->own(sizeof(int32_t) * n);
        fill(F->pcl, 0, nA, s);
        fill(F->pcl + nA, 1, nB, s);
        F->depth = std::max(A->depth, B->depth) + 1;
        FNN_HIP(hipStreamSynchronize(s));  // host arrays above go out of scope
        return F;
    } catch (...) {
        delete F;
        throw;
    }
}

void build_tree(fnn_tree *T, const void *points, Scratch &S)
{
    switch (T->metric) {
    case M_L2:
        build_impl<M_L2>(T, points, S);
        break;
    case M_ANG:
        build_impl<M_ANG>(T, points, S);
        break;
    case M_HAM:
        build_impl<M_HAM>(T, points, S);
        break;
    default:
        build_impl<M_LEV>(T, points, S);
        break;
    }
}

}  // namespace fnn
