// All-points range query over the cover tree (Section IV-B, Algorithm 3 run
// for batches of queries) and CSR emission.
//
// Batched query.  A query batch is a query-tree vertex (a cover-tree vertex,
// or a pack of consecutive sibling leaf blocks) with centre c and radius r
// bounding its points.  A pair of vertices (A, B) can hold an edge only if
// d(c_A, c_B) <= r_A + r_B + eps (triangle inequality, the pruning rule of
// Algorithm 3 applied to two balls).  Starting from (root, root), surviving
// pairs are expanded level by level on the GPU (the vertex with the larger
// radius is split; a self pair (A, A) becomes all child pairs (a_i, a_j),
// i <= j), until both sides are packs.  Each unordered pack pair is produced
// once; its point pairs are then evaluated once and written to both rows.
//
// Leaf tiles.  64 x 64 point pairs per work-group step, register-blocked
// 4 x 4 per thread, coordinates staged through LDS.  Every FP32 key outside
// the rounding band of eps decides the edge directly; keys inside it are
// decided by the FP64 reference predicate.
//
// Emission (plain schedule): count pass -> exclusive scan -> fill pass that
// reserves each row's slots with one atomic per row per tile -> per-row sort
// of the columns.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <string.h>

#include <algorithm>

#include "gram.h"
#include "learn.h"

namespace fnn {

constexpr int TT = 256;   // threads per tile work-group
constexpr int TS = 64;    // tile side
constexpr int KC = 32;    // coordinates per LDS stage
constexpr int LDA = 68;   // padded LDS row (floats)
constexpr int GP_TILE = 64;  // points of a full pack

struct QView {
    const int32_t *cpos, *pb, *pe, *kbeg, *kcnt, *kids;
    const float *rad;
    int nn;  // ids >= nn are packs
};

struct Prune {
    float rel;   // relative slack on r_A + r_B + eps
    float abs_;  // absolute slack
    float eps;   // eps as a distance (floor(eps) for integer metrics)
    // batch of clouds: per-cloud eps (CloudThr::peps) by the cloud of the
    // vertex's first position; null for a single cloud
    const CloudThr *ct;
    const int32_t *pcl;
};

template <int M>
__device__ __forceinline__ bool may_touch(const Pts &P, const QView &Q,
                                          const Prune &pr, int a, int b)
{
    const float k = key32<M>(P, Q.cpos[a], Q.cpos[b]);
    const float d = key_to_dist<M>(k);
    const float e = pr.pcl ? pr.ct[pr.pcl[Q.pb[a]]].peps : pr.eps;
    const float lim = Q.rad[a] + Q.rad[b] + e;
    if constexpr (M == M_HAM || M == M_LEV)
        return d <= lim;
    else
        return d <= lim * (1.f + pr.rel) + pr.abs_;
}

// Seeded sample of pack pairs under the traversal's pack-level test: counts
// the pairs it would prune.
template <int M>
__global__ void k_prune_sample(Pts P, QView Q, Prune pr, int npk, int ns,
                               unsigned long long *__restrict__ pruned)
{
    unsigned long long c = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns;
         i += gridDim.x * blockDim.x) {
        unsigned h = (unsigned)i * 0x9E3779B1u + 0x7F4A7C15u;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        const unsigned h2 = h * 0xC2B2AE35u ^ (h >> 16);
        const int a = Q.nn + (int)(h % (unsigned)npk);
        const int b = Q.nn + (int)(h2 % (unsigned)npk);
        c += (a != b && !may_touch<M>(P, Q, pr, a, b)) ? 1 : 0;
    }
    c = wave_sum(c);
    if ((threadIdx.x & (WAVE - 1)) == 0 && c)
        atomicAdd(pruned, c);
}

// ------------------------------------------------------------ traversal --

struct Emit {
    int2 *next;
    int2 *inter;
    // running counts: next frontier, interactions, node tests
    unsigned long long *cnt_next, *cnt_inter, *cnt_tests;
    long long next_cap, inter_cap;
    int *overflow;
};

// Per-wave staging of emitted pairs in LDS: one global reservation per
// STG entries instead of one contended atomic per wave step.
constexpr int STG = 512;
struct Stage {
    int2 *buf[2];   // [0] next frontier, [1] interactions
    int n[2];       // entries held (wave-uniform)
};

__device__ __forceinline__ void stage_flush(const Emit &E, Stage &sg, int k)
{
    __builtin_amdgcn_wave_barrier();
    const int lane = threadIdx.x & (WAVE - 1);
    const int c = sg.n[k];
    if (c == 0)
        return;
    unsigned long long base = 0;
    if (lane == 0)
        base = atomicAdd(k ? E.cnt_inter : E.cnt_next, (unsigned long long)c);
    base = __shfl(base, 0, WAVE);
    int2 *dst = k ? E.inter : E.next;
    const long long cap = k ? E.inter_cap : E.next_cap;
    for (int i = lane; i < c; i += WAVE) {
        const long long p = (long long)(base + i);
        if (p < cap)
            dst[p] = sg.buf[k][i];
        else
            *E.overflow = 1;
    }
    sg.n[k] = 0;
}

__device__ __forceinline__ void emit_pair(const Emit &E, Stage &sg,
                                          const QView &Q, bool valid, int a,
                                          int b)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const bool term = valid && a >= Q.nn && b >= Q.nn;
    const bool nxt = valid && !term;
    const uint64_t m[2] = {__ballot(nxt), __ballot(term)};
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int c = __popcll(m[k]);
        if (c == 0)
            continue;
        if (sg.n[k] + c > STG)
            stage_flush(E, sg, k);
        if ((m[k] >> lane) & 1ull)
            sg.buf[k][sg.n[k] + __popcll(m[k] & lt)] = make_int2(a, b);
        sg.n[k] += c;
    }
}

// Pruning test by TG cooperating lanes (vector metrics): each lane sums a
// TG-th of the coordinates (16-byte slices, so the TG lanes of a test read
// contiguous memory), the partial sums meet by shuffles.  Every lane of the
// group returns the same answer.  The test only has to be conservative; the
// relative slack in Prune covers any summation order.
template <int M, int TG>
__device__ __forceinline__ bool may_touch_coop(const Pts &P, const QView &Q,
                                               const Prune &pr, int a, int b,
                                               bool active)
{
    const int sl = threadIdx.x & (TG - 1);
    float part = 0.f;
    if (active) {
        const float *X = (M == M_ANG) ? P.xn : P.x;
        const float *ra = X + (size_t)Q.cpos[a] * P.dp;
        const float *rb = X + (size_t)Q.cpos[b] * P.dp;
        for (int k = sl * 4; k < P.dp; k += TG * 4) {
            const float4 u = *reinterpret_cast<const float4 *>(ra + k);
            const float4 v = *reinterpret_cast<const float4 *>(rb + k);
            const float d0 = u.x - v.x, d1 = u.y - v.y, d2 = u.z - v.z,
                        d3 = u.w - v.w;
            part = fmaf(d0, d0, part);
            part = fmaf(d1, d1, part);
            part = fmaf(d2, d2, part);
            part = fmaf(d3, d3, part);
        }
    }
#pragma unroll
    for (int o = 1; o < TG; o <<= 1)
        part += __shfl_xor(part, o, WAVE);
    if (!active)
        return false;
    const float d = key_to_dist<M>(part);
    const float e = pr.pcl ? pr.ct[pr.pcl[Q.pb[a]]].peps : pr.eps;
    const float lim = Q.rad[a] + Q.rad[b] + e;
    return d <= lim * (1.f + pr.rel) + pr.abs_;
}

// Expand one vertex pair (whole wave).  With TG > 1 (vector metrics), TG
// lanes share each test and the group's first lane emits the result.
// Returns the number of tests made by this lane.
// A self pair of more children than this is split into one item per child
// row (frontier item (a, -1 - i)) so that many waves share its tests.
constexpr int SELF_SPLIT = 64;

template <int M, int TG>
__device__ unsigned long long expand_one(const Pts &P, const QView &Q,
                                         const Prune &pr, int a, int b,
                                         const Emit &E, Stage &sg)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int sub = lane / TG;                 // test slot of this lane
    const bool lead = (lane & (TG - 1)) == 0;  // the slot's emitting lane
    constexpr int NS = WAVE / TG;              // tests per wave step
    unsigned long long tests = 0;
    if (b < 0) {
        // row i of a split self pair of a: children (i, j), j >= i (the
        // diagonal pair without a test)
        const int i = -1 - b, m = Q.kcnt[a], k0 = Q.kbeg[a];
        const int ka = Q.kids[k0 + i];
        for (int base = 0; base < m - i; base += NS) {
            const int t = base + sub;
            bool valid = t < m - i;
            const int kb = valid ? Q.kids[k0 + i + t] : 0;
            const bool test = valid && t != 0;
            if constexpr (TG == 1) {
                if (test) {
                    ++tests;
                    valid = may_touch<M>(P, Q, pr, ka, kb);
                }
            } else {
                const bool ok = may_touch_coop<M, TG>(P, Q, pr, ka, kb, test);
                if (test) {
                    tests += lead;
                    valid = ok;
                }
            }
            emit_pair(E, sg, Q, valid && lead, ka, kb);
        }
        return tests;
    }
    if (a == b) {
        if (a >= Q.nn) {  // a single pack against itself
            emit_pair(E, sg, Q, lane == 0, a, a);
            return 0;
        }
        const int m = Q.kcnt[a], k0 = Q.kbeg[a];
        if (m > SELF_SPLIT) {
            // m (m + 1) / 2 tests are too many for one wave: the next round
            // takes them as m row items (a, -1 - i), one wave each
            for (int base = 0; base < m; base += WAVE)
                emit_pair(E, sg, Q, base + lane < m, a, -1 - (base + lane));
            return 0;
        }
        const long long tot = (long long)m * (m + 1) / 2;
        for (long long base = 0; base < tot; base += NS) {
            const long long t = base + sub;
            bool valid = t < tot;
            int i = 0, j = 0;
            if (valid) {
                // t -> (i, j), i <= j, row-major over the upper triangle
                double mm = m + 0.5;
                i = (int)floor(mm - sqrt(mm * mm - 2.0 * (double)t));
                if (i < 0)
                    i = 0;
                while (i > 0 && (long long)i * m - (long long)i * (i - 1) / 2 > t)
                    --i;
                while ((long long)(i + 1) * m - (long long)(i + 1) * i / 2 <= t)
                    ++i;
                j = i + (int)(t - ((long long)i * m - (long long)i * (i - 1) / 2));
            }
            int ka = 0, kb = 0;
            if (valid) {
                ka = Q.kids[k0 + i];
                kb = Q.kids[k0 + j];
            }
            const bool test = valid && i != j;
            if constexpr (TG == 1) {
                if (test) {
                    ++tests;
                    valid = may_touch<M>(P, Q, pr, ka, kb);
                }
            } else {
                const bool ok = may_touch_coop<M, TG>(P, Q, pr, ka, kb, test);
                if (test) {
                    tests += lead;
                    valid = ok;
                }
            }
            emit_pair(E, sg, Q, valid && lead, ka, kb);
        }
    } else {
        const bool at = a >= Q.nn, bt_ = b >= Q.nn;
        int s, o;
        if (at && bt_) {  // cannot happen (packs pairs are emitted directly)
            emit_pair(E, sg, Q, lane == 0, a, b);
            return 0;
        }
        if (at)
            s = b, o = a;
        else if (bt_)
            s = a, o = b;
        else if (Q.rad[a] >= Q.rad[b])
            s = a, o = b;
        else
            s = b, o = a;
        const int m = Q.kcnt[s], k0 = Q.kbeg[s];
        for (int base = 0; base < m; base += NS) {
            const int t = base + sub;
            bool valid = t < m;
            const int ka = valid ? Q.kids[k0 + t] : 0;
            if constexpr (TG == 1) {
                if (valid) {
                    ++tests;
                    valid = may_touch<M>(P, Q, pr, ka, o);
                }
            } else {
                const bool ok = may_touch_coop<M, TG>(P, Q, pr, ka, o, valid);
                if (valid) {
                    tests += lead;
                    valid = ok;
                }
            }
            emit_pair(E, sg, Q, valid && lead, ka, o);
        }
    }
    return tests;
}

// Upper bound of the pairs a level can emit (no distances): m children of
// the split vertex, or m(m+1)/2 child pairs of a self pair.
__global__ void k_expand_bound(QView Q, const int2 *__restrict__ cur,
                               long long ncur,
                               unsigned long long *__restrict__ bound)
{
    unsigned long long b = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ncur;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 p = cur[i];
        const int a = p.x, c = p.y;
        if (c < 0) {  // row -1 - c of a split self pair: pairs (i, j), j >= i
            b += (unsigned long long)(Q.kcnt[a] - (-1 - c));
        } else if (a == c) {
            const long long m = a >= Q.nn ? 1 : Q.kcnt[a];
            b += m > SELF_SPLIT ? (unsigned long long)m  // its row items
                                : (unsigned long long)(m * (m + 1) / 2);
        } else {
            const bool at = a >= Q.nn, ct = c >= Q.nn;
            int s;
            if (at && ct)
                s = -1;
            else if (at)
                s = c;
            else if (ct)
                s = a;
            else
                s = Q.rad[a] >= Q.rad[c] ? a : c;
            b += s < 0 ? 1ull : (unsigned long long)Q.kcnt[s];
        }
    }
    b = wave_sum(b);
    if ((threadIdx.x & (WAVE - 1)) == 0 && b)
        atomicAdd(bound, b);
}

template <int M, int TG>
__global__ void __launch_bounds__(256)
k_expand(Pts P, QView Q, Prune pr, const int2 *__restrict__ cur, long long ncur,
         Emit E)
{
    __shared__ int2 stg[256 / WAVE][2][STG];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const long long wpb = blockDim.x / WAVE;
    Stage sg;
    sg.buf[0] = stg[wid][0];
    sg.buf[1] = stg[wid][1];
    sg.n[0] = sg.n[1] = 0;
    unsigned long long tests = 0;
    for (long long w = (long long)blockIdx.x * wpb + wid; w < ncur;
         w += (long long)gridDim.x * wpb) {
        const int2 pr2 = cur[w];
        tests += expand_one<M, TG>(P, Q, pr, pr2.x, pr2.y, E, sg);
    }
    stage_flush(E, sg, 0);
    stage_flush(E, sg, 1);
    tests = wave_sum(tests);
    if (lane == 0 && tests)
        atomicAdd(E.cnt_tests, tests);
}

// ---- device-queue levels (replayed from a graph) ---------------------------
//
// The same expansion with the frontier's length in device memory: a level
// reads its length, bounds its output, and stops (keeping its frontier, and
// every later level with it) when the bound does not fit the buffers, so a
// fixed sequence of levels can be recorded once into a graph and replayed
// until the frontier is empty; the host only reads the length between
// replays, and finishes with the eager loop after a stop.

__global__ void k_expand_bound_d(QView Q, const int2 *__restrict__ cur,
                                 const unsigned long long *__restrict__ ncur_p,
                                 long long cap, const int *__restrict__ halt,
                                 unsigned long long *__restrict__ bound)
{
    if (*halt)
        return;
    // (a length never exceeds the buffer: the guard stops a level whose
    // bound does not fit; the clamp only keeps reads inside regardless)
    const long long ncur = min((long long)*ncur_p, cap);
    unsigned long long b = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ncur;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 p = cur[i];
        const int a = p.x, c = p.y;
        if (c < 0) {
            b += (unsigned long long)(Q.kcnt[a] - (-1 - c));
        } else if (a == c) {
            const long long m = a >= Q.nn ? 1 : Q.kcnt[a];
            b += m > SELF_SPLIT ? (unsigned long long)m : (unsigned long long)(m * (m + 1) / 2);
        } else {
            const bool at = a >= Q.nn, ct = c >= Q.nn;
            int sv;
            if (at && ct)
                sv = -1;
            else if (at)
                sv = c;
            else if (ct)
                sv = a;
            else
                sv = Q.rad[a] >= Q.rad[c] ? a : c;
            b += sv < 0 ? 1ull : (unsigned long long)Q.kcnt[sv];
        }
    }
    b = wave_sum(b);
    if ((threadIdx.x & (WAVE - 1)) == 0 && b)
        atomicAdd(bound, b);
}

// One thread: stop at this level when its output may not fit (halt = 1 +
// the parity of the level's frontier buffer), else clear the next length.
__global__ void k_level_guard(const unsigned long long *__restrict__ ncur_p,
                              unsigned long long *__restrict__ bound,
                              const unsigned long long *__restrict__ ninter_p,
                              long long next_cap, long long inter_cap, int parity,
                              int *__restrict__ halt,
                              unsigned long long *__restrict__ next_len)
{
    if (*halt)
        return;
    const unsigned long long ncur = *ncur_p, bd = *bound;
    if (ncur > 0 && (bd > (unsigned long long)next_cap ||
                     *ninter_p + bd > (unsigned long long)inter_cap)) {
        *halt = 1 + parity;
        return;
    }
    *next_len = 0ull;
    *bound = 0ull;  // for the next level
}

template <int M, int TG>
__global__ void __launch_bounds__(256)
k_expand_d(Pts P, QView Q, Prune pr, const int2 *__restrict__ cur,
           const unsigned long long *__restrict__ ncur_p, const int *__restrict__ halt,
           Emit E)
{
    if (*halt)
        return;
    __shared__ int2 stg[256 / WAVE][2][STG];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const long long wpb = blockDim.x / WAVE;
    // both frontier buffers have next_cap entries
    const long long ncur = min((long long)*ncur_p, E.next_cap);
    Stage sg;
    sg.buf[0] = stg[wid][0];
    sg.buf[1] = stg[wid][1];
    sg.n[0] = sg.n[1] = 0;
    unsigned long long tests = 0;
    for (long long w = (long long)blockIdx.x * wpb + wid; w < ncur;
         w += (long long)gridDim.x * wpb) {
        const int2 pr2 = cur[w];
        tests += expand_one<M, TG>(P, Q, pr, pr2.x, pr2.y, E, sg);
    }
    stage_flush(E, sg, 0);
    stage_flush(E, sg, 1);
    tests = wave_sum(tests);
    if (lane == 0 && tests)
        atomicAdd(E.cnt_tests, tests);
}

// --------------------------------------------------------------- tiles ---

template <int M>
struct TileSmem;

template <>
struct TileSmem<M_L2> {
    float A[KC][LDA], B[KC][LDA];
};
template <>
struct TileSmem<M_ANG> {
    float A[KC][LDA], B[KC][LDA];
};
constexpr int HAM_MAXW = 16;
template <>
struct TileSmem<M_HAM> {
    uint64_t A[HAM_MAXW][TS], B[HAM_MAXW][TS];
};
template <>
struct TileSmem<M_LEV> {
    int dummy;
};

// Destination of the c entries a tile adds to one row: slots [o, o+c) of
// the CSR (or of the learned schedule's slot array, up to lim); with a spill
// list, entries past lim go there.  Returns the spill base (or ~0 if none);
// c is set to 0 when the row cannot take them (overflow flag / error).
__device__ __forceinline__ unsigned long long place(const TileOut &out, int row,
                                                    int &c,
                                                    unsigned long long &o,
                                                    unsigned long long &lim)
{
    o = atomicAdd(&out.cursor[row], (unsigned long long)c);
    lim = out.row_end ? (unsigned long long)out.row_end[row] : out.nnz;
    if (o + c <= lim)
        return ~0ull;
    if (out.row_end && out.spill) {
        const unsigned long long first = o > lim ? o : lim;
        const unsigned long long nsp = o + c - first;
        const unsigned long long sp = atomicAdd(out.spill_cnt, nsp);
        if (sp + nsp <= out.spill_cap)
            return sp - (first - o);  // entry k >= lim lands at sp0 + k
        out.ovf[row] = 1;
        c = 0;
        return ~0ull;
    }
    if (out.row_end)
        out.ovf[row] = 1;
    else
        atomicOr(out.err, ERR_INDEX);
    c = 0;
    return ~0ull;
}

__device__ __forceinline__ void put(const TileOut &out, int row, int col,
                                    float d, unsigned long long idx,
                                    unsigned long long o, unsigned long long lim,
                                    unsigned long long spb)
{
    // idx = o + k for the k-th entry of this placement
    if (idx < lim) {
        out.col[idx] = col;
        out.dist[idx] = d;
    } else {
        const unsigned long long q = spb + (idx - o);
        out.spill[q] = make_int2(row, col);
        out.spill_dist[q] = d;
    }
}

// Tile pass modes: count row degrees; fill CSR slots; or count and append
// every edge to an edge list in both directions (which replaces the fill
// pass): a row's entries, then a column's, lie next to each other, so the
// scatter claims slots once per run.
enum { TILE_COUNT = 0, TILE_FILL = 1, TILE_LIST = 2 };

template <int M, int MODE>
__global__ void __launch_bounds__(TT)
k_tile(Pts P, const int2 *__restrict__ inter, long long ninter,
       const int32_t *__restrict__ q_pb, const int32_t *__restrict__ q_pe,
       const int32_t *__restrict__ perm, Thr E0, const CloudThr *__restrict__ ct,
       const int32_t *__restrict__ pcl, int fp64_dist, TileOut out)
{
    __shared__ TileSmem<M> sm;
    __shared__ unsigned long long mask[TS];   // edge bits of each row (bit = column)
    __shared__ unsigned long long cmask[TS];  // and of each column (bit = row)
    constexpr bool FILL = MODE == TILE_FILL, LIST = MODE == TILE_LIST;
    constexpr bool DIST = FILL || LIST;  // keep the tile's edge distances
    __shared__ float dt[DIST ? TS * (TS + 1) : 1];
    const int t = threadIdx.x, ty = t / 16, tx = t % 16;
    unsigned long long rechecks = 0, pairs = 0;
    __shared__ long long s_next;
    for (long long it = blockIdx.x; it < ninter;) {
    const int2 pr = inter[out.order ? (long long)out.order[it] : it];
    const int A = pr.x, B = pr.y;
    const bool diag = A == B;
    const int a0 = q_pb[A], na = q_pe[A] - a0;
    const Thr E = pcl ? ct[pcl[a0]].E : E0;  // both packs lie in one cloud
    const int b0 = q_pb[B], nb = q_pe[B] - b0;

    for (int ia = 0; ia < na; ia += TS) {
        for (int jb = diag ? ia : 0; jb < nb; jb += TS) {
            const int ra = min(TS, na - ia), rb = min(TS, nb - jb);
            const bool sdiag = diag && ia == jb;
            const int pa = a0 + ia, pb = b0 + jb;  // first tree positions
            if (t < TS)
                mask[t] = 0ull;
            else if (t < 2 * TS)
                cmask[t - TS] = 0ull;
            float acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = 0.f;

            if constexpr (M == M_L2 || M == M_ANG) {
                const float *X = (M == M_ANG) ? P.xn : P.x;
                const int dp = P.dp;
                for (int k0 = 0; k0 < dp; k0 += KC) {
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int f = t + q * TT;  // float4 index in 64 x 8
                        const int row = f / (KC / 4), c4 = f % (KC / 4);
                        const int kk = k0 + c4 * 4;
                        float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
                        if (row < ra && kk < dp)
                            va = *reinterpret_cast<const float4 *>(
                                X + (size_t)(pa + row) * dp + kk);
                        if (row < rb && kk < dp)
                            vb = *reinterpret_cast<const float4 *>(
                                X + (size_t)(pb + row) * dp + kk);
                        sm.A[c4 * 4 + 0][row] = va.x;
                        sm.A[c4 * 4 + 1][row] = va.y;
                        sm.A[c4 * 4 + 2][row] = va.z;
                        sm.A[c4 * 4 + 3][row] = va.w;
                        sm.B[c4 * 4 + 0][row] = vb.x;
                        sm.B[c4 * 4 + 1][row] = vb.y;
                        sm.B[c4 * 4 + 2][row] = vb.z;
                        sm.B[c4 * 4 + 3][row] = vb.w;
                    }
                    __syncthreads();
                    const int kend = min(KC, dp - k0);
                    for (int k = 0; k < kend; ++k) {
                        const float4 u = *reinterpret_cast<const float4 *>(&sm.A[k][ty * 4]);
                        const float4 v = *reinterpret_cast<const float4 *>(&sm.B[k][tx * 4]);
                        const float ua[4] = {u.x, u.y, u.z, u.w};
                        const float vb[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const float d = ua[i] - vb[j];
                                acc[i][j] = fmaf(d, d, acc[i][j]);
                            }
                    }
                }
            } else if constexpr (M == M_HAM) {
                const int W = P.dp;
                __syncthreads();
                for (int e = t; e < W * TS; e += TT) {
                    const int row = e / W, w = e % W;
                    sm.A[w][row] = row < ra ? P.h[(size_t)(pa + row) * W + w] : 0ull;
                    sm.B[w][row] = row < rb ? P.h[(size_t)(pb + row) * W + w] : 0ull;
                }
                __syncthreads();
                int hc[4][4] = {};
                for (int w = 0; w < W; ++w) {
                    uint64_t ua[4], vb[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        ua[i] = sm.A[w][ty * 4 + i];
                        vb[i] = sm.B[w][tx * 4 + i];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            hc[i][j] += __popcll(ua[i] ^ vb[j]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = (float)hc[i][j];
                __syncthreads();
            } else {  // Levenshtein: one bit-parallel DP per pair
                __syncthreads();
                const int kk = (int)E.lo;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int ri = ty * 4 + i, cj = tx * 4 + j;
                        float v = FLT_MAX;
                        if (ri < ra && cj < rb && (!sdiag || ri < cj)) {
                            const int p = pa + ri, q = pb + cj;
                            const int lp = P.len[p], lq = P.len[q];
                            if (abs(lp - lq) <= kk)
                                v = (float)key32<M_LEV>(P, p, q);
                        }
                        acc[i][j] = v;
                    }
            }

            // ---- exactness guard and edge bits ----------------------------
            unsigned long long rc = 0;
            unsigned cnib[4] = {0u, 0u, 0u, 0u};  // column j's rows (bit i)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ri = ty * 4 + i;
                unsigned nib = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int cj = tx * 4 + j;
                    if (ri < ra && cj < rb && (!sdiag || ri < cj)) {
                        const float k = acc[i][j];
                        bool e;
                        if constexpr (M == M_HAM || M == M_LEV) {
                            e = k <= E.lo;
                        } else {
                            if (k < E.lo)
                                e = true;
                            else if (k > E.hi)
                                e = false;
                            else {
                                ++rc;
                                if constexpr (M == M_L2)
                                    e = l2_sq64(P.x + (size_t)(pa + ri) * P.dp,
                                                P.x + (size_t)(pb + cj) * P.dp,
                                                P.dim) <= E.p64;
                                else
                                    e = ang_within64(P.x + (size_t)(pa + ri) * P.dp,
                                                     P.x + (size_t)(pb + cj) * P.dp,
                                                     P.dim, E.p64);
                            }
                        }
                        if (e) {
                            nib |= 1u << j;
                            cnib[j] |= 1u << i;
                            if constexpr (DIST)
                                dt[ri * (TS + 1) + cj] =
                                    edge_dist<M>(P, pa + ri, pb + cj, k, fp64_dist);
                        }
                    }
                }
                if (nib)
                    atomicOr(&mask[ri], (unsigned long long)nib << (tx * 4));
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (cnib[j])
                    atomicOr(&cmask[tx * 4 + j], (unsigned long long)cnib[j] << (ty * 4));
            rechecks += rc;
            if (t == 0)
                pairs += sdiag ? (unsigned long long)ra * (ra - 1) / 2
                               : (unsigned long long)ra * rb;
            __syncthreads();

            // ---- rows (threads 0..63) and columns (threads 64..127) -------
            if (t < TS) {
                const int r = t;
                const unsigned long long bits = r < ra ? mask[r] : 0ull;
                int c = __popcll(bits);
                const int orow = c ? perm[pa + r] : 0;
                if (c && FILL && out.row_filter && !out.row_filter[orow])
                    c = 0;
                if (c) {
                    if constexpr (!FILL) {
                        atomicAdd(&out.deg[orow], c);
                    } else {
                        unsigned long long o, lim;
                        const unsigned long long spb = place(out, orow, c, o, lim);
                        unsigned long long bb = c ? bits : 0ull;
                        unsigned long long idx = o;
                        while (bb) {
                            const int j = __ffsll((long long)bb) - 1;
                            bb &= bb - 1;
                            put(out, orow, perm[pb + j], dt[r * (TS + 1) + j], idx,
                                o, lim, spb);
                            ++idx;
                        }
                    }
                }
                if constexpr (LIST) {
                    // this row's edges (threads 0..63 are one wave: one
                    // reservation for all of them)
                    int incl = c;
#pragma unroll
                    for (int o = 1; o < WAVE; o <<= 1) {
                        const int v = __shfl_up(incl, o, WAVE);
                        if ((t & (WAVE - 1)) >= o)
                            incl += v;
                    }
                    const int tot = __shfl(incl, WAVE - 1, WAVE);
                    unsigned long long base = 0;
                    if (t == 0 && tot)
                        base = atomicAdd(out.ecnt, (unsigned long long)tot);
                    base = __shfl(base, 0, WAVE) + (unsigned long long)(incl - c);
                    unsigned long long bb = bits;
                    while (bb) {
                        const int j = __ffsll((long long)bb) - 1;
                        bb &= bb - 1;
                        if (base < out.ecap) {
                            out.elist[base] = make_int2(orow, perm[pb + j]);
                            out.edist[base] = dt[r * (TS + 1) + j];
                        }
                        ++base;
                    }
                }
            } else if (t < 2 * TS) {
                const int cc = t - TS;
                const unsigned long long cbits = cc < rb ? cmask[cc] : 0ull;
                int c = __popcll(cbits);
                const int ocol = c ? perm[pb + cc] : 0;
                if constexpr (LIST) {
                    // the same edges seen from this column (threads 64..127
                    // are one wave)
                    int incl = c;
#pragma unroll
                    for (int o = 1; o < WAVE; o <<= 1) {
                        const int v = __shfl_up(incl, o, WAVE);
                        if ((t & (WAVE - 1)) >= o)
                            incl += v;
                    }
                    const int tot = __shfl(incl, WAVE - 1, WAVE);
                    unsigned long long base = 0;
                    if (cc == 0 && tot)
                        base = atomicAdd(out.ecnt, (unsigned long long)tot);
                    base = __shfl(base, 0, WAVE) + (unsigned long long)(incl - c);
                    unsigned long long rbits = cbits;
                    while (rbits) {
                        const int r = __ffsll((long long)rbits) - 1;
                        rbits &= rbits - 1;
                        if (base < out.ecap) {
                            out.elist[base] = make_int2(ocol, perm[pa + r]);
                            out.edist[base] = dt[r * (TS + 1) + cc];
                        }
                        ++base;
                    }
                }
                if (cc < rb) {
                    if (c && FILL && out.row_filter && !out.row_filter[ocol])
                        c = 0;
                    if (c) {
                        if constexpr (!FILL) {
                            atomicAdd(&out.deg[ocol], c);
                        } else {
                            unsigned long long o, lim;
                            const unsigned long long spb = place(out, ocol, c, o, lim);
                            unsigned long long idx = o;
                            unsigned long long rbits = c ? cbits : 0ull;
                            while (rbits) {
                                const int r = __ffsll((long long)rbits) - 1;
                                rbits &= rbits - 1;
                                put(out, ocol, perm[pa + r], dt[r * (TS + 1) + cc], idx, o,
                                    lim, spb);
                                ++idx;
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    // next item: the grid stride, or (ordered work) the next free one
    if (out.next) {
        if (t == 0)
            s_next = (long long)gridDim.x + (long long)atomicAdd(out.next, 1ull);
        __syncthreads();
        it = s_next;
        __syncthreads();  // s_next is rewritten after the next item
    } else {
        it += gridDim.x;
    }
    }
    rechecks = wave_sum(rechecks);
    if ((t & (WAVE - 1)) == 0 && rechecks)
        atomicAdd(&out.cnt[1], rechecks);
    if (t == 0)
        atomicAdd(&out.cnt[0], pairs);
}

// Decided survivors into their CSR slots as packed entries (column << 32 |
// distance bits, the row sort's key): edge i (input ids a, b) goes to slot
// row_ptr[a] + rank.x and row_ptr[b] + rank.y, one 8-byte store each, so the
// scattered stores are half as many as with separate column and distance
// stores; the row sort writes col and dist.  A rank past its row sets
// ERR_INDEX.
__global__ void k_place_packed(const int2 *__restrict__ edges, const float *__restrict__ edist,
                               const int2 *__restrict__ erank, long long ne,
                               const int64_t *__restrict__ row_ptr,
                               unsigned long long *__restrict__ pk, int *__restrict__ err)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = edges[i];
        if (e.x < 0)
            continue;  // a survivor that is no edge
        const int2 r = erank[i];
        const uint32_t d = __float_as_uint(edist[i]);
        const int64_t a0 = row_ptr[e.x], a1 = row_ptr[e.x + 1];
        const int64_t b0 = row_ptr[e.y], b1 = row_ptr[e.y + 1];
        const int64_t s1 = a0 + r.x, s2 = b0 + r.y;
        if (r.x >= 0 && r.y >= 0 && s1 < a1 && s2 < b1) {
            pk[s1] = ((unsigned long long)(uint32_t)e.y << 32) | d;
            pk[s2] = ((unsigned long long)(uint32_t)e.x << 32) | d;
        } else {
            atomicOr(err, ERR_INDEX);
        }
    }
}

// ------------------------------------------------------------ row sort ---

__device__ __forceinline__ unsigned long long pack_entry(int32_t c, float d)
{
    return ((unsigned long long)(uint32_t)c << 32) | __float_as_uint(d);
}

// One row of up to 64*V entries sorted by one wave with a bitonic network
// in registers: element lane*V + v lives in register v of that lane, so
// strides below V swap registers within a lane and only the longer ones
// exchange across lanes.  With 8 or more keys per lane the row moves
// between memory and registers through the wave's LDS tile tr
// (WAVE * (V + 1) words; element g at word g + g / V, so both the coalesced
// side, 64 consecutive slots per instruction, and the lane-major side stay
// within two-way bank sharing); with fewer keys the lane reads its
// consecutive slots directly.  The entries come from pk (packed, same
// slots) when it is non-null, else from col and dist; the sorted row goes
// to col and dist.
template <int V>
__device__ __forceinline__ void wave_sort_row(int32_t *__restrict__ col,
                                              float *__restrict__ dist, int64_t b,
                                              int len, int lane,
                                              const unsigned long long *__restrict__ pk,
                                              unsigned long long *tr)
{
    static_assert(V >= 1 && V <= 32, "keys per lane");
    constexpr bool LT = V >= 8;  // memory side through the LDS tile
    auto idx = [&](int v) { return lane * V + v; };
    auto ld = [&](int i) {
        return i >= len ? ~0ull : pk ? pk[b + i] : pack_entry(col[b + i], dist[b + i]);
    };
    unsigned long long x[V];
    if constexpr (LT) {
        // one wave's LDS accesses complete in order: only the compiler must
        // keep the reads after the writes (and later writes after them)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int g = v * WAVE + lane;
            tr[g + g / V] = ld(g);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int v = 0; v < V; ++v)
            x[v] = tr[lane * (V + 1) + v];
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
            x[v] = ld(idx(v));
    }
#pragma unroll
    for (int k = 2; k <= WAVE * V; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < V) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v & j)
                        continue;
                    const int w = v | j;
                    const bool up = (idx(v) & k) == 0;
                    const unsigned long long a = x[v], c = x[w];
                    if ((a > c) == up) {
                        x[v] = c;
                        x[w] = a;
                    }
                }
            } else {
                const int lj = j / V;  // lane stride
                const bool lower = (lane & lj) == 0;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const unsigned long long o = __shfl_xor(x[v], lj, WAVE);
                    const bool up = (idx(v) & k) == 0;
                    x[v] = (lower == up) ? (o < x[v] ? o : x[v]) : (o > x[v] ? o : x[v]);
                }
            }
        }
    }
    auto st = [&](int i, unsigned long long e) {
        if (i < len) {
            col[b + i] = (int32_t)(e >> 32);
            dist[b + i] = __uint_as_float((uint32_t)e);
        }
    };
    if constexpr (LT) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int v = 0; v < V; ++v)
            tr[lane * (V + 1) + v] = x[v];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int g = v * WAVE + lane;
            st(g, tr[g + g / V]);
        }
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
            st(idx(v), x[v]);
    }
}

// Rows of at most 512 entries: one wave per row (register bitonic sort);
// longer rows are listed for the work-group and global sorts.  With pk
// non-null the entries are read packed from pk (same slots) and every row
// is written to col and dist: sorted here, or unpacked in place for the
// listed sorts.
__global__ void __launch_bounds__(256)
k_sort_small(const int64_t *__restrict__ row_ptr, int n, int32_t *__restrict__ col,
             float *__restrict__ dist, int32_t *__restrict__ mid_list,
             int32_t *__restrict__ long_list, int32_t *__restrict__ counts,
             const unsigned long long *__restrict__ pk)
{
    __shared__ unsigned long long tr_s[256 / WAVE][WAVE * 9];  // 8 keys per lane
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    unsigned long long *tr = tr_s[threadIdx.x / WAVE];
    for (int r = blockIdx.x * wpb + threadIdx.x / WAVE; r < n;
         r += gridDim.x * wpb) {
    const int64_t b = row_ptr[r];
    const int64_t len = row_ptr[r + 1] - b;
    if (pk && (len == 1 || len > 8 * WAVE))
        for (int64_t i = lane; i < len; i += WAVE) {
            const unsigned long long x = pk[b + i];
            col[b + i] = (int32_t)(x >> 32);
            dist[b + i] = __uint_as_float((uint32_t)x);
        }
    if (len <= 1)
        continue;
    if (len > 8 * WAVE) {
        if (lane == 0) {
            if (len <= 4096)
                mid_list[atomicAdd(&counts[0], 1)] = r;
            else
                long_list[atomicAdd(&counts[1], 1)] = r;
        }
        continue;
    }
    if (len > 4 * WAVE) {
        wave_sort_row<8>(col, dist, b, (int)len, lane, pk, tr);
        continue;
    }
    if (len > 2 * WAVE) {
        wave_sort_row<4>(col, dist, b, (int)len, lane, pk, tr);
        continue;
    }
    if (len > WAVE) {
        wave_sort_row<2>(col, dist, b, (int)len, lane, pk, tr);
        continue;
    }
    unsigned long long v = lane >= len ? ~0ull
                           : pk        ? pk[b + lane]
                                       : pack_entry(col[b + lane], dist[b + lane]);
    for (int k = 2; k <= WAVE; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            unsigned long long o = __shfl_xor(v, j, WAVE);
            const bool up = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            const bool take_min = (lower == up);
            v = take_min ? (o < v ? o : v) : (o > v ? o : v);
        }
    }
    if (lane < len) {
        col[b + lane] = (int32_t)(v >> 32);
        dist[b + lane] = __uint_as_float((uint32_t)v);
    }
    }
}

// Rows of 513..2048 entries (from the list of 513..4096): one wave per row,
// the register sort with 16 or 32 entries per lane.
__global__ void __launch_bounds__(256)
k_sort_wave(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ list,
            int nl, int32_t *__restrict__ col, float *__restrict__ dist)
{
    __shared__ unsigned long long tr_s[256 / WAVE][WAVE * 33];  // up to 32 keys per lane
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    unsigned long long *tr = tr_s[threadIdx.x / WAVE];
    for (int li = blockIdx.x * wpb + threadIdx.x / WAVE; li < nl; li += gridDim.x * wpb) {
        const int r = list[li];
        const int64_t b = row_ptr[r];
        const int len = (int)(row_ptr[r + 1] - b);
        if (len > 32 * WAVE)
            continue;  // the work-group sort's
        if (len > 16 * WAVE)
            wave_sort_row<32>(col, dist, b, len, lane, nullptr, tr);
        else
            wave_sort_row<16>(col, dist, b, len, lane, nullptr, tr);
    }
}

// Listed rows of lo+1 .. 1024 NW entries: one work-group of NW waves per
// row, padded to N = 1024 NW.  Entry g = 1024 w + 64 v + lane lives in
// register v of that lane of wave w: bitonic stages with strides below 64
// exchange across lanes, strides up to 512 swap registers, and only the
// stages with strides of 1024 and more go through LDS.
template <int NW>
__global__ void __launch_bounds__(NW * WAVE)
k_sort_blk(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ list,
           int nl, int lo, int32_t *__restrict__ col, float *__restrict__ dist)
{
    constexpr int V = 16, N = NW * V * WAVE;
    __shared__ unsigned long long s[N];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int g0 = w * V * WAVE + lane;  // entry of register 0
    for (int li = blockIdx.x; li < nl; li += gridDim.x) {
        const int r = list[li];
        const int64_t b = row_ptr[r];
        const int64_t len64 = row_ptr[r + 1] - b;
        if (len64 <= lo || len64 > N)
            continue;  // another kernel's (the same for the whole work-group)
        const int len = (int)len64;
        unsigned long long x[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int g = g0 + v * WAVE;
            x[v] = g < len ? pack_entry(col[b + g], dist[b + g]) : ~0ull;
        }
#pragma unroll
        for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (j >= V * WAVE) {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        s[g0 + v * WAVE] = x[v];
                    __syncthreads();
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int g = g0 + v * WAVE;
                        const unsigned long long o = s[g ^ j];
                        const bool up = (g & k) == 0, lower = (g & j) == 0;
                        x[v] = (lower == up) ? (o < x[v] ? o : x[v]) : (o > x[v] ? o : x[v]);
                    }
                    __syncthreads();  // s is written again by the next such stage
                } else if (j >= WAVE) {
                    const int jv = j / WAVE;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        if (v & jv)
                            continue;
                        const bool up = ((g0 + v * WAVE) & k) == 0;
                        const unsigned long long a = x[v], c = x[v | jv];
                        if ((a > c) == up) {
                            x[v] = c;
                            x[v | jv] = a;
                        }
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const unsigned long long o = __shfl_xor(x[v], j, WAVE);
                        const bool up = ((g0 + v * WAVE) & k) == 0;
                        const bool lower = (lane & j) == 0;
                        x[v] = (lower == up) ? (o < x[v] ? o : x[v]) : (o > x[v] ? o : x[v]);
                    }
                }
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int g = g0 + v * WAVE;
            if (g < len) {
                col[b + g] = (int32_t)(x[v] >> 32);
                dist[b + g] = __uint_as_float((uint32_t)x[v]);
            }
        }
    }
}

constexpr int SORT_BLK_MAX = 16 * 16 * WAVE;  // longest row k_sort_blk<16> sorts

// Longer rows: one work-group per row, bitonic sort in a global scratch
// buffer (rare: only rows with more than 16384 neighbours).
__global__ void __launch_bounds__(256)
k_sort_long(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ list,
            const int64_t *__restrict__ soff, unsigned long long *__restrict__ scr,
            int32_t *__restrict__ col, float *__restrict__ dist)
{
    const int r = list[blockIdx.x];
    const int64_t b = row_ptr[r];
    const int64_t len = row_ptr[r + 1] - b;
    if (len <= SORT_BLK_MAX)
        return;  // sorted in registers by k_sort_blk<16>
    unsigned long long *s = scr + soff[blockIdx.x];
    int64_t P2 = 1;
    while (P2 < len)
        P2 <<= 1;
    for (int64_t i = threadIdx.x; i < P2; i += blockDim.x)
        s[i] = i < len ? pack_entry(col[b + i], dist[b + i]) : ~0ull;
    __syncthreads();
    for (int64_t k = 2; k <= P2; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t i = threadIdx.x; i < P2; i += blockDim.x) {
                const int64_t l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    unsigned long long x = s[i], y = s[l];
                    if ((x > y) == up) {
                        s[i] = y;
                        s[l] = x;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
        col[b + i] = (int32_t)(s[i] >> 32);
        dist[b + i] = __uint_as_float((uint32_t)s[i]);
    }
}

__global__ void k_long_sizes(const int64_t *__restrict__ row_ptr,
                             const int32_t *__restrict__ list, int nl,
                             int64_t *__restrict__ p2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl)
        return;
    const int r = list[i];
    const int64_t len = row_ptr[r + 1] - row_ptr[r];
    int64_t P2 = 1;
    while (P2 < len)
        P2 <<= 1;
    p2[i] = P2;
}

__global__ void k_cursor_init(const int64_t *__restrict__ row_ptr, int n,
                              unsigned long long *__restrict__ cur)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        cur[i] = (unsigned long long)row_ptr[i];
}

__global__ void k_cursor_check(const int64_t *__restrict__ row_ptr, int n,
                               const unsigned long long *__restrict__ cur,
                               int *__restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cur[i] != (unsigned long long)row_ptr[i + 1])
        atomicOr(bad, 1);
}

// ------------------------------------------------- learned schedule ----

// Slots per row from the predicted log1p(degree) (tree order p -> row).
__global__ void k_caps(const float *__restrict__ pred, const int32_t *__restrict__ perm,
                       int n, float slack, int32_t *__restrict__ cap)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += gridDim.x * blockDim.x) {
        const float e = fmaxf(expm1f(fminf(pred[2 * p + 1], 30.f)), 0.f);
        float c = ceilf(e * (1.f + slack) + 4.f);
        c = fminf(c, (float)(n - 1));
        cap[perm[p]] = (int32_t)fmaxf(c, 0.f);
    }
}

__global__ void k_deg_from_cursor(const unsigned long long *__restrict__ cur,
                                  const int64_t *__restrict__ sb, int n,
                                  int32_t *__restrict__ deg)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += gridDim.x * blockDim.x)
        deg[r] = (int32_t)(cur[r] - (unsigned long long)sb[r]);
}

// Rows that fitted their slots move to the CSR (one wave per row).
__global__ void k_compact(const int64_t *__restrict__ sb, const int32_t *__restrict__ scol,
                          const float *__restrict__ sdist,
                          const int32_t *__restrict__ ovf,
                          const int64_t *__restrict__ row_ptr, int n,
                          int32_t *__restrict__ col, float *__restrict__ dist,
                          int32_t *__restrict__ novf)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    int cnt = 0;
    for (int r = blockIdx.x * wpb + threadIdx.x / WAVE; r < n;
         r += gridDim.x * wpb) {
        if (ovf[r]) {
            cnt += lane == 0;
            continue;
        }
        const int64_t b = row_ptr[r], s0 = sb[r];
        const int64_t len = min(row_ptr[r + 1] - b, sb[r + 1] - s0);
        for (int64_t i = lane; i < len; i += WAVE) {
            col[b + i] = scol[s0 + i];
            dist[b + i] = sdist[s0 + i];
        }
    }
    if (lane == 0 && cnt)
        atomicAdd(novf, cnt);
}

// Spilled entries go after the row's slot entries (cursor starts there).
__global__ void k_spill_init(const int64_t *__restrict__ row_ptr,
                             const int64_t *__restrict__ sb, int n,
                             unsigned long long *__restrict__ cur)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += gridDim.x * blockDim.x) {
        const int64_t len = row_ptr[r + 1] - row_ptr[r];
        const int64_t cap = sb[r + 1] - sb[r];
        cur[r] = (unsigned long long)(row_ptr[r] + (len < cap ? len : cap));
    }
}

// A reservation that did not fit leaves its slots below the capacity
// unwritten: the list is initialised with row -1 and such entries are
// skipped.
__global__ void k_spill_scatter(const int2 *__restrict__ sp, const float *__restrict__ sd,
                                long long ns, int n, const int32_t *__restrict__ ovf,
                                unsigned long long *__restrict__ cur,
                                const int64_t *__restrict__ row_ptr,
                                int32_t *__restrict__ col, float *__restrict__ dist,
                                int *__restrict__ err)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ns;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = sp[i];
        if (e.x < 0)
            continue;
        if (e.x >= n) {
            atomicOr(err, ERR_INDEX);
            continue;
        }
        if (ovf[e.x])
            continue;
        const unsigned long long p = atomicAdd(&cur[e.x], 1ull);
        if ((long long)p >= row_ptr[e.x + 1]) {
            atomicOr(err, ERR_INDEX);
            continue;
        }
        col[p] = e.y;
        dist[p] = sd[i];
    }
}

// Packs holding an overflowed row, then the block pairs touching them.
__global__ void k_mark_packs(const int32_t *__restrict__ ovf,
                             const int32_t *__restrict__ perm,
                             const int32_t *__restrict__ pack_of, int n,
                             int32_t *__restrict__ flag)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += gridDim.x * blockDim.x)
        if (ovf[perm[p]])
            flag[pack_of[p]] = 1;
}

__global__ void k_sublist(const int2 *__restrict__ inter, long long ni,
                          const int32_t *__restrict__ flag, int2 *__restrict__ out,
                          unsigned long long *__restrict__ cnt)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ni;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = inter[i];
        if (flag[e.x] || flag[e.y])
            out[atomicAdd(cnt, 1ull)] = e;
    }
}

__global__ void k_not(const int32_t *__restrict__ a, int n, int32_t *__restrict__ b)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x)
        b[i] = !a[i];
}

__global__ void k_cursor_check_rows(const int64_t *__restrict__ row_ptr, int n,
                                    const unsigned long long *__restrict__ cur,
                                    const int32_t *__restrict__ only,
                                    int *__restrict__ bad)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x)
        if ((!only || only[i]) && cur[i] != (unsigned long long)row_ptr[i + 1])
            atomicOr(bad, 1);
}

// Per-pack visits (block pairs a pack takes part in).
__global__ void k_visits(const int2 *__restrict__ inter, long long ni, int nn,
                         int32_t *__restrict__ vis)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ni;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 e = inter[i];
        atomicAdd(&vis[e.x - nn], 1);
        if (e.y != e.x)
            atomicAdd(&vis[e.y - nn], 1);
    }
}

__global__ void k_targets(const int32_t *__restrict__ vis,
                          const int32_t *__restrict__ pack_of,
                          const int32_t *__restrict__ perm,
                          const int64_t *__restrict__ row_ptr, int n, int nn,
                          float *__restrict__ tg)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += gridDim.x * blockDim.x) {
        const int r = perm[p];
        tg[2 * p] = log1pf((float)vis[pack_of[p] - nn]);
        tg[2 * p + 1] = log1pf((float)(row_ptr[r + 1] - row_ptr[r]));
    }
}

// Prediction error against the true degrees: sum |pred - log1p(deg)|,
// sum expm1(pred), sum deg.
__global__ void k_pred_err(const float *__restrict__ pred,
                           const int32_t *__restrict__ perm,
                           const int64_t *__restrict__ row_ptr, int n,
                           double *__restrict__ acc)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += gridDim.x * blockDim.x) {
        const int r = perm[p];
        const double d = (double)(row_ptr[r + 1] - row_ptr[r]);
        const double y = pred[2 * p + 1];
        a += fabs(y - log1p(d));
        b += expm1(fmin(y, 30.0));
        c += d;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        atomicAdd(&acc[0], a);
        atomicAdd(&acc[1], b);
        atomicAdd(&acc[2], c);
    }
}

// -------------------------------------------------------------- driver ---

// Two events around one launch (the MFMA filter's own duration).
struct Events {
    hipEvent_t e[2];
    explicit Events(hipStream_t)
    {
        FNN_HIP(hipEventCreate(&e[0]));
        FNN_HIP(hipEventCreate(&e[1]));
    }
    ~Events()
    {
        (void)hipEventDestroy(e[0]);
        (void)hipEventDestroy(e[1]);
    }
    hipEvent_t operator[](int i) const { return e[i]; }
};

struct Timer {
    hipEvent_t e[8];
    int k = 0;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st)
    {
        for (auto &x : e)
            FNN_HIP(hipEventCreate(&x));
    }
    ~Timer()
    {
        for (auto &x : e)
            (void)hipEventDestroy(x);
    }
    void mark() { FNN_HIP(hipEventRecord(e[k++], s)); }
    double ms(int a, int b)
    {
        float v = 0.f;
        FNN_HIP(hipEventElapsedTime(&v, e[a], e[b]));
        return v;
    }
};

// Forest: the traversal starts from the self pair of every cloud root (the
// children of the virtual vertex 0); pairs of different clouds never form.
__global__ void k_forest_frontier(QView Q, int2 *__restrict__ cur, int cap)
{
    const int m = min(Q.kcnt[0], cap), k0 = Q.kbeg[0];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += gridDim.x * blockDim.x) {
        const int k = Q.kids[k0 + i];
        cur[i] = make_int2(k, k);
    }
}

constexpr unsigned EXPAND_GRID = 4096;  // work-groups of the expansion

// Launch of one level of the expansion (eager: ncur from the host; device:
// ncur and the stop flag from device memory, a fixed grid).  Vector metrics:
// lanes share each pruning test (coalesced rows).
template <int M, int TG>
static void launch_expand_tg(const Pts &P, const QView &Q, const Prune &pr,
                             const int2 *cur, long long ncur,
                             const unsigned long long *ncur_d, const int *halt,
                             const Emit &E, hipStream_t s)
{
    const dim3 blk(256);
    if (ncur_d)
        FNN_LAUNCH((k_expand_d<M, TG>), dim3(EXPAND_GRID), blk, 0, s, P, Q, pr, cur, ncur_d,
                   halt, E);
    else
        FNN_LAUNCH((k_expand<M, TG>), dim3(std::min<unsigned>(grid_for(ncur, 4), EXPAND_GRID)),
                   blk, 0, s, P, Q, pr, cur, ncur, E);
}

template <int M>
static void launch_expand(const Pts &P, const QView &Q, const Prune &pr, const int2 *cur,
                          long long ncur, const unsigned long long *ncur_d,
                          const int *halt, const Emit &E, hipStream_t s)
{
    if constexpr (M == M_L2 || M == M_ANG) {
        if (P.dp >= 32)
            launch_expand_tg<M, 8>(P, Q, pr, cur, ncur, ncur_d, halt, E, s);
        else if (P.dp >= 16)
            launch_expand_tg<M, 4>(P, Q, pr, cur, ncur, ncur_d, halt, E, s);
        else if (P.dp >= 8)
            launch_expand_tg<M, 2>(P, Q, pr, cur, ncur, ncur_d, halt, E, s);
        else
            launch_expand_tg<M, 1>(P, Q, pr, cur, ncur, ncur_d, halt, E, s);
    } else {
        launch_expand_tg<M, 1>(P, Q, pr, cur, ncur, ncur_d, halt, E, s);
    }
}

// The level-synchronous expansion.  With gp > 1, levels first run as
// device-queue passes: gp levels (even) recorded once into a graph and
// replayed until the frontier is empty, one host read per replay; a level
// whose output may not fit the fixed buffers stops the replays with its
// frontier intact, and the eager loop below (one bound and one count read
// per level, buffers grown to fit) finishes from there.
template <int M>
static void traverse(const fnn_tree *T, const Pts &P, const QView &Q,
                     const Prune &pr, Scratch &S, int gp, long long list_cap,
                     int2 **inter_out, long long *ninter_out, fnn_stats &st)
{
    hipStream_t s = S.stream();
    const bool cross = T->cross_a >= 0;  // bichromatic: the pair of cloud roots
    const long long nroot = cross ? 1 : (T->ncloud > 1 ? T->ncloud : 1);
    // [0], [1] frontier lengths (ping-pong), [2] interactions, [3] tests,
    // [4] level bound
    unsigned long long *cnt = S.get<unsigned long long>(5);
    int *ovf = S.get<int>(2);  // [0] emission past a bound, [1] halt
    long long cap_cur, cap_next, cap_int;
    if (gp > 1) {
        // fixed buffers for the replayed levels, sized from the tree and a
        // sixteenth of the free memory
        size_t freeb = 0, totb = 0;
        FNN_HIP(hipMemGetInfo(&freeb, &totb));
        const long long room = (long long)(freeb / 16 / sizeof(int2));
        cap_cur = cap_next = std::max(nroot, std::min(room / 4,
                                                      std::max<long long>(1ll << 20, 16 * T->nq)));
        cap_int = std::min(room / 2, std::max<long long>(1ll << 22, 256 * T->npacks));
        if (list_cap > 0) {  // small buffers force the stop and the eager finish
            cap_cur = cap_next = std::max(nroot, list_cap);
            cap_int = list_cap;
        }
    } else {
        cap_cur = std::max<long long>(1 << 16, nroot);
        cap_next = 1 << 16;
        cap_int = std::max<long long>(1 << 20, T->npacks * 16);
    }
    int2 *cur = S.get<int2>(cap_cur), *next = S.get<int2>(cap_next);
    int2 *inter = S.get<int2>(cap_int);
    int2 root = cross ? make_int2(T->cross_a, T->cross_b) : make_int2(T->qroot, T->qroot);
    if (T->ncloud > 1 && !cross)
        FNN_LAUNCH(k_forest_frontier, dim3(grid_for(nroot, 256)), dim3(256), 0, s,
                   Q, cur, (int)nroot);
    else
        FNN_HIP(hipMemcpyAsync(cur, &root, sizeof(int2), hipMemcpyHostToDevice, s));
    long long ncur = nroot, ninter = 0, tests = 0;
    fill(ovf, 0, 2, s);

    if (gp > 1 && ncur > 0) {
        const unsigned long long init[5] = {(unsigned long long)ncur, 0ull, 0ull, 0ull, 0ull};
        FNN_HIP(hipMemcpyAsync(cnt, init, sizeof init, hipMemcpyHostToDevice, s));
        int2 *buf[2] = {cur, next};
        GraphRun gr;
        gr.begin();
        for (int k = 0; k < gp; ++k) {
            const int a = k & 1;  // this level's frontier: buf[a], length cnt[a]
            FNN_LAUNCH(k_expand_bound_d, dim3(256), dim3(256), 0, gr.cs, Q, buf[a], cnt + a,
                       cap_cur, ovf + 1, cnt + 4);
            FNN_LAUNCH(k_level_guard, dim3(1), dim3(1), 0, gr.cs, cnt + a, cnt + 4, cnt + 2,
                       cap_cur, cap_int, a, ovf + 1, cnt + (1 - a));
            Emit E{buf[1 - a], inter, cnt + (1 - a), cnt + 2, cnt + 3, cap_cur, cap_int, ovf};
            launch_expand<M>(P, Q, pr, buf[a], 0, cnt + a, ovf + 1, E, gr.cs);
        }
        gr.end();
        // a tree of depth D takes about 2 D levels; past a generous multiple
        // the eager loop takes over from the frontier in buf[0]
        const int max_replays = (int)(4 * (T->depth + 8) / gp + 4);
        for (int r = 0;; ++r) {
            if (r >= max_replays) {
                cur = buf[0];
                next = buf[1];
                break;
            }
            gr.launch(s);
            unsigned long long hc[5];
            int hf[2];
            FNN_HIP(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, s));
            FNN_HIP(hipMemcpyAsync(hf, ovf, sizeof hf, hipMemcpyDeviceToHost, s));
            FNN_HIP(hipStreamSynchronize(s));
            if (hf[0])
                fail(FNN_EINTERNAL, "traversal emitted more pairs than its bound");
            ninter = (long long)hc[2];
            tests = (long long)hc[3];
            if (hf[1]) {  // continue eagerly from the stopped level's frontier
                const int a = hf[1] - 1;
                ncur = (long long)hc[a];
                cur = buf[a];
                next = buf[1 - a];
                break;
            }
            ncur = (long long)hc[0];  // gp is even: the frontier is back in buf[0]
            if (ncur == 0)
                break;
        }
    }
    while (ncur > 0) {
        // bound the level's output and size both buffers before running it
        fill(cnt + 4, 0ull, 1, s);
        FNN_LAUNCH(k_expand_bound, dim3(grid_for(ncur, 256)), dim3(256), 0, s, Q,
                   cur, ncur, cnt + 4);
        const long long bnd = (long long)read_scalar(cnt + 4, s);
        if (bnd > cap_next) {
            S.release(next);
            cap_next = bnd + bnd / 8 + 1024;
            next = S.get<int2>(cap_next);
        }
        if (ninter + bnd > cap_int) {
            long long nc = std::max(cap_int * 2, ninter + bnd + (ninter + bnd) / 8);
            int2 *ni = S.get<int2>(nc);
            if (ninter > 0)
                FNN_HIP(hipMemcpyAsync(ni, inter, sizeof(int2) * ninter,
                                       hipMemcpyDeviceToDevice, s));
            S.release(inter);
            inter = ni;
            cap_int = nc;
        }
        const unsigned long long init[3] = {0ull, (unsigned long long)ninter, 0ull};
        FNN_HIP(hipMemcpyAsync(cnt + 1, init, sizeof init, hipMemcpyHostToDevice, s));
        fill(ovf, 0, 1, s);
        Emit E{next, inter, cnt + 1, cnt + 2, cnt + 3, cap_next, cap_int, ovf};
        launch_expand<M>(P, Q, pr, cur, ncur, nullptr, nullptr, E, s);
        unsigned long long hc[3];
        int hov = 0;
        FNN_HIP(hipMemcpyAsync(hc, cnt + 1, sizeof hc, hipMemcpyDeviceToHost, s));
        FNN_HIP(hipMemcpyAsync(&hov, ovf, sizeof(int), hipMemcpyDeviceToHost, s));
        FNN_HIP(hipStreamSynchronize(s));
        if (hov)
            fail(FNN_EINTERNAL, "traversal emitted more pairs than its bound");
        ncur = (long long)hc[0];
        ninter = (long long)hc[1];
        tests += (long long)hc[2];
        std::swap(cur, next);
        std::swap(cap_cur, cap_next);
    }
    *inter_out = inter;
    *ninter_out = ninter;
    st.traverse_tests = tests;
    st.interactions = ninter;
}

template <int M>
static void launch_tiles(int mode, const Pts &P, const int2 *inter,
                         long long ninter, const fnn_tree *T, const Thr &E,
                         const CloudThr *ct, int fp64_dist, const TileOut &o,
                         hipStream_t s)
{
    if (ninter <= 0)
        return;
    const dim3 g(grid_cap(ninter, 1, 65536));
    if (mode == TILE_FILL)
        FNN_LAUNCH((k_tile<M, TILE_FILL>), g, dim3(TT), 0, s, P, inter, ninter,
                   T->q_pt_begin, T->q_pt_end, T->perm, E, ct, T->pcl, fp64_dist,
                   o);
    else if (mode == TILE_LIST)
        FNN_LAUNCH((k_tile<M, TILE_LIST>), g, dim3(TT), 0, s, P, inter, ninter,
                   T->q_pt_begin, T->q_pt_end, T->perm, E, ct, T->pcl, fp64_dist,
                   o);
    else
        FNN_LAUNCH((k_tile<M, TILE_COUNT>), g, dim3(TT), 0, s, P, inter, ninter,
                   T->q_pt_begin, T->q_pt_end, T->perm, E, ct, T->pcl, fp64_dist,
                   o);
}

// Upper bound of the point pairs the tiles of an interaction list evaluate.
__global__ void k_pair_bound(const int2 *__restrict__ inter, long long ni,
                             const int32_t *__restrict__ q_pb,
                             const int32_t *__restrict__ q_pe,
                             unsigned long long *__restrict__ out)
{
    unsigned long long b = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ni;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 p = inter[i];
        const unsigned long long na = q_pe[p.x] - q_pb[p.x], nb = q_pe[p.y] - q_pb[p.y];
        b += p.x == p.y ? na * (na - 1) / 2 : na * nb;
    }
    b = wave_sum(b);
    if ((threadIdx.x & (WAVE - 1)) == 0 && b)
        atomicAdd(out, b);
}

// Sorts every CSR row by column (entries are (column, distance) pairs):
// rows of up to 512 entries by one wave, up to 4096 by one wave or four,
// up to 16384 by sixteen waves, longer rows in a global buffer.  pk: the
// entries packed as (column << 32 | distance bits) in their slots, when the
// fill wrote them so (col and dist are then written here); null: they are
// in col and dist.
void sort_csr_rows(const int64_t *row_ptr, int n, int32_t *col, float *dist,
                   int64_t nnz, Scratch &S, const unsigned long long *pk)
{
    hipStream_t s = S.stream();
    int32_t *mid = S.get<int32_t>(n), *lng = S.get<int32_t>(n);
    int32_t *cc = S.get<int32_t>(2);
    fill(cc, 0, 2, s);
    if (nnz > 0) {
        FNN_LAUNCH(k_sort_small, dim3(grid_cap(n, 4, 16384)), dim3(256), 0, s,
                   row_ptr, n, col, dist, mid, lng, cc, pk);
        int32_t hcc[2];
        FNN_HIP(hipMemcpyAsync(hcc, cc, sizeof hcc, hipMemcpyDeviceToHost, s));
        FNN_HIP(hipStreamSynchronize(s));
        if (hcc[0] > 0) {
            FNN_LAUNCH(k_sort_wave, dim3(grid_cap(hcc[0], 4, 4096)), dim3(256), 0, s,
                       row_ptr, mid, hcc[0], col, dist);
            FNN_LAUNCH(k_sort_blk<4>, dim3(grid_cap(hcc[0], 1, 4096)), dim3(4 * WAVE), 0,
                       s, row_ptr, mid, hcc[0], 32 * WAVE, col, dist);
        }
        if (hcc[1] > 0) {
            int64_t *p2 = S.get<int64_t>(hcc[1] + 1);
            int64_t *soff = S.get<int64_t>(hcc[1] + 2);
            FNN_LAUNCH(k_long_sizes, dim3(grid_for(hcc[1], 256)), dim3(256), 0, s,
                       row_ptr, lng, hcc[1], p2);
            scan_i64(p2, soff, hcc[1], S);
            const int64_t tot = read_scalar(soff + hcc[1], s);
            unsigned long long *scr = S.get<unsigned long long>(tot);
            FNN_LAUNCH(k_sort_blk<16>, dim3(grid_cap(hcc[1], 1, 4096)), dim3(16 * WAVE), 0,
                       s, row_ptr, lng, hcc[1], 64 * WAVE, col, dist);
            FNN_LAUNCH(k_sort_long, dim3(hcc[1]), dim3(256), 0, s, row_ptr, lng,
                       soff, scr, col, dist);
        }
    }
}

// ---- LPT work order from the cost model (learned schedule) ----------------
//
// Graham's LPT rule takes jobs in decreasing size and gives each to the
// machine that becomes free first (the paper uses it to place Voronoi cells
// on processes, Section IV-D); it is within 4/3 of the best makespan.  Here
// the jobs are the tile pass's pack pairs, the machines its work-groups, and
// the sizes the cost model's predictions, so heavy pairs start first and no
// work-group is left with a long pair at the end.

// Predicted edge density of every pack: its points' predicted degrees over
// the point pairs its predicted block pairs hold.
__global__ void k_pack_density(const float *__restrict__ pred,
                               const int32_t *__restrict__ q_pb,
                               const int32_t *__restrict__ q_pe, int nn, int npk,
                               float *__restrict__ rho)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npk;
         k += gridDim.x * blockDim.x) {
        const int b = q_pb[nn + k], e = q_pe[nn + k];
        float deg = 0.f;
        for (int p = b; p < e; ++p)
            deg += fmaxf(expm1f(fminf(pred[2 * p + 1], 30.f)), 0.f);
        const float vis = b < e ? fmaxf(expm1f(fminf(pred[2 * b], 30.f)), 1.f) : 1.f;
        rho[k] = deg / ((float)max(e - b, 1) * (float)GP_TILE * vis);
    }
}

// Sort key of every pack pair: its predicted cost (pair evaluations at
// dp-proportional cost plus emitted edges), largest first.
__global__ void k_item_cost(const int2 *__restrict__ inter, long long ni,
                            const int32_t *__restrict__ q_pb,
                            const int32_t *__restrict__ q_pe, int nn,
                            const float *__restrict__ rho, float pair_cost,
                            float edge_cost, uint32_t *__restrict__ key,
                            uint32_t *__restrict__ val)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ni;
         i += (long long)gridDim.x * blockDim.x) {
        const int2 pr = inter[i];
        const float na = (float)(q_pe[pr.x] - q_pb[pr.x]);
        const float nb = (float)(q_pe[pr.y] - q_pb[pr.y]);
        const float pairs = pr.x == pr.y ? 0.5f * na * (na - 1.f) : na * nb;
        const float ra = pr.x >= nn ? rho[pr.x - nn] : 0.f;
        const float rb = pr.y >= nn ? rho[pr.y - nn] : 0.f;
        const float cost = pairs * (pair_cost + edge_cost * fminf(ra + rb, 2.f));
        key[i] = ~__float_as_uint(fmaxf(cost, 0.f));  // descending
        val[i] = (uint32_t)i;
    }
}

// Learned-schedule state of one query.
struct Learned {
    const float *model = nullptr;  // device parameters (null: no model)
    float *feat = nullptr;         // [n][16] tree order
    float *pred = nullptr;         // [n][2]
    float *targ = nullptr;         // [n][2] (trace)
};

const float *cost_model_device();

template <int M>
static void eps_graph_impl(const fnn_tree *Tc, const double *epsv,
                           const Options &opt, fnn_csr *C, fnn_stats &st,
                           Scratch &S, float **trace_feat, float **trace_targ)
{
    fnn_tree *T = const_cast<fnn_tree *>(Tc);  // lazily built caches only
    if (T->cross_a >= 0 && (opt.sched == FNN_SCHED_LEARNED || opt.trace))
        fail(FNN_EUNSUPPORTED, "bichromatic queries run the two-pass schedule, without traces");
    if (opt.precision == FNN_PREC_I8 && (M != M_HAM || T->dp > 4))
        fail(FNN_EUNSUPPORTED, "integer MFMA filter is for Hamming codes of <= 256 bits");
    hipStream_t s = S.stream();
    const int n = (int)T->n;
    Timer tm(s);
    tm.mark();  // 0

    Pts P{};
    P.metric = M;
    P.n = n;
    P.dim = T->dim;
    P.dp = T->dp;
    P.W = T->W;
    P.sigma = T->sigma;
    P.x = T->x;
    P.xn = T->xn;
    P.h = T->h;
    P.s = T->s;
    P.len = T->len;
    P.peq = T->peq;

    QView Q{T->q_center_pos, T->q_pt_begin, T->q_pt_end, T->q_kbeg,
            T->q_kcnt,       T->q_kids,     T->q_radius, (int)T->nnodes};
    // thresholds of every cloud (one entry for an ordinary tree)
    const int ncl = T->ncloud;
    std::vector<CloudThr> ct_h(ncl);
    for (int c = 0; c < ncl; ++c) {
        const double e = epsv[c];
        CloudThr &t = ct_h[c];
        t.E = make_thr_eps(M, T->dp, e);
        t.peps = (M == M_HAM || M == M_LEV) ? t.E.lo : (float)e;
        if (M == M_ANG && e >= M_PI)
            t.peps = 4.f;  // every pair may touch
        t.e2f = gram_eps2(M, e, t.E);
        t.feps = std::max(t.peps, 0.5f);
        t.pad_ = 0.f;
    }
    CloudThr *ct_d = S.get<CloudThr>(ncl);
    FNN_HIP(hipMemcpyAsync(ct_d, ct_h.data(), sizeof(CloudThr) * ncl,
                           hipMemcpyHostToDevice, s));
    const Thr E = ct_h[0].E;
    const double eps = epsv[0];
    Prune pr;
    const double u = 1.0 / 16777216.0;
    pr.rel = (float)std::max(1e-4, 8.0 * (T->dp + 4) * u);
    pr.abs_ = M == M_ANG ? 1e-5f : (M == M_L2 ? 1e-30f : 0.f);
    pr.eps = ct_h[0].peps;
    pr.ct = ncl > 1 ? ct_d : nullptr;
    pr.pcl = ncl > 1 ? T->pcl : nullptr;
    const int fp64_dist = (M == M_ANG) || (M == M_L2 && (T->dim + 2) * u > 1e-5);
    const bool learned = opt.sched == FNN_SCHED_LEARNED;

    // ---- learned cost model: features and predictions ------------------
    Learned Lm;
    if (learned || opt.trace) {
        tree_aux(T, S);
        Lm.feat = opt.trace ? (float *)out_alloc(sizeof(float) * MLP_F * (size_t)n)
                            : S.get<float>((size_t)n * MLP_F);
        if (opt.trace)
            *trace_feat = Lm.feat;
        compute_features(T, P, ct_h[0].feps, ncl > 1 ? ct_d : nullptr, Lm.feat, s);
    }
    if (learned) {
        Lm.model = cost_model_device();
        if (!Lm.model)
            fail(FNN_EINVAL, "learned schedule requested but no cost model is set");
        Lm.pred = S.get<float>(2 * (size_t)n);
        mlp_forward(Lm.model, Lm.feat, n, Lm.pred, s);
    }

    double t2min = HUGE_VAL;  // smallest squared threshold of the filter's key
    for (int c = 0; c < ncl; ++c)
        t2min = std::min(t2min, gram_t2(M, epsv[c], ct_h[c].E));
    // filter precision: the caller's, or (automatic) the MFMA filter where it
    // pays: int8 on short Hamming codes; FP16 on vector data of 16..128
    // coordinates when its rounding margin is small against eps^2
    int prec = opt.precision;
    GramPre gpre;  // the rule's centres and largest |x - mu|, reused below
    if (prec == FNN_PREC_AUTO) {
        prec = FNN_PREC_FP32;
        if (M == M_HAM && T->dp <= 4)
            prec = FNN_PREC_I8;
        if ((M == M_L2 || M == M_ANG) && T->dim >= 16 && T->dp <= 128 &&
            gram_margin_ratio(T, t2min, FNN_PREC_FP16, S, &gpre) <= 0.5)
            prec = FNN_PREC_FP16;
    }
    st.precision_used = prec;
    const bool use_gram = ((M == M_L2 || M == M_ANG) && prec != FNN_PREC_FP32) ||
                          (M == M_HAM && prec == FNN_PREC_I8);

    // ---- traversal ------------------------------------------------------
    // Where the traversal's own pack-level test would keep nearly every pack
    // pair (high-dimensional data), the MFMA filter takes every pair from a
    // closed-form list instead; a seeded sample of pack pairs decides.  Any
    // pair set that contains the needed ones gives the exact graph.
    int2 *inter = nullptr;
    long long ninter = 0;
    bool dense = false;
    if (use_gram && ncl == 1 && !opt.trace && T->npacks >= 256 && gram_packs_fit(T, S)) {
        const int ns = 8192;
        unsigned long long *pc = S.get<unsigned long long>(1);
        fill(pc, 0ull, 1, s);
        FNN_LAUNCH((k_prune_sample<M>), dim3(ns / 256), dim3(256), 0, s, P, Q, pr,
                   (int)T->npacks, ns, pc);
        const unsigned long long pruned = read_scalar(pc, s);
        dense = pruned * 100 <= (unsigned long long)ns;  // at most 1 % prunable
        st.traverse_tests = ns;
    }
    if (dense) {
        ninter = (long long)T->npacks * (T->npacks + 1) / 2;
        st.interactions = ninter;
    } else {
        traverse<M>(T, P, Q, pr, S,
                    opt.graph_passes <= 1 ? 1 : (opt.graph_passes + 1) / 2 * 2,
                    opt.list_cap, &inter, &ninter, st);
    }
    tm.mark();  // 1

    // ---- MFMA filter set-up (vector metrics with dim <= 128, Hamming codes
    // of <= 256 bits) ------------------------------------------------------
    GramArgs G{};
    G.cross = T->cross_a >= 0;
    int2 *plain = inter;
    long long nplain = ninter;
    if constexpr (M == M_L2 || M == M_ANG || M == M_HAM) {
        if (use_gram) {
            gram_prepare(T, prec, opt.proj, eps, E, t2min, inter, ninter, S, G,
                         &plain, &nplain, &gpre);
            G.fp64_dist = fp64_dist;
            G.validate = opt.validate;
            G.perm = T->perm;
            gram_pad_packs(M, prec, G, S);
            G.ct = ncl > 1 ? ct_d : nullptr;
            G.pcl = ncl > 1 ? T->pcl : nullptr;
            if (ncl > 1 && (G.t2mul != 1.0 || G.e2add != 0.0)) {
                // the filter's per-cloud eps^2 on principal coordinates or
                // in scaled units
                std::vector<CloudThr> cg(ct_h);
                for (int c = 0; c < ncl; ++c)
                    cg[c].e2f = gram_eps2(M, epsv[c], cg[c].E, G.t2mul, G.e2add);
                CloudThr *cg_d = S.get<CloudThr>(ncl);
                FNN_HIP(hipMemcpyAsync(cg_d, cg.data(), sizeof(CloudThr) * ncl,
                                       hipMemcpyHostToDevice, s));
                FNN_HIP(hipStreamSynchronize(s));  // cg goes out of scope
                G.ct = cg_d;
            }
            st.proj_dim = G.proj;
            st.proj_captured = G.captured;
        }
    }
    tm.mark();  // 2

    // [0..5] see TileOut, [6..7] the learned path's re-fill, [8] sum of the
    // exact integer filter's position degrees (twice its edges)
    unsigned long long *cnt = S.get<unsigned long long>(9);
    fill(cnt, 0ull, 9, s);
    TileOut o{};
    o.cnt = cnt;
    int *bad = S.get<int>(1);
    fill(bad, 0, 1, s);
    o.err = bad;
    C->n = n;
    C->row_ptr = (int64_t *)out_alloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t nnz = 0;
    int64_t novf = 0;
    unsigned long long *packed = nullptr;  // packed CSR entries (see k_place_packed)
    unsigned long long hc0[9] = {0};

    if (use_gram || !learned) {
        // ---- count pass (plain tiles) / filter + exact survivors (MFMA) ---
        o.deg = S.get<int32_t>(n);
        fill(o.deg, 0, n, s);
        int2 *gedges = nullptr;
        float *gedist = nullptr;
        long long ngedges = 0;
        if (use_gram) {
            unsigned long long *ns = S.get<unsigned long long>(2);
            Events fev(s);
            // survivor list: up to 512 entries per point while they fit in
            // a sixteenth of the free device memory, at least 64 per point
            // (the ~500-neighbour C2 radius passes ~427 per point through
            // the filter, so one filter pass suffices there)
            size_t freeb = 0, totb = 0;
            FNN_HIP(hipMemGetInfo(&freeb, &totb));
            const long long room = (long long)(freeb / 16 / sizeof(int2));
            long long cap = std::max({1ll << 24, 64ll * n, std::min(room, 512ll * n)});
            if (learned) {
                // predicted ordered edges / 2, times the filter's survivor
                // factor (BF16 ~1.5, FP8 tens on high-dimensional data)
                double *acc = S.get<double>(3);
                fill(acc, 0.0, 3, s);
                int64_t *zero_rp = S.get<int64_t>(n + 1);
                fill(zero_rp, (int64_t)0, n + 1, s);
                FNN_LAUNCH(k_pred_err, dim3(grid_for(n, 256)), dim3(256), 0, s,
                           Lm.pred, T->perm, zero_rp, n, acc);
                double hacc[3];
                FNN_HIP(hipMemcpyAsync(hacc, acc, sizeof hacc, hipMemcpyDeviceToHost, s));
                FNN_HIP(hipStreamSynchronize(s));
                const double fac = prec == FNN_PREC_I8     ? 1.25
                                   : prec == FNN_PREC_BF16 || prec == FNN_PREC_FP16 ? 2.5
                                                                    : 40.0;
                cap = std::max<long long>(1ll << 20, (long long)(0.5 * hacc[1] * fac));
            }
            if (opt.validate)
                cap = std::max<long long>(cap, (long long)n * (n - 1) / 2 + 1);
            if (opt.list_cap > 0)
                cap = opt.list_cap;
            // the integer filter on Hamming codes is exact: unless validating,
            // it writes the edges, their distances and the degrees itself
            const bool direct = M == M_HAM && !opt.validate;
            int32_t *degp = direct ? S.get<int32_t>(n) : nullptr;
            for (int attempt = 0;; ++attempt) {
                // a list (and its decided edges) larger than the device
                // cannot be allocated: say so before asking
                if ((double)cap * (sizeof(int2) + sizeof(int2) + sizeof(float)) > (double)totb)
                    fail(FNN_ENOMEM, "survivor list of %lld entries exceeds device memory",
                         (long long)cap);
                G.surv = S.get<int2>(cap);
                G.surv_cap = cap;
                G.nsurv = ns;
                if (direct) {
                    G.degp = degp;
                    fill(degp, 0, n, s);
                }
                fill(ns, 0ull, 2, s);
                fill(cnt + 2, 0ull, 1, s);
                FNN_HIP(hipEventRecord(fev[0], s));
                gram_launch(M, prec, false, P, G, o, s);
                FNN_HIP(hipEventRecord(fev[1], s));
                const long long got = (long long)read_scalar(ns, s);
                if (got <= cap || attempt > 0) {
                    if (got > cap)
                        fail(FNN_EINTERNAL, "survivor list overflow");
                    {
                        float fms = 0.f;
                        FNN_HIP(hipEventSynchronize(fev[1]));
                        FNN_HIP(hipEventElapsedTime(&fms, fev[0], fev[1]));
                        st.filter_ms = fms;
                    }
                    if (direct) {
                        degrees_from_positions(degp, T->perm, n, o.deg, cnt + 8, s);
                        gedges = G.surv;
                        ngedges = got;
                    } else {
                        // with no plain tiles in the query every CSR entry
                        // comes from a survivor: keep the ranks its degree
                        // counters return and place it without cursors
                        // (measured at C2: 2.2 ms faster at ~53 survivors per
                        // point, 15 ms at ~350), while the ranks take under a
                        // quarter of the free device memory
                        size_t free_now = 0, tot_now = 0;
                        FNN_HIP(hipMemGetInfo(&free_now, &tot_now));
                        const bool ranks =
                            nplain == 0 &&
                            (double)(got + 1) * sizeof(int2) < 0.25 * (double)free_now;
                        gedges = S.get<int2>(got + 1);
                        gedist = S.get<float>(got + 1);
                        if (ranks)
                            G.erank = S.get<int2>(got + 1);
                        // slot per survivor: holes where it is no edge
                        survivors_launch(M, P, G, got, gedges, gedist, o, s);
                        ngedges = got;
                    }
                    break;
                }
                S.release(G.surv);
                cap = got + got / 8 + 1024;
                ++novf;  // a second filter pass was needed
            }
        }
        // Plain tiles: count degrees and append each edge, in both
        // directions, to an edge list, so the fill needs no second tile
        // pass.  The list holds up to 512 entries per point (bounded by
        // twice the pairs the tiles can evaluate and by an eighth of the
        // free device memory); if it overflows, the fill pass runs instead.
        bool listed = false;
        long long nlisted = 0;
        if (nplain > 0) {
            unsigned long long *pb_ = S.get<unsigned long long>(1);
            fill(pb_, 0ull, 1, s);
            FNN_LAUNCH(k_pair_bound, dim3(grid_for(nplain, 256)), dim3(256), 0, s,
                       plain, nplain, T->q_pt_begin, T->q_pt_end, pb_);
            const unsigned long long bound = read_scalar(pb_, s);
            size_t freeb = 0, totb = 0;
            FNN_HIP(hipMemGetInfo(&freeb, &totb));
            const unsigned long long room = (unsigned long long)(freeb / 8 / 12);
            o.ecap = std::max<unsigned long long>(
                1024, std::min({2 * bound, room, 512ull * (unsigned long long)n}));
            if (opt.list_cap > 0)
                o.ecap = (unsigned long long)opt.list_cap;
            o.elist = S.get<int2>(o.ecap);
            o.edist = S.get<float>(o.ecap);
            o.ecnt = S.get<unsigned long long>(1);
            fill(o.ecnt, 0ull, 1, s);
            launch_tiles<M>(TILE_LIST, P, plain, nplain, T, E, ct_d, fp64_dist, o, s);
            nlisted = (long long)read_scalar(o.ecnt, s);
            listed = (unsigned long long)nlisted <= o.ecap;
        }
        tm.mark();  // 3

        scan_i32_to_i64(o.deg, C->row_ptr, n, S);
        nnz = read_scalar(C->row_ptr + n, s);
        C->nnz = nnz;
        FNN_HIP(hipMemcpy(hc0, cnt, sizeof hc0, hipMemcpyDeviceToHost));
        C->col = (int32_t *)out_alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
        C->dist = (float *)out_alloc(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
        tm.mark();  // 4

        // ---- fill pass --------------------------------------------------
        o.col = C->col;
        o.dist = C->dist;
        o.nnz = (unsigned long long)nnz;
        if (G.erank) {
            // every entry at its row start plus its rank: the ranks of a row
            // are distinct and below its degree, so the rows fill exactly
            // (a rank past its row raises ERR_INDEX)
            if (nnz > 0) {
                // packed entries while a copy of the CSR's nnz fits easily
                size_t free_now = 0, tot_now = 0;
                FNN_HIP(hipMemGetInfo(&free_now, &tot_now));
                if ((double)nnz * sizeof(unsigned long long) < 0.25 * (double)free_now) {
                    packed = S.get<unsigned long long>(nnz);
                    st.fill_path = 2;
                    FNN_LAUNCH(k_place_packed, dim3(grid_cap(ngedges, 256, 65536)), dim3(256),
                               0, s, gedges, gedist, G.erank, ngedges, C->row_ptr, packed,
                               o.err);
                } else {
                    edges_place(gedges, gedist, G.erank, ngedges, C->row_ptr, o, s);
                    st.fill_path = 1;
                }
            }
        } else {
            o.cursor = S.get<unsigned long long>(n);
            FNN_LAUNCH(k_cursor_init, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       C->row_ptr, n, o.cursor);
            if (nnz > 0) {
                if (G.degp)
                    edges_scatter_ham(gedges, ngedges, P, T->perm, o, s);
                else if (use_gram)
                    edges_scatter(gedges, gedist, ngedges, true, o, s);
                if (listed)
                    edges_scatter(o.elist, o.edist, nlisted, false, o, s);
                else
                    launch_tiles<M>(TILE_FILL, P, plain, nplain, T, E, ct_d, fp64_dist,
                                    o, s);
            }
            FNN_LAUNCH(k_cursor_check_rows, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       C->row_ptr, n, o.cursor, (const int32_t *)nullptr, bad);
        }
        tm.mark();  // 5
    } else {
        // ---- learned schedule: one tile pass into predicted slots ----------
        int32_t *cap = S.get<int32_t>(n);
        const float slack = opt.slack_pct / 100.f;
        FNN_LAUNCH(k_caps, dim3(grid_for(n, 256)), dim3(256), 0, s, Lm.pred, T->perm,
                   n, slack, cap);
        int64_t *sb = S.get<int64_t>(n + 1);
        scan_i32_to_i64(cap, sb, n, S);
        const int64_t nslot = read_scalar(sb + n, s);
        int32_t *scol = S.get<int32_t>(std::max<int64_t>(nslot, 1));
        float *sdist = S.get<float>(std::max<int64_t>(nslot, 1));
        int32_t *ovf = S.get<int32_t>(n);
        fill(ovf, 0, n, s);
        o.cursor = S.get<unsigned long long>(n);
        FNN_LAUNCH(k_cursor_init, dim3(grid_for(n, 256)), dim3(256), 0, s, sb, n,
                   o.cursor);
        o.col = scol;
        o.dist = sdist;
        o.nnz = (unsigned long long)nslot;
        o.row_end = sb + 1;
        o.ovf = ovf;
        const long long spcap = std::max<long long>(1ll << 16, nslot / 2);
        o.spill = S.get<int2>(spcap);
        fill(o.spill, make_int2(-1, -1), spcap, s);
        o.spill_dist = S.get<float>(spcap);
        o.spill_cnt = S.get<unsigned long long>(1);
        fill(o.spill_cnt, 0ull, 1, s);
        o.spill_cap = (unsigned long long)spcap;
        {
            // LPT order of the pack pairs by predicted cost; work-groups take
            // them through a counter
            TileOut om = o;
            if (nplain > 0 && opt.lpt) {
                const int npk = (int)T->npacks;
                float *rho = S.get<float>(npk + 1);
                FNN_LAUNCH(k_pack_density, dim3(grid_for(npk, 256)), dim3(256), 0, s,
                           Lm.pred, T->q_pt_begin, T->q_pt_end, (int)T->nnodes, npk, rho);
                uint32_t *k1 = S.get<uint32_t>(nplain), *v1 = S.get<uint32_t>(nplain);
                uint32_t *k2 = S.get<uint32_t>(nplain), *v2 = S.get<uint32_t>(nplain);
                // a pair costs about dp multiply-adds, an emitted edge about
                // 16 instructions (cursor atomic, two stores, bookkeeping)
                FNN_LAUNCH(k_item_cost, dim3(grid_for(nplain, 256)), dim3(256), 0, s,
                           plain, nplain, T->q_pt_begin, T->q_pt_end, (int)T->nnodes, rho,
                           (float)std::max(T->dp, 4), 16.f, k1, v1);
                radix_sort_pairs(k1, v1, k2, v2, nplain, 32, S);
                om.order = v2;
                om.next = S.get<unsigned long long>(1);
                fill(om.next, 0ull, 1, s);
            }
            launch_tiles<M>(TILE_FILL, P, plain, nplain, T, E, ct_d, fp64_dist, om, s);
        }
        tm.mark();  // 3
        // cursors advanced by every edge, written or not: exact degrees
        o.deg = S.get<int32_t>(n);
        FNN_LAUNCH(k_deg_from_cursor, dim3(grid_for(n, 256)), dim3(256), 0, s,
                   o.cursor, sb, n, o.deg);
        scan_i32_to_i64(o.deg, C->row_ptr, n, S);
        nnz = read_scalar(C->row_ptr + n, s);
        C->nnz = nnz;
        FNN_HIP(hipMemcpy(hc0, cnt, sizeof hc0, hipMemcpyDeviceToHost));
        C->col = (int32_t *)out_alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
        C->dist = (float *)out_alloc(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
        tm.mark();  // 4
        int32_t *nov = S.get<int32_t>(1);
        fill(nov, 0, 1, s);
        FNN_LAUNCH(k_compact, dim3(grid_cap(n, 4, 16384)), dim3(256), 0, s, sb, scol, sdist,
                   ovf, C->row_ptr, n, C->col, C->dist, nov);
        novf = read_scalar(nov, s);
        {
            const long long nsp = std::min<long long>(
                (long long)read_scalar(o.spill_cnt, s), spcap);
            unsigned long long *cur3 = S.get<unsigned long long>(n);
            FNN_LAUNCH(k_spill_init, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       C->row_ptr, sb, n, cur3);
            if (nsp > 0)
                FNN_LAUNCH(k_spill_scatter, dim3(grid_for(nsp, 256)), dim3(256), 0,
                           s, o.spill, o.spill_dist, nsp, n, ovf, cur3, C->row_ptr,
                           C->col, C->dist, bad);
            // rows that were not re-done must now be complete
            int32_t *keep = S.get<int32_t>(n);
            FNN_LAUNCH(k_not, dim3(grid_for(n, 256)), dim3(256), 0, s, ovf, n, keep);
            FNN_LAUNCH(k_cursor_check_rows, dim3(grid_for(n, 256)), dim3(256), 0,
                       s, C->row_ptr, n, cur3, keep, bad);
            st.spilled = nsp;
        }
        if (novf > 0) {
            // overflowed rows: re-run the tiles of the packs holding them,
            // writing only those rows, straight into the CSR
            int32_t *pflag = S.get<int32_t>(T->nq);
            fill(pflag, 0, T->nq, s);
            FNN_LAUNCH(k_mark_packs, dim3(grid_for(n, 256)), dim3(256), 0, s, ovf,
                       T->perm, T->pack_of, n, pflag);
            int2 *sub = S.get<int2>(nplain + 1);
            unsigned long long *sc = S.get<unsigned long long>(1);
            fill(sc, 0ull, 1, s);
            FNN_LAUNCH(k_sublist, dim3(grid_for(nplain, 256)), dim3(256), 0, s,
                       plain, nplain, pflag, sub, sc);
            const long long nsub = (long long)read_scalar(sc, s);
            TileOut o2 = o;
            o2.order = nullptr;  // the sub-list runs in its own order
            o2.next = nullptr;
            o2.cnt = cnt + 6;  // keep the pass counters of the main pass
            o2.row_end = nullptr;
            o2.ovf = nullptr;
            o2.row_filter = ovf;
            o2.col = C->col;
            o2.dist = C->dist;
            o2.nnz = (unsigned long long)nnz;
            o2.cursor = S.get<unsigned long long>(n);
            FNN_LAUNCH(k_cursor_init, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       C->row_ptr, n, o2.cursor);
            launch_tiles<M>(TILE_FILL, P, sub, nsub, T, E, ct_d, fp64_dist, o2, s);
            FNN_LAUNCH(k_cursor_check_rows, dim3(grid_for(n, 256)), dim3(256), 0,
                       s, C->row_ptr, n, o2.cursor, ovf, bad);
        }
        tm.mark();  // 5
    }

    // ---- per-row sort ---------------------------------------------------
    sort_csr_rows(C->row_ptr, n, C->col, C->dist, nnz, S, packed);
    tm.mark();  // 6

    // ---- trace targets, prediction error ---------------------------------
    if (opt.trace) {
        int32_t *vis = S.get<int32_t>(T->npacks + 1);
        fill(vis, 0, T->npacks + 1, s);
        FNN_LAUNCH(k_visits, dim3(grid_for(ninter, 256)), dim3(256), 0, s, inter,
                   ninter, (int)T->nnodes, vis);
        Lm.targ = (float *)out_alloc(sizeof(float) * 2 * (size_t)n);
        *trace_targ = Lm.targ;
        FNN_LAUNCH(k_targets, dim3(grid_for(n, 256)), dim3(256), 0, s, vis,
                   T->pack_of, T->perm, C->row_ptr, n, (int)T->nnodes, Lm.targ);
    }
    if (learned) {
        double *acc = S.get<double>(3);
        fill(acc, 0.0, 3, s);
        FNN_LAUNCH(k_pred_err, dim3(grid_for(n, 256)), dim3(256), 0, s, Lm.pred,
                   T->perm, C->row_ptr, n, acc);
        double hacc[3];
        FNN_HIP(hipMemcpyAsync(hacc, acc, sizeof hacc, hipMemcpyDeviceToHost, s));
        FNN_HIP(hipStreamSynchronize(s));
        st.pred_mae = hacc[0] / std::max(n, 1);
        st.pred_sum_ratio = hacc[2] > 0 ? hacc[1] / hacc[2] : 0.0;
    }
    int hbad = 0;
    FNN_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    if (hbad)
        fail(FNN_EINTERNAL, "count and fill passes disagree");

    st.n = n;
    st.nodes = T->nnodes;
    st.packs = T->npacks;
    hc0[3] += hc0[8] / 2;  // exact integer filter: its edges are its survivors
    st.tile_pairs = (int64_t)(hc0[0] + hc0[3]);
    st.fp64_rechecks = (int64_t)hc0[1];
    st.filter_pairs = (int64_t)hc0[2];
    st.filter_survivors = (int64_t)hc0[3];
    st.validate_mismatch = (int64_t)hc0[4];
    {
        unsigned eb = (unsigned)hc0[5];
        float ef;
        memcpy(&ef, &eb, 4);
        st.max_rel_err = ef;
    }
    st.overflow_rows = novf;
    st.edges = nnz;
    st.traverse_ms = tm.ms(0, 1) + tm.ms(1, 2);
    st.count_ms = tm.ms(2, 3);
    st.scan_ms = tm.ms(3, 4);
    st.fill_ms = tm.ms(4, 5);
    st.sort_ms = tm.ms(5, 6);
    st.tile_ms = st.count_ms + st.fill_ms;
    st.total_ms = tm.ms(0, 6);
}

void eps_graph(const fnn_tree *T, const double *eps, const Options &opt,
               fnn_csr *C, fnn_stats &st, Scratch &S, float **tf, float **tt)
{
    switch (T->metric) {
    case M_L2:
        eps_graph_impl<M_L2>(T, eps, opt, C, st, S, tf, tt);
        break;
    case M_ANG:
        eps_graph_impl<M_ANG>(T, eps, opt, C, st, S, tf, tt);
        break;
    case M_HAM:
        eps_graph_impl<M_HAM>(T, eps, opt, C, st, S, tf, tt);
        break;
    default:
        eps_graph_impl<M_LEV>(T, eps, opt, C, st, S, tf, tt);
        break;
    }
}

}  // namespace fnn
