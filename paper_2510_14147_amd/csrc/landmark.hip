// Landmark mode on one GPU (Section IV-D, Algorithm 5; Section IV-E,
// Lemma 1 and Algorithm 6): the epsilon-graph assembled from per-cell cover
// trees of a Voronoi partition plus the cells' epsilon-ghosts.
//
//  1. Centres: m distinct input points drawn with a seeded SplitMix64 partial
//     shuffle (the paper leaves the choice open and warns that a greedy
//     permutation can give very uneven cells).
//  2. Voronoi cells: every point goes to its nearest centre (ties to the
//     lower centre index), one pass over the m centres per point.
//  3. Ghosts (Lemma 1): if p in V_j has an eps-neighbour in V_i (i != j) then
//     d(p, c_i) <= d(p, c_j) + 2 eps.  p is listed as a ghost of every other
//     cell that passes this test.  The distances here are FP32, so the test
//     is widened by their rounding bound (which also covers a point assigned
//     to a centre that is nearest only up to rounding); extra ghosts cost
//     work, never an edge.  The paper finds these cells with a cover tree
//     over C; with m << n one coalesced pass over C per point is cheaper.
//  4. One forest over the augmented cells V_i + G_i (each cell a cloud of the
//     batched build and query).  Its self-join holds every pair inside a
//     cell, and every pair (p, q), p in V_i, q in V_j, i < j, appears in cell
//     i (q is a ghost of V_i) and in cell j (p is a ghost of V_j).
//  5. Keep a pair of augmented rows when both are members of the cell, or
//     one is a member and the other a ghost whose own cell has the larger
//     index; every ordered pair of the epsilon-graph is then kept exactly
//     once.  Rows are mapped back to input indices and sorted by column.
//
// Where Algorithm 6 queries G_i against a tree of V_i, this builds the tree
// of V_i + G_i and drops ghost-ghost pairs: the same pair set, with the
// batched forest doing the work of all cells in shared launches.
#include <math.h>

#include <algorithm>
#include <unordered_map>
#include <vector>

#include "tree.h"

namespace fnn {

Pts ingest_input(fnn_tree *T, const void *points, Scratch &S);
void sort_csr_rows(const int64_t *row_ptr, int n, int32_t *col, float *dist,
                   int64_t nnz, Scratch &S, const unsigned long long *pk);

namespace {

constexpr int LM_TPB = 256;
constexpr int LM_CBLK = 64;  // centre ids staged in LDS per step

// Distance (FP32, rounding-bounded) between rows i and j of P.
template <int M>
__device__ __forceinline__ float lm_dist(const Pts &P, int i, int j)
{
    return key_to_dist<M>(key32<M>(P, i, j));
}

// Nearest centre of every point: cell[p] and its distance dC[p].
template <int M>
__global__ void __launch_bounds__(LM_TPB)
k_voronoi(Pts P, const int32_t *__restrict__ cid, int m,
          int32_t *__restrict__ cell, float *__restrict__ dC)
{
    __shared__ int32_t sc[LM_CBLK];
    for (long long p0 = (long long)blockIdx.x * LM_TPB; p0 < P.n;
         p0 += (long long)gridDim.x * LM_TPB) {
        const int p = (int)(p0 + threadIdx.x);
        float best = INFINITY;
        int bi = 0;
        for (int c0 = 0; c0 < m; c0 += LM_CBLK) {
            __syncthreads();
            if (threadIdx.x < LM_CBLK && c0 + (int)threadIdx.x < m)
                sc[threadIdx.x] = cid[c0 + threadIdx.x];
            __syncthreads();
            const int cn = min(LM_CBLK, m - c0);
            if (p < P.n)
                for (int k = 0; k < cn; ++k) {
                    const float d = lm_dist<M>(P, p, sc[k]);
                    if (d < best) {  // strict: ties stay with the lower index
                        best = d;
                        bi = c0 + k;
                    }
                }
        }
        if (p < P.n) {
            cell[p] = bi;
            dC[p] = best;
        }
    }
}

struct GhostBound {
    float rel, abs_;  // widening of the FP32 test (vector metrics)
    float eps2;       // 2 eps (2 floor(eps) for integer metrics)
};

// Lemma 1 with rounding: centre c (not p's own) may hold an eps-neighbour
// of p only if d(p, c) <= (d(p, C) + 2 eps) (1 + rel) + abs.
template <int M>
__device__ __forceinline__ float lm_bound(const GhostBound &g, float dC)
{
    if constexpr (M == M_HAM || M == M_LEV)
        return dC + g.eps2;  // exact: small integers
    else
        return __fadd_rn(__fmul_rn(__fadd_rn(dC, g.eps2), 1.f + g.rel), g.abs_);
}

// EMIT = false: cnt[p] = 1 + the number of cells p is a ghost of, and the
// point's ghost bound gb[p] (computed once, so both passes compare the
// same FP32 values).  EMIT = true: at pos[p] .. pos[p + 1], the entries
// (2 cell + 1, p) for those cells after (2 cell[p], p) for p's own cell.
template <int M, bool EMIT>
__global__ void __launch_bounds__(LM_TPB)
k_ghosts(Pts P, const int32_t *__restrict__ cid, int m, GhostBound g,
         const int32_t *__restrict__ cell, const float *__restrict__ dC,
         float *__restrict__ gb, int32_t *__restrict__ cnt,
         const int64_t *__restrict__ pos, uint32_t *__restrict__ key,
         uint32_t *__restrict__ val, int *__restrict__ err)
{
    __shared__ int32_t sc[LM_CBLK];
    for (long long p0 = (long long)blockIdx.x * LM_TPB; p0 < P.n;
         p0 += (long long)gridDim.x * LM_TPB) {
        const int p = (int)(p0 + threadIdx.x);
        const bool live = p < P.n;
        const int own = live ? cell[p] : -1;
        float bnd = 0.f;
        if (live) {
            if (EMIT)
                bnd = gb[p];
            else
                gb[p] = bnd = lm_bound<M>(g, dC[p]);
        }
        int k = 0;
        long long o = 0, oend = 0;
        if (EMIT && live) {
            o = pos[p];
            oend = pos[p + 1];
            key[o] = 2u * (uint32_t)own;
            val[o] = (uint32_t)p;
        }
        for (int c0 = 0; c0 < m; c0 += LM_CBLK) {
            __syncthreads();
            if (threadIdx.x < LM_CBLK && c0 + (int)threadIdx.x < m)
                sc[threadIdx.x] = cid[c0 + threadIdx.x];
            __syncthreads();
            const int cn = min(LM_CBLK, m - c0);
            if (live)
                for (int j = 0; j < cn; ++j) {
                    const int c = c0 + j;
                    if (c == own)
                        continue;
                    if (lm_dist<M>(P, p, sc[j]) <= bnd) {
                        ++k;
                        if (EMIT) {
                            if (o + k < oend) {
                                key[o + k] = 2u * (uint32_t)c + 1u;
                                val[o + k] = (uint32_t)p;
                            } else {
                                atomicOr(err, 1);  // passes disagree (never)
                            }
                        }
                    }
                }
        }
        if (!EMIT && live)
            cnt[p] = 1 + k;
    }
}

// Cell of each augmented row (sorted keys: 2 cell + ghost bit), its input
// index, and the first row of every cell.
__global__ void k_aug_rows(const uint32_t *__restrict__ key,
                           const uint32_t *__restrict__ val, long long na, int m,
                           int32_t *__restrict__ acell, int32_t *__restrict__ aorig,
                           int32_t *__restrict__ aghost, int64_t *__restrict__ first)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < na;
         i += (long long)gridDim.x * blockDim.x) {
        const uint32_t k = key[i];
        const int c = (int)(k >> 1);
        acell[i] = c;
        aorig[i] = (int32_t)val[i];
        aghost[i] = (int32_t)(k & 1u);
        const int cp = i > 0 ? (int)(key[i - 1] >> 1) : -1;
        for (int q = cp + 1; q <= c; ++q)  // cells with no rows get the same start
            first[q] = i;
        if (i == na - 1)
            for (int q = c + 1; q <= m; ++q)
                first[q] = na;
    }
}

// Copy of whole input rows (rowb bytes each, a multiple of 4) in the
// augmented order.
__global__ void k_gather_bytes(const uint8_t *__restrict__ src,
                               const int32_t *__restrict__ idx, long long na,
                               int rowb, uint8_t *__restrict__ dst)
{
    const int w4 = rowb / 4;
    const long long tot = na * w4;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / w4;
        const int w = (int)(e % w4);
        reinterpret_cast<uint32_t *>(dst + r * rowb)[w] =
            reinterpret_cast<const uint32_t *>(src + (size_t)idx[r] * rowb)[w];
    }
}

// Home cell of every augmented row (the Voronoi cell of its input point).
__device__ __forceinline__ bool lm_keep(const int32_t *acell, const int32_t *aghost,
                                        const int32_t *home, int a, int b)
{
    const bool ga = aghost[a] != 0, gb = aghost[b] != 0;
    if (!ga && !gb)
        return true;
    if (ga && gb)
        return false;
    // one member, one ghost of the same cell: kept by the lower of the two
    // home cells, which is this cell exactly when the ghost's home is higher
    return ga ? home[a] > acell[a] : home[b] > acell[b];
}

// FILL = false: deg[orig(a)] += kept entries of augmented row a.
// FILL = true: kept entries written to the output rows through cur.
template <bool FILL>
__global__ void __launch_bounds__(LM_TPB)
k_keep(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
       const float *__restrict__ dist, long long na,
       const int32_t *__restrict__ acell, const int32_t *__restrict__ aorig,
       const int32_t *__restrict__ aghost, const int32_t *__restrict__ home,
       int32_t *__restrict__ deg, unsigned long long *__restrict__ cur,
       const int64_t *__restrict__ orp, int32_t *__restrict__ ocol,
       float *__restrict__ odist, int *__restrict__ err)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (long long a = (long long)blockIdx.x * wpb + threadIdx.x / WAVE; a < na;
         a += (long long)gridDim.x * wpb) {
        const int r = aorig[a];
        const int64_t b0 = rp[a], b1 = rp[a + 1];
        for (int64_t e0 = b0; e0 < b1; e0 += WAVE) {
            const int64_t e = e0 + lane;
            const bool k = e < b1 && lm_keep(acell, aghost, home, (int)a, col[e]);
            const uint64_t mk = __ballot(k);
            const int cnt = __popcll(mk);
            if (!cnt)
                continue;
            if (!FILL) {
                if (lane == 0)
                    atomicAdd(&deg[r], cnt);
            } else {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&cur[r], (unsigned long long)cnt);
                base = __shfl(base, 0, WAVE);
                if (k) {
                    const unsigned long long o =
                        base + __popcll(mk & ((1ull << lane) - 1ull));
                    if ((long long)o < orp[r + 1]) {
                        ocol[o] = aorig[col[e]];
                        odist[o] = dist[e];
                    } else {
                        atomicOr(err, 1);  // count and fill disagree (never)
                    }
                }
            }
        }
    }
}

__global__ void k_home(const int32_t *__restrict__ aorig, long long na,
                       const int32_t *__restrict__ cell, int32_t *__restrict__ home)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < na;
         i += (long long)gridDim.x * blockDim.x)
        home[i] = cell[aorig[i]];
}

__global__ void k_rows_init(const int64_t *__restrict__ rp, int n,
                            unsigned long long *__restrict__ cur)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x)
        cur[i] = (unsigned long long)rp[i];
}

__global__ void k_rows_check(const int64_t *__restrict__ rp, int n,
                             const unsigned long long *__restrict__ cur,
                             int *__restrict__ bad)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x)
        if (cur[i] != (unsigned long long)rp[i + 1])
            atomicOr(bad, 1);
}

uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// m distinct indices of [0, n): the first m entries of a seeded partial
// Fisher-Yates shuffle (the untouched tail of the permutation is implicit).
std::vector<int32_t> draw_centres(int64_t n, int m, uint64_t seed)
{
    std::vector<int32_t> out(m);
    std::unordered_map<int64_t, int64_t> moved;  // sparse permutation
    auto at = [&](int64_t i) {
        auto it = moved.find(i);
        return it == moved.end() ? i : it->second;
    };
    uint64_t s = seed;
    for (int k = 0; k < m; ++k) {
        const uint64_t span = (uint64_t)(n - k);
        const int64_t j = k + (int64_t)(splitmix64(s) % span);
        const int64_t vk = at(k), vj = at(j);
        moved[k] = vj;
        moved[j] = vk;
        out[k] = (int32_t)vj;
    }
    return out;
}

struct VG {
    const int32_t *cid;
    int m;
    GhostBound g;
    int32_t *cell;
    float *dC, *gb;
    int32_t *cnt;
    const int64_t *pos;
    uint32_t *key, *val;
    int *err;
};

template <int M>
void voronoi_ghosts(const Pts &P, const VG &a, bool emit, hipStream_t s)
{
    const dim3 grid(grid_cap(P.n, LM_TPB, 8192)), blk(LM_TPB);
    if (!emit) {
        FNN_LAUNCH((k_voronoi<M>), grid, blk, 0, s, P, a.cid, a.m, a.cell, a.dC);
        FNN_LAUNCH((k_ghosts<M, false>), grid, blk, 0, s, P, a.cid, a.m, a.g, a.cell,
                   a.dC, a.gb, a.cnt, a.pos, a.key, a.val, a.err);
    } else {
        FNN_LAUNCH((k_ghosts<M, true>), grid, blk, 0, s, P, a.cid, a.m, a.g, a.cell,
                   a.dC, a.gb, a.cnt, a.pos, a.key, a.val, a.err);
    }
}

void dispatch_vg(int metric, const Pts &P, const VG &a, bool emit, hipStream_t s)
{
    switch (metric) {
    case M_L2:
        voronoi_ghosts<M_L2>(P, a, emit, s);
        break;
    case M_ANG:
        voronoi_ghosts<M_ANG>(P, a, emit, s);
        break;
    case M_HAM:
        voronoi_ghosts<M_HAM>(P, a, emit, s);
        break;
    default:
        voronoi_ghosts<M_LEV>(P, a, emit, s);
        break;
    }
}

int bitlen_u32(uint32_t v)
{
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

}  // namespace

// Host driver.  `hdr` carries metric, n, dim and dp (no tree is built on
// it).  The per-cell forest and its query go through the public batch
// calls, so they take the caller's options and allocator.
void landmark_graph(fnn_tree *hdr, const void *points, double eps, int m,
                    uint64_t seed, const fnn_options *opt, fnn_csr *C,
                    fnn_stats &st, Scratch &S)
{
    hipStream_t s = S.stream();
    const int64_t n = hdr->n;
    m = (int)std::min<int64_t>(m, n);
    hipEvent_t ev[4];
    for (auto &e : ev)
        FNN_HIP(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < 4; ++i)
                (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    FNN_HIP(hipEventRecord(ev[0], s));

    // ---- centres, Voronoi cells, ghosts ------------------------------------
    Pts P = ingest_input(hdr, points, S);
    const std::vector<int32_t> ch = draw_centres(n, m, seed);
    int32_t *cid = S.get<int32_t>(m);
    FNN_HIP(hipMemcpyAsync(cid, ch.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
    GhostBound g;
    const int M = hdr->metric;
    if (M == M_HAM || M == M_LEV) {
        g.rel = 0.f;
        g.abs_ = 0.f;
        g.eps2 = (float)(2.0 * std::min(floor(eps), 1e9));
    } else {
        // rounding of every FP32 distance: the traversal's relative slack,
        // four times (the chain through an assigned point's centre uses
        // four distances)
        const double u = 1.0 / 16777216.0;
        const double rel = std::max(1e-4, 8.0 * (hdr->dp + 4) * u);
        g.rel = (float)(4.0 * rel);
        // absolute part: FP32 underflow of tiny squared differences (the
        // same (dp + 4) 1e-37 key term as the build's radii), or the angle's
        g.abs_ = M == M_ANG ? 4e-5f : (float)(4.0 * sqrt((hdr->dp + 4) * 1e-37));
        g.eps2 = (float)std::min(2.0 * eps, 1e30);
    }
    VG a{};
    a.cid = cid;
    a.m = m;
    a.g = g;
    a.cell = S.get<int32_t>(n);
    a.dC = S.get<float>(n);
    a.gb = S.get<float>(n);
    a.cnt = S.get<int32_t>(n);
    a.err = S.get<int>(1);
    fill(a.err, 0, 1, s);
    dispatch_vg(M, P, a, false, s);
    int64_t *pos = S.get<int64_t>(n + 1);
    scan_i32_to_i64(a.cnt, pos, n, S);
    const int64_t na = read_scalar(pos + n, s);
    if (na > (int64_t)INT32_MAX / 2 - 1)
        fail(FNN_EUNSUPPORTED, "landmark cells with their ghosts hold %lld rows "
             "(limit 2^30 - 1): use fewer cells", (long long)na);
    uint32_t *key = S.get<uint32_t>(na), *val = S.get<uint32_t>(na);
    a.pos = pos;
    a.key = key;
    a.val = val;
    dispatch_vg(M, P, a, true, s);
    int32_t *cell = a.cell;
    uint32_t *skey = S.get<uint32_t>(na), *sval = S.get<uint32_t>(na);
    radix_sort_pairs(key, val, skey, sval, na, bitlen_u32(2u * (uint32_t)m), S);
    int32_t *acell = S.get<int32_t>(na), *aorig = S.get<int32_t>(na),
            *aghost = S.get<int32_t>(na), *home = S.get<int32_t>(na);
    int64_t *first = S.get<int64_t>(m + 1);
    FNN_LAUNCH(k_aug_rows, dim3(grid_for(na, 256)), dim3(256), 0, s, skey, sval, na, m,
               acell, aorig, aghost, first);
    FNN_LAUNCH(k_home, dim3(grid_for(na, 256)), dim3(256), 0, s, aorig, na, cell, home);
    std::vector<int64_t> off(m + 1);
    FNN_HIP(hipMemcpyAsync(off.data(), first, sizeof(int64_t) * (m + 1),
                           hipMemcpyDeviceToHost, s));
    // augmented rows in the caller's layout
    const int rowb = M == M_L2 || M == M_ANG ? 4 * hdr->dim
                     : M == M_HAM          ? hdr->dim / 8
                                           : hdr->dim;
    const bool w4 = rowb % 4 == 0;
    uint8_t *aug = S.get<uint8_t>((size_t)na * rowb + 16);
    if (w4) {
        FNN_LAUNCH(k_gather_bytes, dim3(grid_cap(na * (rowb / 4), 256, 65536)), dim3(256),
                   0, s, (const uint8_t *)points, aorig, na, rowb, aug);
    } else {
        fail(FNN_EUNSUPPORTED, "landmark mode needs rows of a multiple of 4 bytes");
    }
    FNN_HIP(hipStreamSynchronize(s));  // off is read below
    if (read_scalar(a.err, s))
        fail(FNN_EINTERNAL, "landmark: ghost count and emission disagree");
    FNN_HIP(hipEventRecord(ev[1], s));

    // ---- per-cell forest and its self-join -----------------------------
    fnn_tree *T = nullptr;
    int rc = fnn_tree_build_batch(aug, off.data(), m, hdr->dim, (fnn_metric)M, opt, &T);
    if (rc != FNN_OK)
        fail(rc, "%s", fnn_last_error());
    struct TreeGuard {
        fnn_tree *t;
        ~TreeGuard() { fnn_free(t); }
    } tg{T};
    std::vector<double> ev_eps(m, eps);
    fnn_csr *A = nullptr;
    rc = fnn_eps_graph_batch(T, ev_eps.data(), m, opt, &A);
    if (rc != FNN_OK)
        fail(rc, "%s", fnn_last_error());
    struct CsrGuard {
        fnn_csr *c;
        ~CsrGuard() { fnn_free(c); }
    } cg{A};
    fnn_stats qs{};
    fnn_get_stats(A, &qs);
    fnn_stats bs{};
    fnn_get_stats(T, &bs);
    FNN_HIP(hipEventRecord(ev[2], s));

    // ---- keep each ordered pair once, rows back to input indices -------
    int32_t *deg = S.get<int32_t>(n);
    fill(deg, 0, (int64_t)n, s);
    const dim3 kg(grid_cap(na, 4, 16384));
    FNN_LAUNCH(k_keep<false>, kg, dim3(LM_TPB), 0, s, A->row_ptr, A->col, A->dist, na,
               acell, aorig, aghost, home, deg, (unsigned long long *)nullptr,
               (const int64_t *)nullptr, (int32_t *)nullptr, (float *)nullptr, a.err);
    C->n = n;
    C->row_ptr = (int64_t *)out_alloc(sizeof(int64_t) * ((size_t)n + 1));
    scan_i32_to_i64(deg, C->row_ptr, n, S);
    const int64_t nnz = read_scalar(C->row_ptr + n, s);
    C->nnz = nnz;
    C->col = (int32_t *)out_alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
    C->dist = (float *)out_alloc(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
    unsigned long long *cur = S.get<unsigned long long>(n);
    FNN_LAUNCH(k_rows_init, dim3(grid_for(n, 256)), dim3(256), 0, s, C->row_ptr, (int)n, cur);
    FNN_LAUNCH(k_keep<true>, kg, dim3(LM_TPB), 0, s, A->row_ptr, A->col, A->dist, na,
               acell, aorig, aghost, home, deg, cur, C->row_ptr, C->col, C->dist, a.err);
    int *bad = a.err;
    FNN_LAUNCH(k_rows_check, dim3(grid_for(n, 256)), dim3(256), 0, s, C->row_ptr, (int)n,
               cur, bad);
    sort_csr_rows(C->row_ptr, (int)n, C->col, C->dist, nnz, S, nullptr);
    FNN_HIP(hipEventRecord(ev[3], s));
    if (read_scalar(bad, s))
        fail(FNN_EINTERNAL, "landmark: kept-pair count and fill disagree");

    float t01 = 0.f, t12 = 0.f, t23 = 0.f;
    FNN_HIP(hipEventElapsedTime(&t01, ev[0], ev[1]));
    FNN_HIP(hipEventElapsedTime(&t12, ev[1], ev[2]));
    FNN_HIP(hipEventElapsedTime(&t23, ev[2], ev[3]));
    st = qs;
    st.n = n;
    st.edges = nnz;
    st.nodes = bs.nodes;
    st.rounds = bs.rounds;
    st.netsel_passes = bs.netsel_passes;
    st.build_dist_evals = bs.build_dist_evals + (int64_t)n * m * 2;
    st.build_ms = bs.build_ms;
    // landmark fields: cells, augmented rows, phase times
    st.landmark_cells = m;
    st.landmark_rows = na;
    st.landmark_partition_ms = t01;
    st.landmark_forest_ms = t12;
    st.landmark_merge_ms = t23;
    st.total_ms = t01 + t12 + t23;
}

}  // namespace fnn
