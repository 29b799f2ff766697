// Learned cost model: per-point features from the cover tree, a 16-64-64-2
// perceptron (SiLU) with hand-written forward, backward and Adam kernels,
// and inference.  It predicts, for every point, log1p of the number of
// block pairs its query pack takes part in ("visits") and log1p of its
// neighbour count.  The predictions only size CSR rows and order work; no
// edge decision depends on them.
//
// Parameter layout (row-major, one contiguous float buffer):
//   W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [2][64], b3 [2].
// Loss: L = 1/(2B) * sum_b sum_o (y_bo - t_bo)^2.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "learn.h"

namespace fnn {

constexpr int OW1 = 0, OB1 = OW1 + MLP_H * MLP_F, OW2 = OB1 + MLP_H,
              OB2 = OW2 + MLP_H * MLP_H, OW3 = OB2 + MLP_H,
              OB3 = OW3 + MLP_O * MLP_H;
static_assert(OB3 + MLP_O == MLP_NPAR, "parameter layout");

__device__ __forceinline__ float silu(float z) { return z / (1.f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.f / (1.f + expf(-z));
    return s * (1.f + z * (1.f - s));
}

// ------------------------------------------------------------- features --

__global__ void k_parent(const int32_t *__restrict__ cbeg,
                         const int32_t *__restrict__ ccnt, int nn,
                         int32_t *__restrict__ parent)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
         v += gridDim.x * blockDim.x) {
        if (v == 0)
            parent[0] = -1;
        for (int c = 0; c < ccnt[v]; ++c)
            parent[cbeg[v] + c] = v;
    }
}

__global__ void k_depth(const int32_t *__restrict__ parent, int nn,
                        int32_t *__restrict__ depth)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
         v += gridDim.x * blockDim.x) {
        int d = 0, u = v;
        while (parent[u] >= 0 && d < 4096) {
            u = parent[u];
            ++d;
        }
        depth[v] = d;
    }
}

// owner[pos] = id of the range [pb, pe) holding pos, for ranges that tile
// the positions (leaf blocks, or packs).
__global__ void k_owner(const int32_t *__restrict__ pb, const int32_t *__restrict__ pe,
                        const int32_t *__restrict__ ccnt, int first, int count,
                        int only_leaves, int32_t *__restrict__ owner)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    for (int k = blockIdx.x * wpb + threadIdx.x / WAVE; k < count;
         k += gridDim.x * wpb) {
        const int v = first + k;
        if (only_leaves && ccnt[v] != 0)
            continue;
        for (int p = pb[v] + lane; p < pe[v]; p += WAVE)
            owner[p] = v;
    }
}

// Per-point features (16, scale-free; eps is the point's own cloud's):
//  0 log2(1 + pack size) / 6        1 depth of the point's leaf / 8
//  2 log2(r_pack / eps)             3 d(p, pack centre) / eps (<= 16)
//  4 log2(r / eps) of the parent    5 the same for the grandparent
//  6 d(p, centre) / r of the parent 7 the same for the grandparent (<= 2)
//  8, 9, 10 log1p(pack members within eps, 2 eps, eps / 2) / 6
// 11 mean distance to the pack members / eps (each <= 16)
// 12 log2(1 + size of the smallest ancestor with r >= eps) / 20
// 13 log2(1 + the parent's child count) / 8
// 14 log2(1 + the parent's size) / 20
// 15 distance to the nearest other pack member / eps (<= 4)
// No feature is constant over a whole tree (such a value would let the
// network recognise the training set instead of the point's surroundings).
template <int M>
__global__ void k_features(Pts P, FeatArgs A, int local_done, float *__restrict__ feat)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P.n;
         p += gridDim.x * blockDim.x) {
        float f[MLP_F];
        const int pk = A.pack_of[p];
        const int v0 = A.leaf_of[p];
        const int cl = A.pcl ? A.pcl[p] : -1;
        const float eps = cl >= 0 ? A.ct[cl].feps : A.eps;
        const float tiny = 1.0f / 1048576.0f;
        const int qb = A.q_pb[pk], qe = A.q_pe[pk];
        f[0] = log2f(1.f + (float)(qe - qb)) / 6.f;
        f[1] = (float)A.depth[v0] / 8.f;
        f[2] = log2f(A.q_rad[pk] / eps + tiny);
        f[3] = fminf(key_to_dist<M>(key32<M>(P, p, A.q_cpos[pk])) / eps, 16.f);
        int v = v0;
        for (int k = 0; k < 2; ++k) {
            if (A.parent[v] >= 0)
                v = A.parent[v];
            const float r = A.radius[v];
            f[4 + k] = log2f(r / eps + tiny);
            const float d = key_to_dist<M>(key32<M>(P, p, A.center_pos[v]));
            f[6 + k] = fminf(d / (r + 1e-30f), 2.f);
        }
        // the point's own pack as a local sample of its neighbourhood: the
        // whole pack when it holds at most 64 points (then the lanes of a
        // pack read the same member rows in step), else 64 members around p
        // (a duplicate leaf can be larger)
        // packs of at most 64 points get these from k_pack_local when it runs
        const bool mine = !local_done || qe - qb > 64;
        const int lo = qe - qb <= 64 ? qb : max(qb, min(p - 32, qe - 64));
        const int hi = mine ? min(qe, lo + 64) : lo;
        int c1 = 0, c2 = 0, ch = 0;
        float sum = 0.f, dmin = 4.f * eps;
        for (int q = lo; q < hi; ++q) {
            if (q == p)
                continue;
            const float d = key_to_dist<M>(key32<M>(P, p, q));
            c1 += d <= eps;
            c2 += d <= 2.f * eps;
            ch += d <= 0.5f * eps;
            sum += fminf(d, 16.f * eps);
            dmin = fminf(dmin, d);
        }
        const int others = max(hi - lo - 1, 1);
        f[8] = log1pf((float)c1) / 6.f;
        f[9] = log1pf((float)c2) / 6.f;
        f[10] = log1pf((float)ch) / 6.f;
        f[11] = sum / ((float)others * eps);
        int u = v0;
        while (A.radius[u] < eps && A.parent[u] >= 0)
            u = A.parent[u];
        f[12] = log2f(1.f + (float)(A.pe[u] - A.pb[u])) / 20.f;
        const int v1 = A.parent[v0] >= 0 ? A.parent[v0] : v0;
        f[13] = log2f(1.f + (float)A.ccnt[v1]) / 8.f;
        f[14] = log2f(1.f + (float)(A.pe[v1] - A.pb[v1])) / 20.f;
        f[15] = dmin / eps;
#pragma unroll
        for (int k = 0; k < MLP_F; ++k)
            if (mine || (k != 8 && k != 9 && k != 10 && k != 11 && k != 15))
                feat[(size_t)p * MLP_F + k] = f[k];
    }
}

// Features 8-11 and 15 (the pack as a local sample) for vector rows of at
// most LOC_MAXD floats: one work-group per pack of at most 64 points, its
// rows staged in LDS (odd row stride: lanes reading one coordinate of
// different rows hit different banks); thread t takes point t / 4 against
// every fourth member, and the four partial results meet by shuffles.
constexpr int LOC_MAXD = 128;
template <int M>
__global__ void __launch_bounds__(256)
k_pack_local(Pts P, FeatArgs A, float *__restrict__ feat)
{
    __shared__ float rows[64 * (LOC_MAXD + 1)];
    const float *X = M == M_L2 ? P.x : P.xn;
    const int dp = P.dp, ld = dp + 1, t = threadIdx.x;
    const int npk = A.npacks;
    for (int k = blockIdx.x; k < npk; k += gridDim.x) {
        const int pk = A.first_pack + k;
        const int qb = A.q_pb[pk], qe = A.q_pe[pk], m = qe - qb;
        __syncthreads();  // rows of the previous pack are no longer read
        if (m > 64)
            continue;     // k_features handles large packs
        for (int e = t; e < m * dp; e += blockDim.x)
            rows[(e / dp) * ld + e % dp] = X[(size_t)qb * dp + e];
        __syncthreads();
        const int i = t >> 2, j0 = t & 3;
        const int p = qb + i;
        const int cl = A.pcl ? A.pcl[min(p, qe - 1)] : -1;
        const float eps = cl >= 0 ? A.ct[cl].feps : A.eps;
        int c1 = 0, c2 = 0, ch = 0;
        float sum = 0.f, dmin = 4.f * eps;
        if (i < m)
            for (int j = j0; j < m; j += 4) {
                if (j == i)
                    continue;
                const float *a = rows + i * ld, *b = rows + j * ld;
                float acc = 0.f;
                for (int c = 0; c < dp; ++c) {
                    const float d = a[c] - b[c];
                    acc = fmaf(d, d, acc);
                }
                const float d = key_to_dist<M>(acc);
                c1 += d <= eps;
                c2 += d <= 2.f * eps;
                ch += d <= 0.5f * eps;
                sum += fminf(d, 16.f * eps);
                dmin = fminf(dmin, d);
            }
        // the four threads of a point are adjacent lanes
#pragma unroll
        for (int o = 1; o < 4; o <<= 1) {
            c1 += __shfl_xor(c1, o, WAVE);
            c2 += __shfl_xor(c2, o, WAVE);
            ch += __shfl_xor(ch, o, WAVE);
            sum += __shfl_xor(sum, o, WAVE);
            dmin = fminf(dmin, __shfl_xor(dmin, o, WAVE));
        }
        if (i < m && j0 == 0) {
            float *f = feat + (size_t)p * MLP_F;
            f[8] = log1pf((float)c1) / 6.f;
            f[9] = log1pf((float)c2) / 6.f;
            f[10] = log1pf((float)ch) / 6.f;
            f[11] = sum / ((float)max(m - 1, 1) * eps);
            f[15] = dmin / eps;
        }
    }
}

// ------------------------------------------------------------------ MLP --

// y = W3 silu(W2 silu(W1 x + b1) + b2) + b3, one sample per thread.
__global__ void __launch_bounds__(256)
k_mlp_fwd(const float *__restrict__ th, const float *__restrict__ X, long long n,
          float *__restrict__ Y)
{
    __shared__ float w[MLP_NPAR];
    for (int i = threadIdx.x; i < MLP_NPAR; i += blockDim.x)
        w[i] = th[i];
    __syncthreads();
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (long long)gridDim.x * blockDim.x) {
        float x[MLP_F], h1[MLP_H];
#pragma unroll
        for (int k = 0; k < MLP_F; ++k)
            x[k] = X[s * MLP_F + k];
#pragma unroll
        for (int j = 0; j < MLP_H; ++j) {
            float z = w[OB1 + j];
#pragma unroll
            for (int k = 0; k < MLP_F; ++k)
                z = fmaf(w[OW1 + j * MLP_F + k], x[k], z);
            h1[j] = silu(z);
        }
        float y0 = w[OB3], y1 = w[OB3 + 1];
        for (int j = 0; j < MLP_H; ++j) {
            float z = w[OB2 + j];
#pragma unroll
            for (int k = 0; k < MLP_H; ++k)
                z = fmaf(w[OW2 + j * MLP_H + k], h1[k], z);
            const float h2 = silu(z);
            y0 = fmaf(w[OW3 + j], h2, y0);
            y1 = fmaf(w[OW3 + MLP_H + j], h2, y1);
        }
        Y[s * 2] = y0;
        Y[s * 2 + 1] = y1;
    }
}

// Gradient of the loss over the samples idx[0..B) (or 0..B if idx is
// NULL).  A block takes 32 samples at a time: each thread runs one sample
// forward and backward into LDS, then the block reduces the outer products
// parameter-major.  PART = false: sums are added to grad and *loss with
// atomics.  PART = true: work-group b owns row b of grad ([gridDim][NPAR])
// and loss[b], written without atomics (thread t always owns the same
// parameters), for a fixed-order reduction afterwards.
constexpr int GS = 32;
template <bool PART>
__global__ void __launch_bounds__(256)
k_mlp_grad(const float *__restrict__ th, const float *__restrict__ X,
           const float *__restrict__ T, const int32_t *__restrict__ idx,
           long long B, float invB, float *__restrict__ grad,
           double *__restrict__ loss)
{
    if (PART) {
        grad += (size_t)blockIdx.x * MLP_NPAR;
        for (int p = threadIdx.x; p < MLP_NPAR; p += blockDim.x)
            grad[p] = 0.f;
    }
    __shared__ float w[MLP_NPAR];
    __shared__ float sx[GS][MLP_F], sh1[GS][MLP_H], sh2[GS][MLP_H],
        sg1[GS][MLP_H], sg2[GS][MLP_H], sgy[GS][MLP_O];
    for (int i = threadIdx.x; i < MLP_NPAR; i += blockDim.x)
        w[i] = th[i];
    __syncthreads();
    double lsum = 0.0;
    for (long long b0 = (long long)blockIdx.x * GS; b0 < B;
         b0 += (long long)gridDim.x * GS) {
        const int t = threadIdx.x;
        const int ns = (int)std::min<long long>(GS, B - b0);
        if (t < GS) {
            if (t < ns) {
                const long long s = idx ? idx[b0 + t] : b0 + t;
                float x[MLP_F];
#pragma unroll
                for (int k = 0; k < MLP_F; ++k)
                    x[k] = sx[t][k] = X[s * MLP_F + k];
                // layer 1: z1 kept in sg1 until the backward pass
                for (int j = 0; j < MLP_H; ++j) {
                    float z = w[OB1 + j];
#pragma unroll
                    for (int k = 0; k < MLP_F; ++k)
                        z = fmaf(w[OW1 + j * MLP_F + k], x[k], z);
                    sg1[t][j] = z;
                    sh1[t][j] = silu(z);
                }
                // layer 2: z2 kept in sg2
                float y0 = w[OB3], y1 = w[OB3 + 1];
                for (int j = 0; j < MLP_H; ++j) {
                    float z = w[OB2 + j];
                    for (int k = 0; k < MLP_H; ++k)
                        z = fmaf(w[OW2 + j * MLP_H + k], sh1[t][k], z);
                    sg2[t][j] = z;
                    const float h2 = sh2[t][j] = silu(z);
                    y0 = fmaf(w[OW3 + j], h2, y0);
                    y1 = fmaf(w[OW3 + MLP_H + j], h2, y1);
                }
                const float e0 = y0 - T[s * 2], e1 = y1 - T[s * 2 + 1];
                lsum += 0.5 * ((double)e0 * e0 + (double)e1 * e1);
                const float gy0 = e0 * invB, gy1 = e1 * invB;
                sgy[t][0] = gy0;
                sgy[t][1] = gy1;
                for (int j = 0; j < MLP_H; ++j) {
                    const float gh2 = w[OW3 + j] * gy0 + w[OW3 + MLP_H + j] * gy1;
                    sg2[t][j] = gh2 * dsilu(sg2[t][j]);
                }
                for (int k = 0; k < MLP_H; ++k) {
                    float gh1 = 0.f;
                    for (int j = 0; j < MLP_H; ++j)
                        gh1 = fmaf(w[OW2 + j * MLP_H + k], sg2[t][j], gh1);
                    sg1[t][k] = gh1 * dsilu(sg1[t][k]);
                }
            } else {
                for (int k = 0; k < MLP_F; ++k)
                    sx[t][k] = 0.f;
                for (int j = 0; j < MLP_H; ++j)
                    sh1[t][j] = sh2[t][j] = sg1[t][j] = sg2[t][j] = 0.f;
                sgy[t][0] = sgy[t][1] = 0.f;
            }
        }
        __syncthreads();
        for (int p = threadIdx.x; p < MLP_NPAR; p += blockDim.x) {
            float g = 0.f;
            if (p < OB1) {
                const int j = p / MLP_F, k = p % MLP_F;
                for (int s = 0; s < ns; ++s)
                    g = fmaf(sg1[s][j], sx[s][k], g);
            } else if (p < OW2) {
                const int j = p - OB1;
                for (int s = 0; s < ns; ++s)
                    g += sg1[s][j];
            } else if (p < OB2) {
                const int j = (p - OW2) / MLP_H, k = (p - OW2) % MLP_H;
                for (int s = 0; s < ns; ++s)
                    g = fmaf(sg2[s][j], sh1[s][k], g);
            } else if (p < OW3) {
                const int j = p - OB2;
                for (int s = 0; s < ns; ++s)
                    g += sg2[s][j];
            } else if (p < OB3) {
                const int o = (p - OW3) / MLP_H, k = (p - OW3) % MLP_H;
                for (int s = 0; s < ns; ++s)
                    g = fmaf(sgy[s][o], sh2[s][k], g);
            } else {
                const int o = p - OB3;
                for (int s = 0; s < ns; ++s)
                    g += sgy[s][o];
            }
            if (PART)
                grad[p] += g;
            else if (g != 0.f)
                atomicAdd(&grad[p], g);
        }
        __syncthreads();
    }
    lsum = wave_sum(lsum);
    if (PART) {
        __shared__ double wl[256 / WAVE];
        if ((threadIdx.x & (WAVE - 1)) == 0)
            wl[threadIdx.x / WAVE] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < (int)(blockDim.x / WAVE); ++w)
                t += wl[w];
            loss[blockIdx.x] = t;
        }
    } else if ((threadIdx.x & (WAVE - 1)) == 0 && lsum != 0.0) {
        atomicAdd(loss, lsum);
    }
}

// Fixed-order sum of the per-work-group partials: grad[p] = sum over g of
// part[g][p]; *loss = (sum over g of ploss[g]) / n.
__global__ void k_mlp_grad_reduce(const float *__restrict__ part,
                                  const double *__restrict__ ploss, int groups,
                                  long long n, float *__restrict__ grad,
                                  double *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPAR) {
        float g = 0.f;
        for (int k = 0; k < groups; ++k)
            g += part[(size_t)k * MLP_NPAR + p];
        grad[p] = g;
    }
    if (p == 0) {
        double t = 0.0;
        for (int k = 0; k < groups; ++k)
            t += ploss[k];
        *loss = n > 0 ? t / (double)n : 0.0;
    }
}

// Adam (Kingma & Ba), bias-corrected; step counts from 1.
__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, int n,
                       float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        th[i] -= lr * mh / (sqrtf(vh) + eps);
    }
}

// SplitMix64 (Steele, Lea, Flood 2014) keys for a seeded shuffle.
__global__ void k_shuffle_keys(long long n, unsigned long long seed,
                               uint32_t *__restrict__ key, uint32_t *__restrict__ val)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        key[i] = (uint32_t)(z >> 32);
        val[i] = (uint32_t)i;
    }
}

// ------------------------------------------------------------ host side --

void mlp_forward(const float *theta, const float *X, long long n, float *Y,
                 hipStream_t s)
{
    if (n <= 0)
        return;
    FNN_LAUNCH(k_mlp_fwd, dim3(grid_for(n, 256)), dim3(256), 0, s, theta, X, n, Y);
}

double mlp_loss_grad(const float *theta, const float *X, const float *T,
                     long long n, float *grad, Scratch &S)
{
    hipStream_t s = S.stream();
    double *loss = S.get<double>(1);
    fill(loss, 0.0, 1, s);
    fill(grad, 0.f, MLP_NPAR, s);
    if (n > 0)
        FNN_LAUNCH(k_mlp_grad<false>, dim3(grid_for(n, GS)), dim3(256), 0, s, theta,
                   X, T, (const int32_t *)nullptr, n, 1.0f / (float)n, grad, loss);
    return read_scalar(loss, s) / (double)std::max<long long>(n, 1);
}

void mlp_train(float *theta, const float *X, const float *T, long long n,
               int epochs, int batch, float lr, unsigned long long seed,
               double *epoch_loss, Scratch &S)
{
    hipStream_t s = S.stream();
    if (n <= 0 || epochs <= 0)
        return;
    if (batch <= 0)
        batch = 4096;
    float *g = S.get<float>(MLP_NPAR), *m = S.get<float>(MLP_NPAR),
          *v = S.get<float>(MLP_NPAR);
    fill(m, 0.f, MLP_NPAR, s);
    fill(v, 0.f, MLP_NPAR, s);
    double *loss = S.get<double>(1);
    uint32_t *k1 = S.get<uint32_t>(n), *v1 = S.get<uint32_t>(n);
    uint32_t *k2 = S.get<uint32_t>(n), *perm = S.get<uint32_t>(n);
    const float b1 = 0.9f, b2 = 0.999f, ae = 1e-8f;
    long long step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        FNN_LAUNCH(k_shuffle_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                   seed + 0x1234567ull * (unsigned long long)(ep + 1), k1, v1);
        radix_sort_pairs(k1, v1, k2, perm, n, 32, S);
        fill(loss, 0.0, 1, s);
        for (long long b0 = 0; b0 < n; b0 += batch) {
            const long long B = std::min<long long>(batch, n - b0);
            fill(g, 0.f, MLP_NPAR, s);
            FNN_LAUNCH(k_mlp_grad<false>, dim3(grid_for(B, GS)), dim3(256), 0, s,
                       theta, X, T, (const int32_t *)(perm + b0), B, 1.0f / (float)B,
                       g, loss);
            ++step;
            const float c1 = 1.f - powf(b1, (float)step);
            const float c2 = 1.f - powf(b2, (float)step);
            FNN_LAUNCH(k_adam, dim3(grid_for(MLP_NPAR, 256)), dim3(256), 0, s,
                       theta, g, m, v, MLP_NPAR, lr, b1, b2, ae, c1, c2);
        }
        if (epoch_loss)
            epoch_loss[ep] = read_scalar(loss, s) / (double)n;
    }
    FNN_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------- allocation-free gradient --
//
// fnn_mlp_loss_grad_noalloc keeps its partial sums in a fixed device array
// instead of scratch memory from the pool: NA_GROUPS rows of per-work-group
// partial gradients, then NA_GROUPS partial losses (doubles).  Host code
// never passes `scratch` itself to a kernel (in host code the name is a
// stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr int NA_GROUPS = 256;
constexpr size_t NA_GRAD_BYTES = sizeof(float) * (size_t)NA_GROUPS * MLP_NPAR;
constexpr size_t NA_BYTES = NA_GRAD_BYTES + sizeof(double) * NA_GROUPS;
static_assert(NA_GRAD_BYTES % alignof(double) == 0, "loss partials alignment");
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

static std::mutex g_na_mu;
static void *g_na_ptr[64] = {nullptr};

static unsigned char *noalloc_scratch()
{
    int dev = 0;
    FNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        fail(FNN_EUNSUPPORTED, "device id %d", dev);
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(FNN_EHIP, "hipGetSymbolAddress(scratch) failed: %s",
                 hipGetErrorString(e));
        g_na_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_na_ptr[dev]);
}

size_t mlp_noalloc_scratch_bytes() { return NA_BYTES; }

void mlp_loss_grad_noalloc(const float *theta, const float *X, const float *T,
                           long long n, float *grad, double *loss, hipStream_t s)
{
    unsigned char *base = noalloc_scratch();
    float *part = reinterpret_cast<float *>(base);
    double *ploss = reinterpret_cast<double *>(base + NA_GRAD_BYTES);
    // every work-group clears and fills its own row, so no clear is needed
    // before the launch; the reduction reads exactly `groups` rows
    const long long want = cdiv(std::max<long long>(n, 1), GS);
    const int groups = (int)std::min<long long>(want, NA_GROUPS);
    if (groups < 1 || groups > NA_GROUPS)
        fail(FNN_EINTERNAL, "gradient work-groups out of range");
    FNN_LAUNCH(k_mlp_grad<true>, dim3(groups), dim3(256), 0, s, theta, X, T,
               (const int32_t *)nullptr, n, n > 0 ? 1.0f / (float)n : 0.f, part,
               ploss);
    FNN_LAUNCH(k_mlp_grad_reduce, dim3(grid_for(MLP_NPAR, 256)), dim3(256), 0, s,
               part, ploss, groups, n, grad, loss);
}

void tree_aux(fnn_tree *T, Scratch &S)
{
    hipStream_t s = S.stream();
    const int nn = (int)T->nnodes, n = (int)T->n;
    if (T->parent)
        return;
    T->parent = (int32_t *)T->own(sizeof(int32_t) * nn);
    T->depth_v = (int32_t *)T->own(sizeof(int32_t) * nn);
    T->leaf_of = (int32_t *)T->own(sizeof(int32_t) * n);
    T->pack_of = (int32_t *)T->own(sizeof(int32_t) * n);
    FNN_LAUNCH(k_parent, dim3(grid_for(nn, 256)), dim3(256), 0, s, T->child_begin,
               T->child_count, nn, T->parent);
    if (T->ncloud > 1)  // cloud roots are roots: the virtual vertex 0 is no parent
        fill(T->parent + 1, -1, T->ncloud, s);
    FNN_LAUNCH(k_depth, dim3(grid_for(nn, 256)), dim3(256), 0, s, T->parent, nn,
               T->depth_v);
    FNN_LAUNCH(k_owner, dim3(grid_for(nn, 4)), dim3(256), 0, s, T->pt_begin,
               T->pt_end, T->child_count, 0, nn, 1, T->leaf_of);
    FNN_LAUNCH(k_owner, dim3(grid_for(T->npacks, 4)), dim3(256), 0, s,
               T->q_pt_begin, T->q_pt_end, T->q_kcnt, (int)T->nnodes,
               (int)T->npacks, 0, T->pack_of);
}

void compute_features(const fnn_tree *T, const Pts &P, float eps,
                      const CloudThr *ct, float *feat, hipStream_t s)
{
    FeatArgs A;
    A.pack_of = T->pack_of;
    A.leaf_of = T->leaf_of;
    A.parent = T->parent;
    A.depth = T->depth_v;
    A.center_pos = T->center_pos;
    A.radius = T->radius;
    A.pb = T->pt_begin;
    A.pe = T->pt_end;
    A.ccnt = T->child_count;
    A.q_cpos = T->q_center_pos;
    A.q_rad = T->q_radius;
    A.q_pb = T->q_pt_begin;
    A.q_pe = T->q_pt_end;
    A.eps = eps;
    A.ct = ct;
    A.pcl = ct ? T->pcl : nullptr;
    A.first_pack = (int)T->nnodes;
    A.npacks = (int)T->npacks;
    const dim3 g(grid_for(T->n, 256));
    const bool vec = T->metric == M_L2 || T->metric == M_ANG;
    // vector rows of at most 128 floats: the pack sample from LDS; larger
    // packs (duplicates) are still taken by k_features, which then writes
    // every feature of their points
    const int local = vec && T->dp <= LOC_MAXD;
    switch (T->metric) {
    case M_L2:
        FNN_LAUNCH((k_features<M_L2>), g, dim3(256), 0, s, P, A, local, feat);
        break;
    case M_ANG:
        FNN_LAUNCH((k_features<M_ANG>), g, dim3(256), 0, s, P, A, local, feat);
        break;
    case M_HAM:
        FNN_LAUNCH((k_features<M_HAM>), g, dim3(256), 0, s, P, A, 0, feat);
        break;
    default:
        FNN_LAUNCH((k_features<M_LEV>), g, dim3(256), 0, s, P, A, 0, feat);
        break;
    }
    if (local) {
        const dim3 gp(grid_cap(T->npacks, 1, 16384));
        if (T->metric == M_L2)
            FNN_LAUNCH((k_pack_local<M_L2>), gp, dim3(256), 0, s, P, A, feat);
        else
            FNN_LAUNCH((k_pack_local<M_ANG>), gp, dim3(256), 0, s, P, A, feat);
    }
}

}  // namespace fnn
