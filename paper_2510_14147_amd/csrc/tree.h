// The device-resident cover tree behind the opaque fnn_tree handle, and the
// host-side threshold helpers shared by the build and the query.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/fnn.h"
#include "common.h"
#include "runtime.h"

namespace fnn {

constexpr uint32_t KIND_TREE = 0x54524545u;  // "TREE"
constexpr uint32_t KIND_CSR = 0x43535221u;   // "CSR!"

struct Options {
    int zeta = 64;
    int pack = 64;
    int precision = FNN_PREC_FP32;
    int sched = FNN_SCHED_TWO_PASS;
    int validate = 0;
    int kmax = 64;
    int trace = 0;
    int slack_pct = 30;
    int graph_passes = 4;
    int proj = 0;
    long long list_cap = 0;  // initial survivor / edge list entries (0: automatic)
    int lpt = 0;             // learned schedule: LPT order of the tile pass
};

Options read_options(const fnn_options *o);

}  // namespace fnn

struct fnn_tree {
    uint32_t kind = fnn::KIND_TREE;
    int metric = 0;
    int64_t n = 0;
    int dim = 0;
    int dp = 0;     // row stride: floats (L2/ANG), words (HAM), bytes (LEV)
    int W = 0;      // Levenshtein words per pattern
    int sigma = 0;  // Levenshtein alphabet
    fnn::Options opt;

    // point data in tree order
    float *x = nullptr;
    float *xn = nullptr;
    uint64_t *h = nullptr;
    uint8_t *s = nullptr;
    int32_t *len = nullptr;
    uint64_t *peq = nullptr;
    int32_t *perm = nullptr;  // tree position -> input index

    // cover tree (Algorithms 1-2), vertices in creation (level) order
    int64_t nnodes = 0;
    int32_t *center = nullptr;      // input index
    int32_t *center_pos = nullptr;  // tree position of the centre
    float *radius = nullptr;        // upper bound of d(centre, x) in subtree
    int32_t *level = nullptr;
    int32_t *child_begin = nullptr;
    int32_t *child_count = nullptr;
    int32_t *pt_begin = nullptr;
    int32_t *pt_end = nullptr;

    // query tree: internal vertices keep their ids, packs of consecutive
    // sibling leaf blocks get ids nnodes .. nnodes + npacks - 1
    int64_t npacks = 0;
    int64_t nq = 0;
    int32_t qroot = 0;
    int32_t *q_center_pos = nullptr;  // [nq]
    float *q_radius = nullptr;
    int32_t *q_pt_begin = nullptr;
    int32_t *q_pt_end = nullptr;
    int32_t *q_kbeg = nullptr;   // children list offsets (packs: count 0)
    int32_t *q_kcnt = nullptr;
    int32_t *q_kids = nullptr;

    // auxiliary arrays of the learned schedule (built on first use)
    int32_t *parent = nullptr;   // [nnodes], -1 at the root
    int32_t *depth_v = nullptr;  // [nnodes]
    int32_t *leaf_of = nullptr;  // [n] leaf block of each tree position
    int32_t *pack_of = nullptr;  // [n] query-tree pack of each position

    // batch of independent clouds (forest): vertex 0 is a virtual root whose
    // children 1..ncloud are the cloud roots; cloud c holds the input rows
    // and tree positions [cloud_off_h[c], cloud_off_h[c + 1]).  With one
    // cloud the tree is an ordinary cover tree and pcl is null.
    int ncloud = 1;
    std::vector<int64_t> cloud_off_h;  // compact (non-empty) clouds
    std::vector<int32_t> cloud_src;    // caller's index of each compact cloud
    int32_t ncloud_in = 1;             // clouds as the caller numbered them
    int32_t *pcl = nullptr;            // [n] cloud of each tree position
    // two-tree forest of a bichromatic query: the query-tree roots of the
    // two clouds, whose pair seeds the traversal (-1 otherwise)
    int32_t cross_a = -1, cross_b = -1;

    int depth = 0;
    fnn_stats stats{};
    std::vector<void *> owned;

    void *own(size_t bytes)
    {
        void *p = fnn::out_alloc(bytes);
        owned.push_back(p);
        return p;
    }
    // One allocation carved into N arrays of the given sizes (each starting
    // 256-byte aligned): one call of the caller's allocator instead of N.
    template <size_t N>
    void own_many(const size_t (&bytes)[N], void *(&out)[N])
    {
        size_t off[N], tot = 0;
        for (size_t i = 0; i < N; ++i) {
            off[i] = tot;
            tot += (bytes[i] + 255) / 256 * 256;
        }
        char *p = static_cast<char *>(own(tot > 0 ? tot : 256));
        for (size_t i = 0; i < N; ++i)
            out[i] = p + off[i];
    }
    ~fnn_tree()
    {
        for (void *p : owned)
            fnn::out_free(p);
    }
};

namespace fnn {

// Host-side threshold tables (implemented in build.hip).
Thr make_thr_eps(int metric, int dp, double eps);
void make_level_table(int metric, int dp, LevelTab *tab);

// Radius (distance, rounded up) from an FP32 key maximum; device and host.
__host__ __device__ inline float radius_from_key(int metric, int dp, float kmax)
{
    if (kmax <= 0.f)
        return 0.f;
    const double u = 1.0 / 16777216.0;  // 2^-24
    double r;
    if (metric == M_L2) {
        double b = 2.0 * (dp + 4) * u;
        r = sqrt((double)kmax * (1.0 + b) + (dp + 4) * 1e-37);
        r = r * (1.0 + 4.0 * u);
    } else if (metric == M_ANG) {
        double c2 = (double)kmax;
        double dl = c2 * 2.0 * (3.0 * dp + 24) * u + 16.0 * u * sqrt(c2) + 1e-9;
        double ch = sqrt(c2 + dl) * 0.5;
        if (ch > 1.0)
            ch = 1.0;
        r = 2.0 * asin(ch) * (1.0 + 1e-5) + 1e-6;
    } else {
        return kmax;
    }
    float f = (float)r;
    if ((double)f < r)
        f = nextafterf(f, __builtin_huge_valf());
    return f;
}

// Smallest integer l with 2^l >= r (r > 0).
__host__ __device__ inline int level_of(float r)
{
    int e;
    float m = frexpf(r, &e);
    return m == 0.5f ? e - 1 : e;
}

}  // namespace fnn
