// C ABI entry points (include/fnn.h): argument checks, error codes,
// ownership.  No exception crosses this boundary.
#include <math.h>
#include <string.h>

#include <new>
#include <string>

#include <mutex>

#include "learn.h"

namespace fnn {
extern thread_local hipStream_t g_stream;
void set_alloc_hook(fnn_alloc_fn a, fnn_free_fn f, void *ctx);
void build_tree(fnn_tree *T, const void *points, Scratch &S);
fnn_tree *forest_pair(const fnn_tree *A, const fnn_tree *B, Scratch &S);
void eps_graph(const fnn_tree *T, const double *eps, const Options &opt,
               fnn_csr *C, fnn_stats &st, Scratch &S, float **tf, float **tt);
void landmark_graph(fnn_tree *hdr, const void *points, double eps, int m,
                    uint64_t seed, const fnn_options *opt, fnn_csr *C,
                    fnn_stats &st, Scratch &S);

// The installed cost model: one device copy per device.
static std::mutex g_model_mu;
static std::vector<float> g_model_host;
static float *g_model_dev[64] = {nullptr};
static uint64_t g_model_gen = 0, g_model_dev_gen[64] = {0};

const float *cost_model_device()
{
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (g_model_host.empty())
        return nullptr;
    int dev = 0;
    FNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        fail(FNN_EUNSUPPORTED, "device id %d", dev);
    if (!g_model_dev[dev])
        FNN_HIP(hipMalloc(&g_model_dev[dev], sizeof(float) * MLP_NPAR));
    if (g_model_dev_gen[dev] != g_model_gen) {
        FNN_HIP(hipMemcpy(g_model_dev[dev], g_model_host.data(),
                          sizeof(float) * MLP_NPAR, hipMemcpyHostToDevice));
        g_model_dev_gen[dev] = g_model_gen;
    }
    return g_model_dev[dev];
}

static thread_local std::string g_err;

static int set_err(int code, const std::string &m)
{
    g_err = m;
    return code;
}

int api_error(int code, const char *msg) { return set_err(code, msg); }

Options read_options(const fnn_options *o)
{
    Options r;
    if (!o)
        return r;
    if (o->struct_size < (int32_t)offsetof(fnn_options, reserved))
        fail(FNN_EINVAL, "fnn_options.struct_size is too small (%d)",
             (int)o->struct_size);
    if (o->zeta < 0 || o->pack < 0 || o->kmax < 0)
        fail(FNN_EINVAL, "negative option");
    if (o->zeta)
        r.zeta = o->zeta;
    if (o->pack)
        r.pack = o->pack;
    if (o->precision < 0 || o->precision > FNN_PREC_FP16)
        fail(FNN_EINVAL, "unknown precision %d", (int)o->precision);
    r.precision = o->precision;
    if (o->sched < 0 || o->sched > FNN_SCHED_LEARNED)
        fail(FNN_EINVAL, "unknown schedule %d", (int)o->sched);
    r.sched = o->sched;
    r.validate = o->validate ? 1 : 0;
    if (o->kmax)
        r.kmax = o->kmax > 256 ? 256 : o->kmax;
    r.trace = o->trace ? 1 : 0;
    if (o->slack_pct)
        r.slack_pct = o->slack_pct < -90 ? -90 : o->slack_pct;
    if (o->graph_passes < 0)
        fail(FNN_EINVAL, "negative graph_passes");
    if (o->graph_passes)
        r.graph_passes = o->graph_passes > 64 ? 64 : o->graph_passes;
    if (o->proj < -1 || o->proj > 128 || (o->proj > 0 && o->proj % 16))
        fail(FNN_EINVAL, "proj must be -1, 0 or a multiple of 16 up to 128 (got %d)",
             (int)o->proj);
    r.proj = o->proj;
    if (o->list_cap < 0)
        fail(FNN_EINVAL, "negative list_cap");
    r.list_cap = o->list_cap;
    r.lpt = o->lpt ? 1 : 0;
    return r;
}

// Launches of one call, from the thread's counters.
struct LaunchDelta {
    LaunchCount c0 = launch_count();
    void into(fnn_stats &st) const
    {
        const LaunchCount &c = launch_count();
        st.launches = c.kernels - c0.kernels;
        st.graph_launches = c.graphs - c0.graphs;
        st.graph_kernels = c.graph_kernels - c0.graph_kernels;
    }
};

struct CsrBox {
    fnn_csr pub;
    fnn_stats stats;
    float *trace_feat;
    float *trace_targ;
};

// Rows [r0, r0 + m) of a CSR: row_ptr shifted to start at 0.
__global__ void k_row_slice(const int64_t *__restrict__ rp, int64_t r0, int64_t m,
                            int64_t *__restrict__ out)
{
    const int64_t b = rp[r0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = rp[r0 + i] - b;
}

static void free_box(CsrBox *B)
{
    out_free(B->pub.row_ptr);
    out_free(B->pub.col);
    out_free(B->pub.dist);
    out_free(B->trace_feat);
    out_free(B->trace_targ);
    B->pub.kind = 0;
    delete B;
}

}  // namespace fnn

using namespace fnn;

extern "C" {

int fnn_version(void) { return 100; }

const char *fnn_last_error(void) { return g_err.c_str(); }

int fnn_set_stream(void *stream)
{
    g_stream = (hipStream_t)stream;
    return FNN_OK;
}

int fnn_set_allocator(fnn_alloc_fn alloc, fnn_free_fn free_, void *ctx)
{
    if ((alloc == nullptr) != (free_ == nullptr))
        return set_err(FNN_EINVAL, "allocator and free must both be set or both NULL");
    set_alloc_hook(alloc, free_, ctx);
    return FNN_OK;
}

// Row stride of the device copy (floats, words or bytes) under the
// per-metric dimension rules.
static int row_stride(fnn_metric metric, int32_t dim)
{
    switch (metric) {
    case FNN_L2:
    case FNN_ANGULAR:
        if (dim > 65536)
            fail(FNN_EUNSUPPORTED, "dim > 65536");
        return (dim + 3) / 4 * 4;
    case FNN_HAMMING:
        if (dim % 64)
            fail(FNN_EINVAL, "Hamming dim (bits) must be a multiple of 64");
        if (dim / 64 > 16)
            fail(FNN_EUNSUPPORTED, "Hamming codes longer than 1024 bits");
        return dim / 64;
    default:
        if (dim > 64 * MAX_LEV_WORDS)
            fail(FNN_EUNSUPPORTED, "Levenshtein stride > %d", 64 * MAX_LEV_WORDS);
        return dim;
    }
}

static int tree_build_any(const void *points, int64_t n, const int64_t *offsets,
                          int32_t nclouds, int32_t dim, fnn_metric metric,
                          const fnn_options *opt, fnn_tree **out)
{
    if (!out)
        return set_err(FNN_EINVAL, "out is NULL");
    *out = nullptr;
    fnn_tree *T = nullptr;
    try {
        if (!points)
            fail(FNN_EINVAL, "points is NULL");
        if (n < 1 || n > (int64_t)INT32_MAX / 2 - 1)
            fail(FNN_EINVAL, "n must be in [1, 2^30 - 1] (got %lld)", (long long)n);
        if (metric < FNN_L2 || metric > FNN_LEVENSHTEIN)
            fail(FNN_EINVAL, "unknown metric %d", (int)metric);
        if (dim < 1)
            fail(FNN_EINVAL, "dim must be >= 1");
        Options o = read_options(opt);
        if (o.zeta < 1)
            fail(FNN_EINVAL, "zeta must be >= 1");
        // Strings: unrelated strings sit at similar edit distances, so the
        // tree is shallow and sibling leaf blocks lie far apart; a pack
        // that merges them has the radius of its parent and prunes nothing
        // (C4: 3.8e9 pair evaluations with packs of 64 points, 2.4e6 with
        // one leaf block per pack).  The default there is one block.
        if (metric == FNN_LEVENSHTEIN && !(opt && opt->pack))
            o.pack = 1;
        T = new fnn_tree();
        T->metric = metric;
        T->n = n;
        T->dim = dim;
        T->opt = o;
        T->ncloud_in = nclouds;
        if (offsets) {
            // compact the non-empty clouds
            for (int32_t c = 0; c < nclouds; ++c) {
                if (offsets[c + 1] < offsets[c])
                    fail(FNN_EINVAL, "offsets must be non-decreasing");
                if (offsets[c + 1] > offsets[c]) {
                    T->cloud_off_h.push_back(offsets[c]);
                    T->cloud_src.push_back(c);
                }
            }
            T->cloud_off_h.push_back(n);
        } else {
            T->cloud_off_h = {0, n};
            T->cloud_src = {0};
        }
        T->ncloud = (int)T->cloud_src.size();
        T->dp = row_stride(metric, dim);
        LaunchDelta ld;
        {
            Scratch S(current_stream());
            build_tree(T, points, S);
        }
        ld.into(T->stats);
        *out = T;
        return FNN_OK;
    } catch (const Error &e) {
        delete T;
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        delete T;
        return set_err(FNN_ENOMEM, "host allocation failed");
    } catch (...) {
        delete T;
        return set_err(FNN_EINTERNAL, "unexpected exception");
    }
}

int fnn_tree_build_ex(const void *points, int64_t n, int32_t dim,
                      fnn_metric metric, const fnn_options *opt, fnn_tree **out)
{
    return tree_build_any(points, n, nullptr, 1, dim, metric, opt, out);
}

int fnn_tree_build_batch(const void *points, const int64_t *offsets,
                         int32_t nclouds, int32_t dim, fnn_metric metric,
                         const fnn_options *opt, fnn_tree **out)
{
    if (out)
        *out = nullptr;
    if (!offsets)
        return set_err(FNN_EINVAL, "offsets is NULL");
    if (nclouds < 1)
        return set_err(FNN_EINVAL, "nclouds must be >= 1");
    if (offsets[0] != 0)
        return set_err(FNN_EINVAL, "offsets[0] must be 0");
    return tree_build_any(points, offsets[nclouds], offsets, nclouds, dim, metric,
                          opt, out);
}

int fnn_tree_build(const void *points, int64_t n, int32_t dim,
                   fnn_metric metric, fnn_tree **out)
{
    return fnn_tree_build_ex(points, n, dim, metric, nullptr, out);
}

static int eps_graph_any(const fnn_tree *tree, const double *eps, int32_t neps,
                         bool per_cloud, const fnn_options *opt, fnn_csr **out)
{
    if (!out)
        return set_err(FNN_EINVAL, "out is NULL");
    *out = nullptr;
    CsrBox *B = nullptr;
    try {
        if (!tree || tree->kind != KIND_TREE)
            fail(FNN_EINVAL, "not a tree handle");
        if (!eps)
            fail(FNN_EINVAL, "eps is NULL");
        if (per_cloud && neps != tree->ncloud_in)
            fail(FNN_EINVAL, "nclouds (%d) differs from the tree's (%d)", (int)neps,
                 (int)tree->ncloud_in);
        // thresholds of the non-empty clouds, in the tree's compact order
        std::vector<double> ev(tree->ncloud);
        for (int c = 0; c < tree->ncloud; ++c) {
            const double e = per_cloud ? eps[tree->cloud_src[c]] : eps[0];
            if (!(e > 0.0) || !isfinite(e))
                fail(FNN_EINVAL, "eps must be finite and > 0");
            ev[c] = e;
        }
        Options o = read_options(opt);
        B = new CsrBox();
        memset(&B->pub, 0, sizeof B->pub);
        memset(&B->stats, 0, sizeof B->stats);
        B->trace_feat = B->trace_targ = nullptr;
        B->pub.kind = KIND_CSR;
        LaunchDelta ld;
        {
            Scratch S(current_stream());
            eps_graph(tree, ev.data(), o, &B->pub, B->stats, S, &B->trace_feat,
                      &B->trace_targ);
        }
        ld.into(B->stats);
        *out = &B->pub;
        return FNN_OK;
    } catch (const Error &e) {
        if (B)
            free_box(B);
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        if (B)
            free_box(B);
        return set_err(FNN_ENOMEM, "host allocation failed");
    } catch (...) {
        if (B)
            free_box(B);
        return set_err(FNN_EINTERNAL, "unexpected exception");
    }
}

int fnn_eps_query(const fnn_tree *tree, const void *queries, int64_t nq, double eps,
                  const fnn_options *opt, fnn_csr **out)
{
    if (!out)
        return set_err(FNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tree || tree->kind != KIND_TREE)
        return set_err(FNN_EINVAL, "not a tree handle");
    if (tree->ncloud != 1 || tree->ncloud_in != 1)
        return set_err(FNN_EUNSUPPORTED, "bichromatic queries need a single-cloud tree");
    if (!(eps > 0.0) || !isfinite(eps))
        return set_err(FNN_EINVAL, "eps must be finite and > 0");
    // the query points get a cover tree of their own (same options)
    fnn_tree *TQ = nullptr;
    const int rc = tree_build_any(queries, nq, nullptr, 1, tree->dim,
                                  (fnn_metric)tree->metric, opt, &TQ);
    if (rc != FNN_OK)
        return rc;
    fnn_tree *F = nullptr;
    CsrBox *full = nullptr, *B = nullptr;
    try {
        Options o = read_options(opt);
        Scratch S(current_stream());
        hipStream_t s = S.stream();
        F = forest_pair(tree, TQ, S);
        full = new CsrBox();
        memset(&full->pub, 0, sizeof full->pub);
        memset(&full->stats, 0, sizeof full->stats);
        full->trace_feat = full->trace_targ = nullptr;
        full->pub.kind = KIND_CSR;
        const double ev[2] = {eps, eps};
        float *tf = nullptr, *tt = nullptr;
        eps_graph(F, ev, o, &full->pub, full->stats, S, &tf, &tt);
        // the query rows: input rows nA .. nA + nq - 1 of the pair forest,
        // whose columns are the tree's points (only pairs across clouds)
        const int64_t nA = tree->n;
        int64_t se[2];
        FNN_HIP(hipMemcpyAsync(se, full->pub.row_ptr + nA, sizeof(int64_t),
                               hipMemcpyDeviceToHost, s));
        FNN_HIP(hipMemcpyAsync(se + 1, full->pub.row_ptr + nA + nq, sizeof(int64_t),
                               hipMemcpyDeviceToHost, s));
        FNN_HIP(hipStreamSynchronize(s));
        const int64_t nnz = se[1] - se[0];
        B = new CsrBox();
        memset(&B->pub, 0, sizeof B->pub);
        B->stats = full->stats;
        B->stats.n = nq;
        B->stats.build_ms += TQ->stats.build_ms;
        B->stats.build_dist_evals += TQ->stats.build_dist_evals;
        B->stats.edges = nnz;
        B->trace_feat = B->trace_targ = nullptr;
        B->pub.kind = KIND_CSR;
        B->pub.n = nq;
        B->pub.nnz = nnz;
        B->pub.row_ptr = (int64_t *)out_alloc(sizeof(int64_t) * (size_t)(nq + 1));
        B->pub.col = (int32_t *)out_alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
        B->pub.dist = (float *)out_alloc(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
        FNN_LAUNCH(k_row_slice, dim3(grid_cap(nq + 1, 256, 4096)), dim3(256), 0, s,
                   full->pub.row_ptr, nA, nq, B->pub.row_ptr);
        if (nnz > 0) {
            FNN_HIP(hipMemcpyAsync(B->pub.col, full->pub.col + se[0], sizeof(int32_t) * nnz,
                                   hipMemcpyDeviceToDevice, s));
            FNN_HIP(hipMemcpyAsync(B->pub.dist, full->pub.dist + se[0], sizeof(float) * nnz,
                                   hipMemcpyDeviceToDevice, s));
        }
        FNN_HIP(hipStreamSynchronize(s));
        free_box(full);
        delete F;
        delete TQ;
        *out = &B->pub;
        return FNN_OK;
    } catch (const Error &e) {
        if (full)
            free_box(full);
        if (B)
            free_box(B);
        delete F;
        delete TQ;
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        if (full)
            free_box(full);
        if (B)
            free_box(B);
        delete F;
        delete TQ;
        return set_err(FNN_ENOMEM, "host allocation failed");
    } catch (...) {
        if (full)
            free_box(full);
        if (B)
            free_box(B);
        delete F;
        delete TQ;
        return set_err(FNN_EINTERNAL, "unexpected exception");
    }
}

int fnn_landmark_eps_graph(const void *points, int64_t n, int32_t dim,
                           fnn_metric metric, double eps, int32_t ncells,
                           uint64_t seed, const fnn_options *opt, fnn_csr **out)
{
    if (!out)
        return set_err(FNN_EINVAL, "out is NULL");
    *out = nullptr;
    CsrBox *B = nullptr;
    try {
        if (!points)
            fail(FNN_EINVAL, "points is NULL");
        if (n < 1 || n > (int64_t)INT32_MAX / 2 - 1)
            fail(FNN_EINVAL, "n must be in [1, 2^30 - 1] (got %lld)", (long long)n);
        if (metric < FNN_L2 || metric > FNN_LEVENSHTEIN)
            fail(FNN_EINVAL, "unknown metric %d", (int)metric);
        if (dim < 1)
            fail(FNN_EINVAL, "dim must be >= 1");
        if (!(eps > 0.0) || !isfinite(eps))
            fail(FNN_EINVAL, "eps must be finite and > 0");
        if (ncells < 1)
            fail(FNN_EINVAL, "ncells must be >= 1");
        Options o = read_options(opt);
        if (o.trace)
            fail(FNN_EUNSUPPORTED, "traces are not available in landmark mode");
        fnn_tree hdr;  // shape only: no tree is built on it
        hdr.metric = metric;
        hdr.n = n;
        hdr.dim = dim;
        hdr.dp = row_stride(metric, dim);
        hdr.opt = o;
        B = new CsrBox();
        memset(&B->pub, 0, sizeof B->pub);
        memset(&B->stats, 0, sizeof B->stats);
        B->trace_feat = B->trace_targ = nullptr;
        B->pub.kind = KIND_CSR;
        LaunchDelta ld;
        {
            Scratch S(current_stream());
            landmark_graph(&hdr, points, eps, ncells, seed, opt, &B->pub, B->stats, S);
        }
        ld.into(B->stats);
        *out = &B->pub;
        return FNN_OK;
    } catch (const Error &e) {
        if (B)
            free_box(B);
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        if (B)
            free_box(B);
        return set_err(FNN_ENOMEM, "host allocation failed");
    } catch (...) {
        if (B)
            free_box(B);
        return set_err(FNN_EINTERNAL, "unexpected exception");
    }
}

int fnn_eps_graph_ex(const fnn_tree *tree, double eps, const fnn_options *opt,
                     fnn_csr **out)
{
    return eps_graph_any(tree, &eps, 1, false, opt, out);
}

int fnn_eps_graph(const fnn_tree *tree, double eps, fnn_csr **out)
{
    return fnn_eps_graph_ex(tree, eps, nullptr, out);
}

int fnn_eps_graph_batch(const fnn_tree *tree, const double *eps, int32_t nclouds,
                        const fnn_options *opt, fnn_csr **out)
{
    return eps_graph_any(tree, eps, nclouds, true, opt, out);
}

void fnn_free(void *handle)
{
    if (!handle)
        return;
    uint32_t kind = *(const uint32_t *)handle;
    if (kind == KIND_TREE) {
        fnn_tree *T = (fnn_tree *)handle;
        T->kind = 0;
        delete T;
    } else if (kind == KIND_CSR) {
        free_box((CsrBox *)handle);  // pub is the first member
    }
}

int fnn_get_stats(const void *handle, fnn_stats *out)
{
    if (!handle || !out)
        return set_err(FNN_EINVAL, "NULL argument");
    uint32_t kind = *(const uint32_t *)handle;
    if (kind == KIND_TREE)
        *out = ((const fnn_tree *)handle)->stats;
    else if (kind == KIND_CSR)
        *out = ((const CsrBox *)handle)->stats;
    else
        return set_err(FNN_EINVAL, "not a library handle");
    return FNN_OK;
}

int fnn_tree_info(const fnn_tree *tree, int64_t *n, int64_t *nodes)
{
    if (!tree || tree->kind != KIND_TREE)
        return set_err(FNN_EINVAL, "not a tree handle");
    if (n)
        *n = tree->n;
    if (nodes)
        *nodes = tree->nnodes;
    return FNN_OK;
}

int fnn_tree_export(const fnn_tree *T, int32_t *order, int32_t *center,
                    float *radius, int32_t *level, int32_t *child_begin,
                    int32_t *child_count, int32_t *pt_begin, int32_t *pt_end)
{
    if (!T || T->kind != KIND_TREE)
        return set_err(FNN_EINVAL, "not a tree handle");
    try {
        hipStream_t s = current_stream();
        const size_t nb = sizeof(int32_t) * (size_t)T->nnodes;
        struct {
            void *dst;
            const void *src;
            size_t bytes;
        } cp[] = {{order, T->perm, sizeof(int32_t) * (size_t)T->n},
                  {center, T->center, nb},
                  {radius, T->radius, sizeof(float) * (size_t)T->nnodes},
                  {level, T->level, nb},
                  {child_begin, T->child_begin, nb},
                  {child_count, T->child_count, nb},
                  {pt_begin, T->pt_begin, nb},
                  {pt_end, T->pt_end, nb}};
        for (auto &c : cp)
            if (c.dst)
                FNN_HIP(hipMemcpyAsync(c.dst, c.src, c.bytes,
                                       hipMemcpyDeviceToHost, s));
        FNN_HIP(hipStreamSynchronize(s));
        return FNN_OK;
    } catch (const Error &e) {
        return set_err(e.code, e.msg);
    }
}

int fnn_set_cost_model(const float *params, int64_t nparams)
{
    if (!params || nparams != MLP_NPAR)
        return set_err(FNN_EINVAL, "cost model needs 5378 parameters");
    for (int64_t i = 0; i < nparams; ++i)
        if (!isfinite(params[i]))
            return set_err(FNN_EINVAL, "cost model parameter is not finite");
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_model_host.assign(params, params + nparams);
    ++g_model_gen;
    return FNN_OK;
}

int fnn_get_trace(const fnn_csr *csr, const float **features,
                  const float **targets, int64_t *n)
{
    if (!csr || csr->kind != KIND_CSR)
        return set_err(FNN_EINVAL, "not a CSR handle");
    const CsrBox *B = (const CsrBox *)csr;
    if (!B->trace_feat || !B->trace_targ)
        return set_err(FNN_EINVAL, "query was not run with options.trace = 1");
    if (features)
        *features = B->trace_feat;
    if (targets)
        *targets = B->trace_targ;
    if (n)
        *n = csr->n;
    return FNN_OK;
}

int fnn_mlp_forward(const float *params, const float *X, int64_t n, float *Y)
{
    if (!params || (n > 0 && (!X || !Y)) || n < 0)
        return set_err(FNN_EINVAL, "bad argument");
    try {
        hipStream_t s = current_stream();
        mlp_forward(params, X, n, Y, s);
        FNN_HIP(hipStreamSynchronize(s));
        return FNN_OK;
    } catch (const Error &e) {
        return set_err(e.code, e.msg);
    }
}

int fnn_mlp_loss_grad(const float *params, const float *X, const float *T,
                      int64_t n, float *grad, double *loss)
{
    if (!params || !grad || n < 0 || (n > 0 && (!X || !T)))
        return set_err(FNN_EINVAL, "bad argument");
    try {
        Scratch S(current_stream());
        const double l = mlp_loss_grad(params, X, T, n, grad, S);
        if (loss)
            *loss = l;
        return FNN_OK;
    } catch (const Error &e) {
        return set_err(e.code, e.msg);
    }
}

int fnn_mlp_loss_grad_noalloc(const float *params, const float *X, const float *T,
                              int64_t n, float *grad, double *loss)
{
    if (!params || !grad || !loss || n < 0 || (n > 0 && (!X || !T)))
        return set_err(FNN_EINVAL, "bad argument");
    if (n > FNN_NOALLOC_MAX_SAMPLES)
        return set_err(FNN_EINVAL, "fnn_mlp_loss_grad_noalloc: n = " + std::to_string(n) +
                                       " exceeds FNN_NOALLOC_MAX_SAMPLES");
    try {
        mlp_loss_grad_noalloc(params, X, T, n, grad, loss, current_stream());
        return FNN_OK;
    } catch (const Error &e) {
        return set_err(e.code, e.msg);
    }
}

int fnn_mlp_train(float *params, const float *X, const float *T, int64_t n,
                  int32_t epochs, int32_t batch, float lr, uint64_t seed,
                  double *epoch_loss)
{
    if (!params || n < 0 || (n > 0 && (!X || !T)) || epochs < 0 || batch < 0 ||
        !(lr > 0.f))
        return set_err(FNN_EINVAL, "bad argument");
    if (n > (int64_t)UINT32_MAX)
        return set_err(FNN_EUNSUPPORTED, "too many samples");
    try {
        Scratch S(current_stream());
        mlp_train(params, X, T, n, epochs, batch, lr, seed, epoch_loss, S);
        return FNN_OK;
    } catch (const Error &e) {
        return set_err(e.code, e.msg);
    }
}

}  // extern "C"
