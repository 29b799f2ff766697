// Autotuner: times the whole path (build + query) under candidate options on
// the caller's input and returns the fastest.  Every option it varies changes
// only the schedule or the filter arithmetic, never the graph, so any
// candidate's result is the exact graph.
//
// Search: coordinate descent from the defaults (or the caller's base
// options): filter precision, then CSR schedule, then leaf size zeta, the
// net-selection width kmax, the tile block (pack) size, the passes per
// net-selection graph replay (queue granularity) and, for the learned
// schedule, the LPT work order; each coordinate keeps its best value before
// the next is tried.  Answers are cached in-process per input shape (metric,
// dim, log2 n, log2 clouds, base options); a cached answer is returned
// without timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tree.h"

namespace fnn {
const float *cost_model_device();
int api_error(int code, const char *msg);
}

using namespace fnn;

namespace {

using Key = std::tuple<int, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<Key, fnn_tune_result> g_tune_cache;

int ilog2(int64_t v)
{
    int l = 0;
    while (v > 1) {
        v >>= 1;
        ++l;
    }
    return l;
}

struct Runner {
    const void *points;
    const int64_t *offsets;
    int32_t nclouds, dim;
    fnn_metric metric;
    const double *eps;
    int64_t n;
    int reps;
    int ncand = 0;

    // median wall time of build + query in ms; < 0 when the options fail
    double time(const fnn_options &o)
    {
        std::vector<double> t;
        for (int r = 0; r < reps; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            fnn_tree *T = nullptr;
            fnn_csr *C = nullptr;
            int rc = offsets ? fnn_tree_build_batch(points, offsets, nclouds, dim,
                                                    metric, &o, &T)
                             : fnn_tree_build_ex(points, n, dim, metric, &o, &T);
            if (rc == FNN_OK)
                rc = offsets ? fnn_eps_graph_batch(T, eps, nclouds, &o, &C)
                             : fnn_eps_graph_ex(T, eps[0], &o, &C);
            const auto t1 = std::chrono::steady_clock::now();
            fnn_free(C);
            fnn_free(T);
            if (rc != FNN_OK)
                return -1.0;
            t.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        ++ncand;
        std::sort(t.begin(), t.end());
        return t[t.size() / 2];
    }
};

}  // namespace

extern "C" int fnn_autotune(const void *points, const int64_t *offsets,
                            int32_t nclouds, int32_t dim, fnn_metric metric,
                            const double *eps, const fnn_options *base,
                            int32_t reps, fnn_tune_result *out)
{
    if (!out || !points || !eps || !offsets)
        return api_error(FNN_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    if (nclouds < 1 || reps < 0)
        return api_error(FNN_EINVAL, "nclouds must be >= 1 and reps >= 0");
    if (offsets[0] != 0)
        return api_error(FNN_EINVAL, "offsets[0] must be 0");
    const int64_t n = offsets[nclouds];
    fnn_options o0;
    memset(&o0, 0, sizeof o0);
    if (base) {
        if (base->struct_size < (int32_t)offsetof(fnn_options, reserved))
            return api_error(FNN_EINVAL, "fnn_options.struct_size is too small");
        memcpy(&o0, base, std::min<size_t>(sizeof o0, (size_t)base->struct_size));
    }
    o0.struct_size = sizeof o0;
    o0.trace = 0;
    o0.validate = 0;
    {
        const Options d;  // explicit defaults, so no candidate repeats one
        if (!o0.zeta)
            o0.zeta = d.zeta;
        if (!o0.kmax)
            o0.kmax = d.kmax;
        if (!o0.pack && metric != FNN_LEVENSHTEIN)
            o0.pack = d.pack;
        if (!o0.graph_passes)
            o0.graph_passes = d.graph_passes;
    }

    const Key key{(int)metric, (int)dim, ilog2(n), ilog2(nclouds),
                  o0.zeta * 4096 + o0.pack, o0.kmax * 256 + o0.graph_passes,
                  ((o0.precision * 8 + o0.sched) * 256 + (o0.proj + 1)) * 2 + (o0.lpt ? 1 : 0)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            out->cached = 1;
            return FNN_OK;
        }
    }

    Runner R{points, nclouds > 1 ? offsets : nullptr, nclouds, dim, metric, eps,
             n, reps < 1 ? 1 : reps};
    // with a single cloud the plain calls run (the batch of one is the same)
    if (nclouds == 1)
        R.offsets = nullptr;

    fnn_options best = o0;
    R.reps = 1;
    (void)R.time(best);  // untimed: first-use costs (code load, pool growth)
    R.reps = reps < 1 ? 1 : reps;
    R.ncand = 0;
    double best_ms = R.time(best);
    if (best_ms < 0)
        return api_error(FNN_EINVAL, "the base options fail on this input");
    const double default_ms = best_ms;

    auto try_values = [&](int32_t fnn_options::*field, const std::vector<int> &vals) {
        for (int v : vals) {
            if (best.*field == v)
                continue;
            fnn_options c = best;
            c.*field = v;
            const double ms = R.time(c);
            if (ms >= 0 && ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    };
    const bool vec = metric == FNN_L2 || metric == FNN_ANGULAR;
    if (vec && dim <= 128)
        try_values(&fnn_options::precision, {FNN_PREC_FP32, FNN_PREC_FP16});
    else if (metric == FNN_HAMMING && dim <= 256)
        try_values(&fnn_options::precision, {FNN_PREC_FP32, FNN_PREC_I8});
    bool have_model = false;
    try {
        have_model = cost_model_device() != nullptr;
    } catch (const Error &e) {
        return api_error(e.code, e.msg.c_str());
    }
    if (have_model)
        try_values(&fnn_options::sched, {FNN_SCHED_TWO_PASS, FNN_SCHED_LEARNED});
    try_values(&fnn_options::zeta, {32, 64, 128});
    try_values(&fnn_options::kmax, {32, 64, 128});
    // tile shape of the leaf work: points per query / leaf block (strings
    // keep one leaf block per pack)
    if (metric != FNN_LEVENSHTEIN)
        try_values(&fnn_options::pack, {32, 64});
    // queue granularity of the build: net-selection passes per graph replay
    // between host checks of the device queue
    try_values(&fnn_options::graph_passes, {2, 4, 8});
    if (best.sched == FNN_SCHED_LEARNED)
        try_values(&fnn_options::lpt, {0, 1});

    out->best = best;
    out->best_ms = best_ms;
    out->base_ms = default_ms;
    out->ncand = R.ncand;
    out->cached = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = *out;
    }
    return FNN_OK;
}

extern "C" void fnn_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}
