// Runtime helpers and device primitives: error state, stream binding,
// scratch pool, exclusive scan, stable radix sort.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "../../include/fnn.h"
#include "common.h"
#include "runtime.h"

namespace fnn {

// ---------------------------------------------------------------- errors --

void fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, std::string(buf)};
}

// --------------------------------------------------------------- streams --

thread_local hipStream_t g_stream = nullptr;

hipStream_t current_stream() { return g_stream; }

// One non-blocking stream per device on which launch sequences are recorded
// into graphs (recording never runs them; the caller's stream, which may be
// the null stream, runs the instantiated graph).  Default priority.
static std::mutex g_cap_mu;
static hipStream_t g_cap_stream[64] = {nullptr};

hipStream_t capture_stream()
{
    int dev = 0;
    FNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        fail(-4, "device id %d", dev);
    std::lock_guard<std::mutex> lk(g_cap_mu);
    if (!g_cap_stream[dev])
        FNN_HIP(hipStreamCreateWithFlags(&g_cap_stream[dev], hipStreamNonBlocking));
    return g_cap_stream[dev];
}

int num_cus()
{
    static std::atomic<int> cus[64];
    int dev = 0;
    FNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64)
        fail(-4, "device id %d", dev);
    int c = cus[dev].load();
    if (c == 0) {
        FNN_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
        c = std::max(1, c);
        cus[dev].store(c);
    }
    return c;
}

LaunchCount &launch_count()
{
    static thread_local LaunchCount c;
    return c;
}

GraphRun::~GraphRun()
{
    if (capturing)
        launch_count().capturing = false;
    if (capturing) {  // an error left the recording open: close and drop it
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g)
            (void)hipGraphDestroy(g);
    }
    if (exec)
        (void)hipGraphExecDestroy(exec);
    if (graph)
        (void)hipGraphDestroy(graph);
}

void GraphRun::begin()
{
    cs = capture_stream();
    FNN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    capturing = true;
    launch_count().capturing = true;
}

void GraphRun::end()
{
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    capturing = false;
    launch_count().capturing = false;
    if (e != hipSuccess || !g)
        fail(-3, "graph capture failed: %s", hipGetErrorString(e));
    graph = g;
    size_t nn = 0;
    FNN_HIP(hipGraphGetNodes(graph, nullptr, &nn));
    nkernels = (long long)nn;
    FNN_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
}

void GraphRun::launch(hipStream_t s)
{
    FNN_HIP(hipGraphLaunch(exec, s));
    LaunchCount &c = launch_count();
    ++c.graphs;
    c.graph_kernels += nkernels;
}

// --------------------------------------------------------------- scratch --
//
// Scratch memory is bump-allocated from large chunks.  When the caller has
// set an allocator (fnn_set_allocator), every chunk is taken from it and
// handed back when the call's scope ends, after its stream has drained, so
// all device memory of a call goes through the caller (a caching allocator
// then keeps the chunks).  Otherwise a call's chunks come from a per-device
// cache of idle hipMalloc'd chunks (best fit, so a repeated call reuses the
// same chunks) and go back to it; a steady stream of calls then makes no
// device allocation at all.  Idle chunks beyond a cap are freed.

// The caller's allocator (defined with out_alloc below): true and *p set
// when one is installed (fails with FNN_ENOMEM if it returns NULL).
static bool hook_alloc(size_t bytes, void **p);
static void hook_free(void *p);

namespace {
struct Chunk {
    char *base;
    size_t cap;
};
std::mutex g_chunk_mu;
std::vector<Chunk> g_idle[64];
size_t g_idle_bytes[64] = {0};
constexpr size_t CHUNK = (size_t)256 << 20;         // usual chunk size
constexpr size_t IDLE_CAP = (size_t)32 << 30;       // idle bytes kept per device
constexpr size_t ALIGN = 256;
}  // namespace

Scratch::Scratch(hipStream_t s) : s_(s)
{
    FNN_HIP(hipGetDevice(&dev_));
    if (dev_ < 0 || dev_ >= 64)
        fail(FNN_EUNSUPPORTED, "device id %d", dev_);
}

void *Scratch::raw(size_t bytes)
{
    bytes = (std::max<size_t>(bytes, 16) + ALIGN - 1) / ALIGN * ALIGN;
    if (!chunks_.empty() && used_ + bytes <= chunks_.back().second) {
        void *p = static_cast<char *>(chunks_.back().first) + used_;
        used_ += bytes;
        return p;
    }
    const size_t want = std::max(bytes, CHUNK);
    void *base = nullptr;
    size_t cap = 0;
    if (hook_alloc(want, &base)) {
        chunks_.emplace_back(base, want);
        hooked_.push_back(true);
        used_ = bytes;
        return base;
    }
    {
        std::lock_guard<std::mutex> lk(g_chunk_mu);
        auto &idle = g_idle[dev_];
        int best = -1;
        for (int i = 0; i < (int)idle.size(); ++i)
            if (idle[i].cap >= bytes && (best < 0 || idle[i].cap < idle[best].cap))
                best = i;
        if (best >= 0) {
            base = idle[best].base;
            cap = idle[best].cap;
            g_idle_bytes[dev_] -= cap;
            idle[best] = idle.back();
            idle.pop_back();
        }
    }
    if (!base) {
        hipError_t e = hipMalloc(&base, want);
        if (e != hipSuccess || !base) {
            (void)hipGetLastError();
            fail(FNN_ENOMEM, "device scratch allocation of %zu bytes failed: %s",
                 want, hipGetErrorString(e));
        }
        cap = want;
    }
    chunks_.emplace_back(base, cap);
    hooked_.push_back(false);
    used_ = bytes;
    return base;
}

void Scratch::release(void *)
{
    // bump allocation: the space returns with the scope's chunks
}

Scratch::~Scratch()
{
    if (chunks_.empty())
        return;
    // the chunks may be reused by any stream once this one has drained
    (void)hipStreamSynchronize(s_);
    for (size_t i = 0; i < chunks_.size(); ++i)
        if (hooked_[i])
            hook_free(chunks_[i].first);
    std::lock_guard<std::mutex> lk(g_chunk_mu);
    for (size_t i = 0; i < chunks_.size(); ++i) {
        if (hooked_[i])
            continue;
        const auto &c = chunks_[i];
        g_idle[dev_].push_back(Chunk{static_cast<char *>(c.first), c.second});
        g_idle_bytes[dev_] += c.second;
    }
    auto &idle = g_idle[dev_];
    while (g_idle_bytes[dev_] > IDLE_CAP && !idle.empty()) {
        int big = 0;
        for (int i = 1; i < (int)idle.size(); ++i)
            if (idle[i].cap > idle[big].cap)
                big = i;
        (void)hipFree(idle[big].base);
        g_idle_bytes[dev_] -= idle[big].cap;
        idle[big] = idle.back();
        idle.pop_back();
    }
}

// ------------------------------------------------------ output allocator --

struct AllocHook {
    fnn_alloc_fn alloc = nullptr;
    fnn_free_fn free_ = nullptr;
    void *ctx = nullptr;
};
static AllocHook g_hook;
static std::mutex g_hook_mu;

void set_alloc_hook(fnn_alloc_fn a, fnn_free_fn f, void *ctx)
{
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_hook.alloc = a;
    g_hook.free_ = f;
    g_hook.ctx = ctx;
}

static bool hook_alloc(size_t bytes, void **p)
{
    AllocHook h;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        h = g_hook;
    }
    if (!h.alloc)
        return false;
    *p = h.alloc(bytes, h.ctx);
    if (!*p)
        fail(FNN_ENOMEM, "user allocator returned NULL for %zu bytes of scratch", bytes);
    return true;
}

static void hook_free(void *p)
{
    AllocHook h;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        h = g_hook;
    }
    if (h.free_)
        h.free_(p, h.ctx);
}

void *out_alloc(size_t bytes)
{
    if (bytes == 0)
        bytes = 16;
    AllocHook h;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        h = g_hook;
    }
    void *p = nullptr;
    if (h.alloc) {
        p = h.alloc(bytes, h.ctx);
        if (!p)
            fail(FNN_ENOMEM, "user allocator returned NULL for %zu bytes",
                 bytes);
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p)
        fail(FNN_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes,
             hipGetErrorString(e));
    return p;
}

void out_free(void *p)
{
    if (!p)
        return;
    AllocHook h;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        h = g_hook;
    }
    if (h.free_)
        h.free_(p, h.ctx);
    else
        (void)hipFree(p);
}

// ------------------------------------------------------------------ scan --

constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

template <class T>
__device__ T block_excl_scan(T v, T *total)
{
    __shared__ T wsum[SCAN_T / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    T incl = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        T u = __shfl_up(incl, o, WAVE);
        if (lane >= o)
            incl += u;
    }
    if (lane == WAVE - 1)
        wsum[wid] = incl;
    __syncthreads();
    T off = 0, tot = 0;
    for (int w = 0; w < SCAN_T / WAVE; ++w) {
        if (w < wid)
            off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

template <class TI, class TO>
__global__ void __launch_bounds__(SCAN_T)
k_scan_tiles(const TI *__restrict__ in, TO *__restrict__ out,
             TO *__restrict__ tile_sums, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE +
                         (int64_t)threadIdx.x * SCAN_ITEMS;
    TO v[SCAN_ITEMS];
    TO s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t g = base + i;
        v[i] = g < n ? (TO)in[g] : (TO)0;
        s += v[i];
    }
    TO tot;
    TO off = block_excl_scan<TO>(s, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t g = base + i;
        if (g < n)
            out[g] = off;
        off += v[i];
    }
    if (threadIdx.x == 0)
        tile_sums[blockIdx.x] = tot;
}

template <class TO>
__global__ void __launch_bounds__(SCAN_T)
k_scan_add(TO *__restrict__ out, const TO *__restrict__ tile_off, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    const TO o = tile_off[blockIdx.x];
    for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_T) {
        int64_t g = base + i;
        if (g < n)
            out[g] += o;
    }
}

template <class TO>
__global__ void k_scan_total(TO *__restrict__ out, const TO *__restrict__ tile_off,
                             int64_t ntiles, int64_t n)
{
    out[n] = tile_off[ntiles];
}

template <class TO>
__global__ void k_scan_single(TO *__restrict__ offs, const TO *__restrict__ sums)
{
    offs[0] = 0;
    offs[1] = sums[0];
}

template <class TI, class TO>
static void scan_impl(const TI *in, TO *out, int64_t n, Scratch &S)
{
    hipStream_t s = S.stream();
    if (n <= 0) {
        fill(out, (TO)0, 1, s);
        return;
    }
    int64_t ntiles = cdiv(n, SCAN_TILE);
    TO *sums = S.get<TO>(ntiles + 1);
    TO *offs = S.get<TO>(ntiles + 1);
    FNN_LAUNCH((k_scan_tiles<TI, TO>), dim3((unsigned)ntiles),
                       dim3(SCAN_T), 0, s, in, out, sums, n);
    if (ntiles == 1) {
        FNN_LAUNCH((k_scan_single<TO>), dim3(1), dim3(1), 0, s, offs,
                           sums);
    } else {
        scan_impl<TO, TO>(sums, offs, ntiles, S);
    }
    FNN_LAUNCH((k_scan_add<TO>), dim3((unsigned)ntiles), dim3(SCAN_T),
                       0, s, out, offs, n);
    FNN_LAUNCH((k_scan_total<TO>), dim3(1), dim3(1), 0, s, out, offs,
                       ntiles, n);
}

void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, Scratch &S)
{
    scan_impl<int32_t, int64_t>(in, out, n, S);
}
void scan_i64(const int64_t *in, int64_t *out, int64_t n, Scratch &S)
{
    scan_impl<int64_t, int64_t>(in, out, n, S);
}
void scan_i32(const int32_t *in, int32_t *out, int64_t n, Scratch &S)
{
    scan_impl<int32_t, int32_t>(in, out, n, S);
}

// ------------------------------------------------------------ radix sort --
// One pass per 8-bit digit.  Pass: per-tile digit histograms (digit-major in
// global memory), an exclusive scan over them, then a stable scatter in
// which each wave ranks its 64 items with ballots (items keep their order).

constexpr int RS_T = 256;
constexpr int RS_ITEMS = 4;
constexpr int RS_TILE = RS_T * RS_ITEMS;
constexpr int RS_BINS = 256;

__global__ void __launch_bounds__(RS_T)
k_rs_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
          int32_t *__restrict__ hist, int64_t ntiles)
{
    __shared__ int32_t h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = threadIdx.x; i < RS_TILE; i += RS_T) {
        int64_t g = base + i;
        if (g < n)
            atomicAdd(&h[(keys[g] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(RS_T)
k_rs_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
             uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
             int64_t n, int shift, const int64_t *__restrict__ offs,
             int64_t ntiles)
{
    __shared__ int32_t run[RS_BINS];              // items of each digit so far
    __shared__ int32_t wcnt[RS_T / WAVE][RS_BINS];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    run[threadIdx.x] = 0;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int step = 0; step < RS_ITEMS; ++step) {
        for (int w = 0; w < RS_T / WAVE; ++w)
            wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t g = base + (int64_t)step * RS_T + threadIdx.x;
        const bool valid = g < n;
        uint32_t k = valid ? kin[g] : 0u;
        uint32_t v = valid ? vin[g] : 0u;
        int d = (int)((k >> shift) & 0xFF);
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1);
            match &= ((d >> b) & 1) ? bal : ~bal;
        }
        int rank = __popcll(match & lt);
        int cnt = __popcll(match);
        // the last lane of each digit group publishes the wave's count
        bool leader = valid && ((match >> lane) >> 1) == 0ull;
        if (leader)
            wcnt[wid][d] = cnt;
        __syncthreads();
        if (valid) {
            int before = run[d];
            for (int w = 0; w < wid; ++w)
                before += wcnt[w][d];
            int64_t pos = offs[(int64_t)d * ntiles + blockIdx.x] + before + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        {
            int t = threadIdx.x;  // one thread per digit bin
            int add = 0;
            for (int w = 0; w < RS_T / WAVE; ++w)
                add += wcnt[w][t];
            run[t] += add;
        }
        __syncthreads();
    }
}

void radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in,
                      uint32_t *keys_out, uint32_t *vals_out, int64_t n,
                      int bits, Scratch &S)
{
    hipStream_t s = S.stream();
    if (n <= 0)
        return;
    if (bits < 1)
        bits = 1;
    const int passes = (bits + 7) / 8;
    const int64_t ntiles = cdiv(n, RS_TILE);
    int32_t *hist = S.get<int32_t>((size_t)RS_BINS * ntiles);
    int64_t *offs = S.get<int64_t>((size_t)RS_BINS * ntiles + 1);
    uint32_t *tk = S.get<uint32_t>(n), *tv = S.get<uint32_t>(n);
    // Ping-pong so that the last pass writes keys_out / vals_out.
    const uint32_t *ck = keys_in, *cv = vals_in;
    for (int p = 0; p < passes; ++p) {
        bool last = p == passes - 1;
        bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *ok = to_out ? keys_out : tk;
        uint32_t *ov = to_out ? vals_out : tv;
        (void)last;
        FNN_LAUNCH(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_T), 0, s,
                           ck, n, p * 8, hist, ntiles);
        scan_i32_to_i64(hist, offs, (int64_t)RS_BINS * ntiles, S);
        FNN_LAUNCH(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_T), 0,
                           s, ck, cv, ok, ov, n, p * 8, offs, ntiles);
        ck = ok;
        cv = ov;
    }
}

}  // namespace fnn
