// Host runtime helpers: error propagation, stream binding, stream-ordered
// scratch memory, and the device primitives (scan, radix sort) used by the
// build and the query.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

namespace fnn {

// Internal exception; converted to an error code at the C ABI.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char *fmt, ...);

#define FNN_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            ::fnn::fail(-3, "%s failed: %s (%s:%d)", #call,                  \
                        hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

// Launches issued by this thread (kernels launched eagerly, graphs
// replayed); kernels recorded into a graph count when it is replayed.
struct LaunchCount {
    long long kernels = 0, graphs = 0, graph_kernels = 0;
    bool capturing = false;
};
LaunchCount &launch_count();

#define FNN_LAUNCH(kernel, grid, block, shmem, stream, ...)                  \
    do {                                                                     \
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__); \
        FNN_HIP(hipGetLastError());                                          \
        ::fnn::LaunchCount &lc_ = ::fnn::launch_count();                     \
        if (!lc_.capturing)                                                  \
            ++lc_.kernels;                                                   \
    } while (0)

hipStream_t current_stream();

// A launch sequence recorded once (begin(); launches on `cs`; end()) and
// replayed on any stream.  Recorded sequences hold only kernel launches:
// clears are fill kernels, never memset nodes.
hipStream_t capture_stream();

// Compute units of the current device (cached per device id).
int num_cus();
struct GraphRun {
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool capturing = false;
    long long nkernels = 0;  // kernel nodes recorded
    GraphRun() = default;
    GraphRun(const GraphRun &) = delete;
    GraphRun &operator=(const GraphRun &) = delete;
    ~GraphRun();
    void begin();
    void end();
    void launch(hipStream_t s);
};

// Scratch memory of one call: bump-allocated from device chunks.  With a
// caller allocator set (fnn_set_allocator) every chunk comes from it and
// goes back to it on scope exit; otherwise chunks come from a per-device
// cache of hipMalloc'd chunks and return to it.  Either way the stream
// drains first.
class Scratch {
  public:
    explicit Scratch(hipStream_t s);
    ~Scratch();
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    void *raw(size_t bytes);
    template <class T>
    T *get(size_t count)
    {
        return static_cast<T *>(raw(count * sizeof(T) + 16));
    }
    void release(void *p);
    hipStream_t stream() const { return s_; }

  private:
    hipStream_t s_;
    int dev_ = 0;
    std::vector<std::pair<void *, size_t>> chunks_;  // held by this scope
    std::vector<bool> hooked_;  // chunk came from the caller's allocator
    size_t used_ = 0;                                // bump offset in the last
};

// Memory handed to the caller (tree / CSR arrays): the user allocator if one
// is set, else hipMalloc.
void *out_alloc(size_t bytes);
void out_free(void *p);

// Exclusive scan: out[0..n] with out[n] = total.
void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, Scratch &S);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, Scratch &S);
void scan_i32(const int32_t *in, int32_t *out, int64_t n, Scratch &S);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// key.  Sorted output lands in keys_out / vals_out.
void radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in,
                      uint32_t *keys_out, uint32_t *vals_out, int64_t n,
                      int bits, Scratch &S);

// Device fill with a kernel (never a memset node, so the call is safe to
// record in a captured graph).
template <class T>
__global__ void k_fill(T *__restrict__ p, T v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st)
        p[i] = v;
}

template <class T>
void fill(T *p, T v, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    FNN_LAUNCH((k_fill<T>), dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

template <class T>
T read_scalar(const T *dptr, hipStream_t s)
{
    T v;
    FNN_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
    FNN_HIP(hipStreamSynchronize(s));
    return v;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A dispatch carries its grid size in work-items as a 32-bit number, so a
// launch is capped at MAX_BLOCKS work-groups and kernels whose item count
// grows with the input loop over items with a grid stride.
constexpr int64_t MAX_BLOCKS = 1 << 20;
inline unsigned grid_for(int64_t items, int64_t items_per_block)
{
    int64_t b = cdiv(items, items_per_block);
    if (b < 1)
        b = 1;
    if (b > MAX_BLOCKS)
        b = MAX_BLOCKS;
    return (unsigned)b;
}

// Grid for kernels that stride over their items: at most `cap` work-groups.
// Launching one short-lived work-group per small item leaves the chip
// bound by work-group dispatch (few resident waves); a bounded grid keeps
// every CU busy with long-lived waves.
inline unsigned grid_cap(int64_t items, int64_t items_per_block, unsigned cap)
{
    const unsigned g = grid_for(items, items_per_block);
    return g < cap ? g : cap;
}

}  // namespace fnn
