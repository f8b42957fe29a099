// Error reporting, device helpers and small ABI functions of libgila.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>
#include <algorithm>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "device_util.h"
#include "gila_internal.h"

namespace gila {

// ------------------------------------------------------------------ exclusive scan (int64)
constexpr int kScanItems = 8;                  // items per thread
constexpr int kScanTile = kBlock * kScanItems;  // items per workgroup

__global__ __launch_bounds__(kBlock) void scan_tiles_kernel(const int64_t* __restrict__ in,
                                                            int64_t* __restrict__ out, int64_t n,
                                                            int64_t* __restrict__ tile_sums) {
    __shared__ int64_t s_red[4];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (t0 + i < n) ? in[t0 + i] : 0;
        sum += v[i];
    }
    int64_t total;
    int64_t run = block_exclusive_scan<int64_t>(sum, s_red, total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        run += v[i];
        if (t0 + i < n) out[t0 + i + 1] = run;
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void scan_sums_kernel(int64_t* __restrict__ sums, int64_t m) {
    // in place: sums[i] <- sums[0] + ... + sums[i-1] (one workgroup)
    __shared__ int64_t s_red[4];
    int64_t carry = 0;
    for (int64_t b = 0; b < m; b += kBlock) {
        const int64_t i = b + threadIdx.x;
        const int64_t x = i < m ? sums[i] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan<int64_t>(x, s_red, total);
        if (i < m) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kBlock) void scan_add_kernel(int64_t* __restrict__ out, int64_t n,
                                                          const int64_t* __restrict__ offs) {
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    const int64_t add = offs[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        const int64_t j = t0 + i;
        if (j < n) out[j + 1] += add;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

int64_t scan_workspace_count(int64_t n) { return n <= 0 ? 1 : (n + kScanTile - 1) / kScanTile; }

int enqueue_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* ws,
                               hipStream_t s) {
    if (n <= 0) {
        hipLaunchKernelGGL(scan_add_kernel, dim3(1), dim3(kBlock), 0, s, out, (int64_t)0, ws);
        GILA_HIP(hipGetLastError());
        return GILA_OK;
    }
    const int64_t tiles = scan_workspace_count(n);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, n,
                       ws);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kBlock), 0, s, ws, tiles);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)tiles), dim3(kBlock), 0, s, out, n, ws);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

int exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    int64_t* ws = nullptr;
    GILA_TRY(dalloc_t(&ws, (size_t)scan_workspace_count(n)));
    const int rc = enqueue_exclusive_scan_i64(in, out, n, ws, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    dfree_on(ws, s);
    if (rc) return rc;
    if (e2 != hipSuccess) return fail(GILA_EDEVICE, "scan failed: %s", hipGetErrorString(e2));
    return GILA_OK;
}

static double wall_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

// A phase timer is also a roctx range of the whole call, with a marker at
// the end of each phase.
PhaseTimer::PhaseTimer(const char* w, hipStream_t s) : what(w), stream(s) {
    roctxRangePushA(w);
    const char* e = getenv("GILA_TIMING");
    on = e && e[0] == '1';
    t0 = last = on ? wall_s() : 0.0;
}

void PhaseTimer::mark(const char* phase) {
    char name[96];
    snprintf(name, sizeof(name), "%s: %s done", what, phase);
    roctxMarkA(name);
    if (!on) return;
    (void)quiet(hipStreamSynchronize(stream));
    const double t = wall_s();
    char buf[128];
    snprintf(buf, sizeof(buf), " %s=%.2f", phase, (t - last) * 1e3);
    log += buf;
    last = t;
}

PhaseTimer::~PhaseTimer() {
    if (on) fprintf(stderr, "[gila timing] %s total=%.2f ms:%s\n", what, (wall_s() - t0) * 1e3,
                    log.c_str());
    roctxRangePop();
}

// A fixed buffer per thread: recording an error never allocates.
static thread_local char t_last_error[1024];

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_last_error, sizeof(t_last_error), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { t_last_error[0] = '\0'; }

// ------------------------------------------------------------------ device memory cache
// hipFree synchronises the whole device.  Blocks released with dfree_on() go to
// a cache instead and are reused by a later dalloc() of the same size class
// once the work on the releasing stream has completed (an event marks it), so
// code that runs beside other streams (the layout server's builder, batched
// launches, ticks) never waits for the whole device.  dfree() keeps
// hipFree's semantics.  Cached blocks beyond kCacheLimit are returned to the
// device (oldest first), and all of them when an allocation fails.
namespace {
struct CachedBlock {
    void* p;
    size_t bytes;
    hipEvent_t ev;  // null: reusable at once
    uint64_t seq;
};
struct LiveBlock {
    int device;
    size_t bytes;
};
std::mutex g_mem_mu;
std::multimap<std::pair<int, size_t>, CachedBlock> g_cache;
std::map<void*, LiveBlock> g_live;
size_t g_cached_bytes = 0;
uint64_t g_seq = 0;
constexpr size_t kCacheLimit = (size_t)16 << 30;

size_t size_class(size_t b) {
    constexpr size_t kBig = (size_t)64 << 20;
    if (b > kBig) return (b + kBig - 1) / kBig * kBig;
    size_t r = 512;
    while (r < b) r <<= 1;
    return r;
}

// hipEventQuery reports pending work as hipErrorNotReady (and may refuse the
// query, e.g. while another thread captures a stream), which HIP also keeps
// as the thread's last error: it is taken back here, so that the next launch
// check does not report it; a block whose event cannot be queried waits.
bool block_ready(const CachedBlock& c) {
    if (!c.ev) return true;
    return quiet(hipEventQuery(c.ev)) == hipSuccess;
}

// Returns ready cached blocks to the device until at most `keep` bytes stay
// cached (all ready blocks for keep = 0).  Lock held.
void trim_locked(size_t keep) {
    std::vector<std::multimap<std::pair<int, size_t>, CachedBlock>::iterator> order;
    for (auto it = g_cache.begin(); it != g_cache.end(); ++it) order.push_back(it);
    std::sort(order.begin(), order.end(),
              [](const auto& a, const auto& b) { return a->second.seq < b->second.seq; });
    for (auto it : order) {
        if (g_cached_bytes <= keep) break;
        if (!block_ready(it->second)) continue;
        DeviceGuard dg(it->first.first);
        if (quiet(hipFree(it->second.p)) != hipSuccess) continue;  // kept for a later trim
        if (it->second.ev) (void)quiet(hipEventDestroy(it->second.ev));
        g_cached_bytes -= it->second.bytes;
        g_cache.erase(it);
    }
}
}  // namespace

int dalloc(void** p, size_t bytes) {
    *p = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GILA_EDEVICE, "no current device");
    const size_t rb = size_class(bytes ? bytes : 16);
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto range = g_cache.equal_range({dev, rb});
        for (auto it = range.first; it != range.second; ++it) {
            if (!block_ready(it->second)) continue;
            *p = it->second.p;
            if (it->second.ev) (void)quiet(hipEventDestroy(it->second.ev));
            g_cached_bytes -= rb;
            g_cache.erase(it);
            g_live[*p] = LiveBlock{dev, rb};
            return GILA_OK;
        }
    }
    hipError_t e = hipMalloc(p, rb);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_mem_mu);
            trim_locked(0);
        }
        e = hipMalloc(p, rb);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? GILA_ENOMEM : GILA_EDEVICE,
                    "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_live[*p] = LiveBlock{dev, rb};
    return GILA_OK;
}

void dfree(void* p) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        g_live.erase(p);
    }
    (void)quiet(hipFree(p));
}

void dfree_on(void* p, hipStream_t s, bool idle) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) {  // not from dalloc: plain free
        (void)quiet(hipFree(p));
        return;
    }
    CachedBlock c{p, it->second.bytes, nullptr, ++g_seq};
    if (!idle) {
        if (hipEventCreateWithFlags(&c.ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(c.ev, s) != hipSuccess) {
            // cannot mark the stream: wait for it instead
            if (c.ev) (void)quiet(hipEventDestroy(c.ev));
            c.ev = nullptr;
            (void)quiet(hipStreamSynchronize(s));
        }
    }
    g_cache.insert({{it->second.device, c.bytes}, c});
    g_cached_bytes += c.bytes;
    g_live.erase(it);
    if (g_cached_bytes > kCacheLimit) trim_locked(kCacheLimit / 2);
}

int64_t release_cached() {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    const size_t before = g_cached_bytes;
    trim_locked(0);
    return (int64_t)(before - g_cached_bytes);
}

Release public_release() {
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return Release{};
    }
    return Release{true, nullptr, true};
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
}

DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)quiet(hipSetDevice(prev));
}

static std::mutex g_mu;
static std::map<int, DeviceInfo> g_info;

// Capture streams are per thread (captures on one stream from two threads
// would interleave) and are destroyed when the thread exits.
struct CaptureStreams {
    std::map<int, hipStream_t> by_device;
    ~CaptureStreams() {
        for (auto& kv : by_device) (void)quiet(hipStreamDestroy(kv.second));
    }
};
static thread_local CaptureStreams t_capture;

hipStream_t capture_stream(int device) {
    auto it = t_capture.by_device.find(device);
    if (it != t_capture.by_device.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    t_capture.by_device[device] = s;
    return s;
}

const DeviceInfo& device_info(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_info.find(device);
    if (it != g_info.end()) return it->second;
    DeviceInfo di;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        v > 0)
        di.cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess &&
        v > 0)
        di.max_lds_per_block = (size_t)v;
    g_info[device] = di;
    return g_info[device];
}

}  // namespace gila

extern "C" {

const char* gila_strerror(int status) {
    switch (status) {
        case GILA_OK: return "ok";
        case GILA_EINVAL: return "invalid argument or malformed graph";
        case GILA_ENOMEM: return "out of memory";
        case GILA_EDEVICE: return "device error";
        case GILA_EAGAIN: return "not ready";
        case GILA_ECANCELED: return "cancelled";
        case GILA_EUNSUPPORTED: return "unsupported";
        case GILA_ENONFINITE: return "non-finite force";
        default: return "unknown status";
    }
}

const char* gila_last_error(void) { return gila::t_last_error; }

int gila_version(void) { return 10000; }

int64_t gila_release_cached_memory(void) { return gila::release_cached(); }

}  // extern "C"
