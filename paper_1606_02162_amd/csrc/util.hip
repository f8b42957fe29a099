// Error reporting, device helpers and small ABI functions of libgila.
#include <cstdio>
#include <map>

#include "gila_internal.h"

namespace gila {

static thread_local std::string t_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return code;
}

void clear_error() { t_last_error.clear(); }

int dalloc(void** p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? GILA_ENOMEM : GILA_EDEVICE,
                    "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return GILA_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
}

DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
}

static std::mutex g_mu;
static std::map<int, hipStream_t> g_capture_streams;
static std::map<int, DeviceInfo> g_info;

hipStream_t capture_stream(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_capture_streams.find(device);
    if (it != g_capture_streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_capture_streams[device] = s;
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
        default: return "unknown status";
    }
}

const char* gila_last_error(void) { return gila::t_last_error.c_str(); }

int gila_version(void) { return 10000; }

}  // extern "C"
