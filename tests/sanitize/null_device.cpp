// A "null device" for host-side tests of the library (test code only; never
// linked into libmrtlbm.so): the HIP runtime calls that the library's host
// code and its kernel launch stubs make, implemented on host memory. Device
// memory is host memory, copies are memcpy, streams and events complete at
// once, and a kernel launch is recorded by the name the kernel was registered
// under, not executed. The library's own host code (descriptor validation,
// workspace carving, bookkeeping of time and buffers, graph building,
// snapshot format, status codes) runs unchanged on top of it.
//
// Only the two reduction kernels are given a behaviour, the one the host code
// depends on: their three sums come out 0, 0, 1 (finite), or all three NaN
// when a population of the state they read is not finite, which is what a
// real reduction over such a state returns. Nothing else of the method is
// computed here.
//
// Test hooks (extern "C", declared by tests/sanitize/null_driver.cpp):
//   null_device_launches(sub)      launches (direct and graph replays) of
//                                  kernels whose name contains sub
//   null_device_fail_after(n)      the n-th next fallible call (launch, copy,
//                                  synchronisation, graph launch) fails with
//                                  hipErrorLaunchFailure (n = 0: the next one;
//                                  n < 0: never)
//   null_device_poke_state(i, x, y, v)
//                                  writes v into population i of node (x, y)
//                                  of the state the last reduction read
//                                  (FP32 storage)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_device.h"

namespace {

std::mutex g_mu;
std::map<const void *, std::string> &kernel_names() {
    static std::map<const void *, std::string> m;
    return m;
}
std::map<const void *, std::vector<unsigned char>> &variables() {
    static std::map<const void *, std::vector<unsigned char>> m;
    return m;
}
std::map<std::string, long> &launch_counts() {
    static std::map<std::string, long> m;
    return m;
}
int g_fail_after = -1;
hipError_t g_last = hipSuccess;
bool g_reduce_bad = false;
mrt::Dom g_reduce_dom{};
bool g_have_reduce_dom = false;

struct Config {
    dim3 grid, block;
    size_t shmem;
    hipStream_t stream;
};
thread_local std::vector<Config> g_config;

struct NullEvent { int recorded = 0; };
struct NullGraph { std::vector<const void *> nodes; };
struct NullExec { std::vector<const void *> nodes; };

// consumes one fallible call; true when it is to fail
bool inject_failure() {
    if (g_fail_after < 0) return false;
    if (g_fail_after-- == 0) {
        g_last = hipErrorLaunchFailure;
        return true;
    }
    return false;
}

bool name_has(const std::string &name, const char *sub) { return name.find(sub) != std::string::npos; }

// the state a reduction reads: 8 planes of [ny][pitch], FP32 or binary16
bool state_finite(const mrt::Dom &d, bool half) {
    for (int i = 0; i < 8; ++i)
        for (int y = 0; y < d.ny; ++y)
            for (int x = 0; x < d.nx; ++x) {
                const int64_t k = (int64_t)i * d.plane + (int64_t)y * d.pitch + x;
                if (half) {
                    uint16_t h;
                    std::memcpy(&h, (const unsigned char *)d.fin + 2 * k, 2);
                    if ((h & 0x7c00u) == 0x7c00u) return false;
                } else {
                    float v;
                    std::memcpy(&v, (const unsigned char *)d.fin + 4 * k, 4);
                    if (!std::isfinite(v)) return false;
                }
            }
    return true;
}

void run_kernel(const void *fn, void **args) {
    std::string name;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = kernel_names().find(fn);
        name = it == kernel_names().end() ? std::string("<unregistered>") : it->second;
        ++launch_counts()[name];
    }
    if (!args) return;  // a graph replay: recorded only
    if (name_has(name, "k_reduce_final")) {
        // (const double *partials, int nblocks, double *result)
        double *result = *(double **)args[2];
        const double bad = std::nan("");
        result[0] = g_reduce_bad ? bad : 0.0;
        result[1] = g_reduce_bad ? bad : 0.0;
        result[2] = g_reduce_bad ? bad : 1.0;
    } else if (name_has(name, "k_reduce")) {
        // (Dom cur, int src, const float *uprev, double *partials)
        g_reduce_dom = *(const mrt::Dom *)args[0];
        g_have_reduce_dom = true;
        g_reduce_bad = !state_finite(g_reduce_dom, name_has(name, "DF16_"));
    }
}

}  // namespace

extern "C" {

long null_device_launches(const char *sub) {
    std::lock_guard<std::mutex> lock(g_mu);
    long n = 0;
    for (const auto &kv : launch_counts())
        if (name_has(kv.first, sub)) n += kv.second;
    return n;
}

void null_device_fail_after(int n) { g_fail_after = n; }

int null_device_poke_state(int i, int x, int y, float v) {
    if (!g_have_reduce_dom) return -1;
    const mrt::Dom &d = g_reduce_dom;
    if (i < 0 || i >= 8 || x < 0 || x >= d.nx || y < 0 || y >= d.ny) return -1;
    float *f = (float *)d.fin;
    f[(int64_t)i * d.plane + (int64_t)y * d.pitch + x] = v;
    return 0;
}

// --- registration and launch hooks of HIP-Clang's host code ---

void **__hipRegisterFatBinary(const void *) {
    static void *module = nullptr;
    return &module;
}

void __hipUnregisterFatBinary(void **) {}

void __hipRegisterFunction(void **, const void *hostFunction, char *, const char *deviceName, unsigned int,
                           uint3 *, uint3 *, dim3 *, dim3 *, int *) {
    std::lock_guard<std::mutex> lock(g_mu);
    kernel_names()[hostFunction] = deviceName ? deviceName : "";
}

void __hipRegisterVar(void **, void *var, char *, char *, int, size_t size, int, int) {
    std::lock_guard<std::mutex> lock(g_mu);
    variables()[var].assign(size, 0);
}

hipError_t __hipPushCallConfiguration(dim3 gridDim, dim3 blockDim, size_t sharedMem, hipStream_t stream) {
    g_config.push_back(Config{gridDim, blockDim, sharedMem, stream});
    return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3 *gridDim, dim3 *blockDim, size_t *sharedMem, hipStream_t *stream) {
    if (g_config.empty()) return hipErrorInvalidConfiguration;
    const Config c = g_config.back();
    g_config.pop_back();
    *gridDim = c.grid;
    *blockDim = c.block;
    *sharedMem = c.shmem;
    *stream = c.stream;
    return hipSuccess;
}

}  // extern "C"

// --- runtime API ---

hipError_t hipLaunchKernel(const void *function_address, dim3, dim3, void **args, size_t, hipStream_t) {
    if (inject_failure()) return hipErrorLaunchFailure;
    run_kernel(function_address, args);
    return hipSuccess;
}

hipError_t hipGetLastError(void) {
    const hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}

const char *hipGetErrorString(hipError_t e) {
    switch (e) {
    case hipSuccess: return "no error";
    case hipErrorLaunchFailure: return "launch failure (injected by the null device)";
    case hipErrorInvalidValue: return "invalid value";
    case hipErrorInvalidDevice: return "invalid device";
    default: return "null-device error";
    }
}

hipError_t hipGetDevice(int *dev) {
    *dev = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidDevice; }

hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *prop, int dev) {
    if (dev != 0) return hipErrorInvalidDevice;
    std::memset(prop, 0, sizeof(*prop));
    std::strcpy(prop->name, "null device");
    std::strcpy(prop->gcnArchName, "null");
    prop->multiProcessorCount = 4;
    return hipSuccess;
}

hipError_t hipDeviceGetAttribute(int *pi, hipDeviceAttribute_t attr, int dev) {
    if (dev != 0) return hipErrorInvalidDevice;
    *pi = attr == hipDeviceAttributeMultiprocessorCount ? 4 : 0;
    return hipSuccess;
}

hipError_t hipGetSymbolAddress(void **devPtr, const void *symbol) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = variables().find(symbol);
    if (it == variables().end()) return hipErrorInvalidSymbol;
    *devPtr = it->second.data();
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t) {
    if (inject_failure()) return hipErrorLaunchFailure;
    if (bytes) std::memmove(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind, hipStream_t) {
    if (inject_failure()) return hipErrorLaunchFailure;
    if (width > dpitch || width > spitch) return hipErrorInvalidValue;
    for (size_t r = 0; r < height; ++r)
        std::memmove((char *)dst + r * dpitch, (const char *)src + r * spitch, width);
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) {
    if (inject_failure()) return hipErrorLaunchFailure;
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) {
    *e = reinterpret_cast<hipEvent_t>(new NullEvent());
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e) {
    delete reinterpret_cast<NullEvent *>(e);
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    ++reinterpret_cast<NullEvent *>(e)->recorded;
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t) {
    if (inject_failure()) return hipErrorLaunchFailure;
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float *ms, hipEvent_t start, hipEvent_t stop) {
    if (!reinterpret_cast<NullEvent *>(start)->recorded || !reinterpret_cast<NullEvent *>(stop)->recorded)
        return hipErrorInvalidHandle;
    *ms = 1.0f;  // every candidate of a tuner takes equally long
    return hipSuccess;
}

hipError_t hipGraphCreate(hipGraph_t *g, unsigned int) {
    *g = reinterpret_cast<hipGraph_t>(new NullGraph());
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<NullGraph *>(g);
    return hipSuccess;
}

hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t g, const hipGraphNode_t *, size_t,
                                 const hipKernelNodeParams *p) {
    NullGraph *G = reinterpret_cast<NullGraph *>(g);
    G->nodes.push_back(p->func);
    *node = reinterpret_cast<hipGraphNode_t>(G->nodes.size());
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    *exec = reinterpret_cast<hipGraphExec_t>(new NullExec{reinterpret_cast<NullGraph *>(g)->nodes});
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
    delete reinterpret_cast<NullExec *>(exec);
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t) {
    if (inject_failure()) return hipErrorLaunchFailure;
    for (const void *fn : reinterpret_cast<NullExec *>(exec)->nodes) run_kernel(fn, nullptr);
    return hipSuccess;
}
