// Host-only stand-in for the subset of the HIP runtime API that the library's
// host code (umi_host.hip, umi_server.hip) calls, so that code can be built
// with g++ and run under the address, undefined-behaviour and thread
// sanitizers on a machine without a GPU.  "Device" memory is host memory and
// every operation runs to completion when it is enqueued, so streams and
// events need no tracking; a stream capture records the copies, fills and
// (through record_or_run) kernel launches made on the capturing thread, and
// a graph launch replays them in order.  One device with 256 compute units
// exists.  Kernel launches are not part of it: the test driver supplies the
// launch wrappers the host code calls.  Test infrastructure only.
#pragma once

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#define __host__
#define __device__
#define __global__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))

struct int2 { int x, y; };
struct int4 { int x, y, z, w; };
inline int2 make_int2(int x, int y) { return int2{x, y}; }

typedef enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1,
               hipErrorNoDevice = 100, hipErrorLaunchFailure = 719 } hipError_t;
typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 } hipMemcpyKind;
typedef enum { hipDeviceAttributeMultiprocessorCount = 16 } hipDeviceAttribute_t;
typedef enum { hipStreamCaptureModeThreadLocal = 1 } hipStreamCaptureMode;
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph_t* hipGraph_t;
typedef struct ihipGraphExec_t* hipGraphExec_t;
typedef struct ihipGraphNode_t* hipGraphNode_t;
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u
#define hipStreamNonBlocking 1u

namespace fake_hip {
// counters the driver reads to check that calls balance (any thread may move them)
inline std::atomic<long>& live_device_blocks() { static std::atomic<long> n{0}; return n; }
inline std::atomic<long>& live_host_blocks() { static std::atomic<long> n{0}; return n; }
inline std::atomic<long>& live_events() { static std::atomic<long> n{0}; return n; }
inline std::atomic<long>& live_graphs() { static std::atomic<long> n{0}; return n; }
inline std::atomic<long>& device_mallocs() { static std::atomic<long> n{0}; return n; }
inline std::atomic<long>& live_streams() { static std::atomic<long> n{0}; return n; }

// A captured graph: the operations recorded between begin and end capture.
struct Graph {
    std::vector<std::function<hipError_t()>> ops;
};
inline Graph*& capturing()
{
    static thread_local Graph* g = nullptr;
    return g;
}
// Runs `op` now, or records it into the graph this thread is capturing.
inline hipError_t record_or_run(std::function<hipError_t()> op)
{
    if (capturing()) {
        capturing()->ops.push_back(std::move(op));
        return hipSuccess;
    }
    return op();
}
}  // namespace fake_hip

inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake hip error"; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n)
{
    *p = std::malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    ++fake_hip::live_device_blocks();
    ++fake_hip::device_mallocs();
    return hipSuccess;
}
inline hipError_t hipFree(void* p)
{
    if (p) --fake_hip::live_device_blocks();
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned)
{
    *p = std::malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    ++fake_hip::live_host_blocks();
    return hipSuccess;
}
// pinned memory is reachable by the device at its own address
inline hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned)
{
    *d = h;
    return hipSuccess;
}
inline hipError_t hipHostFree(void* p)
{
    if (p) --fake_hip::live_host_blocks();
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t)
{
    return fake_hip::record_or_run([=] {
        if (n) std::memcpy(d, s, n);
        return hipSuccess;
    });
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t)
{
    return fake_hip::record_or_run([=] {
        if (n) std::memset(d, v, n);
        return hipSuccess;
    });
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned)
{
    *s = reinterpret_cast<hipStream_t>(new char[1]);
    ++fake_hip::live_streams();
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s)
{
    if (s) --fake_hip::live_streams();
    delete[] reinterpret_cast<char*>(s);
    return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned)
{
    *e = reinterpret_cast<hipEvent_t>(new char[1]);
    ++fake_hip::live_events();
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e)
{
    if (e) --fake_hip::live_events();
    delete[] reinterpret_cast<char*>(e);
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode)
{
    if (fake_hip::capturing()) return hipErrorInvalidValue;
    fake_hip::capturing() = new fake_hip::Graph();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g)
{
    fake_hip::Graph* c = fake_hip::capturing();
    if (!c) return hipErrorInvalidValue;
    fake_hip::capturing() = nullptr;
    *g = reinterpret_cast<hipGraph_t>(c);
    ++fake_hip::live_graphs();
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t)
{
    *x = reinterpret_cast<hipGraphExec_t>(new fake_hip::Graph(*reinterpret_cast<fake_hip::Graph*>(g)));
    ++fake_hip::live_graphs();
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t)
{
    for (auto& op : reinterpret_cast<fake_hip::Graph*>(x)->ops) {
        const hipError_t e = op();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    if (x) --fake_hip::live_graphs();
    delete reinterpret_cast<fake_hip::Graph*>(x);
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g)
{
    if (g) --fake_hip::live_graphs();
    delete reinterpret_cast<fake_hip::Graph*>(g);
    return hipSuccess;
}
enum hipMemoryType { hipMemoryTypeUnregistered = 0, hipMemoryTypeHost = 1, hipMemoryTypeDevice = 2 };
struct hipPointerAttribute_t {
    enum hipMemoryType type;
    int device;
    void* devicePointer;
    void* hostPointer;
    int isManaged;
    unsigned allocationFlags;
};
// every pointer counts as pinned host memory reachable at its own address
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p)
{
    a->type = hipMemoryTypeHost;
    a->device = 0;
    a->devicePointer = const_cast<void*>(p);
    a->hostPointer = const_cast<void*>(p);
    a->isManaged = 0;
    a->allocationFlags = 0;
    return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
template <class T>
inline hipError_t hipGetSymbolAddress(void** p, T sym)
{
    *p = const_cast<void*>(static_cast<const void*>(sym));
    return hipSuccess;
}
