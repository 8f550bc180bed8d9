// Host-only stand-in for the HIP runtime API, for building the query
// server's host logic on the CPU (under AddressSanitizer or ThreadSanitizer)
// without a GPU.  Only the calls the server makes are declared.  Semantics
// (fake_hip.cpp):
//   - "device" memory is host memory; kernels do not exist (the server's
//     device work is done by stub launchers that enqueue host closures);
//   - a stream is a worker thread running its queued operations in order
//     (copies, host functions, stub kernels, graph launches);
//   - stream capture records the operations enqueued on the capturing
//     stream into a graph instead of running them; a stream-ordered
//     allocation under capture becomes graph-owned memory whose contents
//     are poisoned when the graph frees it and when a replay allocates it;
//   - hipGraphLaunch enqueues one operation that runs the graph's
//     operations in order.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>

typedef int hipError_t;
enum : int {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorIllegalState = 401,
    hipErrorStreamCaptureUnsupported = 900
};

typedef struct FakeStream *hipStream_t;
typedef struct FakeGraph *hipGraph_t;
typedef struct FakeGraph *hipGraphExec_t;
typedef struct FakeGraph *hipGraphNode_t;
typedef void (*hipHostFn_t)(void *);

enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
                            hipStreamCaptureModeRelaxed = 2 };
#define hipStreamNonBlocking 0x01

const char *hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int *dev);
hipError_t hipSetDevice(int dev);
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned flags = 0);
hipError_t hipHostFree(void *p);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemset(void *dst, int value, size_t bytes);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipMallocAsync(void **p, size_t bytes, hipStream_t s);
hipError_t hipFreeAsync(void *p, hipStream_t s);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void *arg);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *err_node, char *log, size_t n);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);

// Harness side: enqueue a closure on a stream (or into its capture), as a
// kernel launch would be; and the counters the driver reports.
hipError_t fake_enqueue(hipStream_t s, std::function<void()> fn);
struct FakeStats {
    long ops, graph_launches, captures, captures_on_busy_stream, max_live_device_bytes;
};
FakeStats fake_stats();
