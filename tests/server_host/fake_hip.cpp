// Host-only stand-in for the HIP runtime (see hip/hip_runtime.h).
#include "hip/hip_runtime.h"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

struct Buffer {
    void *p;
    size_t bytes;
};

std::mutex g_mu;  // counters and the live-allocation table
std::map<void *, size_t> g_live;
long g_live_bytes = 0, g_max_live = 0, g_ops = 0, g_graph_launches = 0, g_captures = 0, g_busy_captures = 0;

void *dev_alloc(size_t bytes)
{
    void *p = std::malloc(bytes ? bytes : 1);
    std::lock_guard<std::mutex> lk(g_mu);
    g_live[p] = bytes;
    g_live_bytes += (long)bytes;
    if (g_live_bytes > g_max_live) g_max_live = g_live_bytes;
    return p;
}

void dev_free(void *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_live.find(p);
        if (it == g_live.end()) {
            std::fprintf(stderr, "fake_hip: free of an unknown pointer %p\n", p);
            std::abort();
        }
        g_live_bytes -= (long)it->second;
        g_live.erase(it);
    }
    std::free(p);
}

}  // namespace

struct FakeGraph {
    std::vector<std::function<void()>> ops;
    std::vector<Buffer> owned;  // graph-owned allocations (freed with the graph)
};

struct FakeStream {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    bool running = false, stop = false;
    FakeGraph *capture = nullptr;
    std::thread::id capture_thread;
    std::thread worker;

    void loop()
    {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv.wait(lk, [&] { return stop || !q.empty(); });
            if (q.empty() && stop) return;
            std::function<void()> fn = std::move(q.front());
            q.pop_front();
            running = true;
            lk.unlock();
            fn();
            lk.lock();
            running = false;
            cv.notify_all();
        }
    }
};

namespace {

// Run now on the stream's worker, or record into its capture.  Operations
// from a thread other than the capturing one are an error under capture.
hipError_t enqueue(hipStream_t s, std::function<void()> fn)
{
    if (!s) {
        fn();  // the null stream: run synchronously
        return hipSuccess;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->capture) {
        if (std::this_thread::get_id() != s->capture_thread) return hipErrorStreamCaptureUnsupported;
        s->capture->ops.push_back(std::move(fn));
        return hipSuccess;
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        ++g_ops;
    }
    s->q.push_back(std::move(fn));
    s->cv.notify_all();
    return hipSuccess;
}

}  // namespace

const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake hip error"; }
hipError_t hipGetDevice(int *dev)
{
    *dev = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t bytes)
{
    *p = dev_alloc(bytes);
    return hipSuccess;
}
hipError_t hipFree(void *p)
{
    dev_free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned)
{
    *p = std::malloc(bytes ? bytes : 1);
    return hipSuccess;
}
hipError_t hipHostFree(void *p)
{
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind)
{
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemset(void *dst, int v, size_t bytes)
{
    std::memset(dst, v, bytes);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    FakeStream *f = new FakeStream();
    f->worker = std::thread([f] { f->loop(); });
    *s = f;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    if (!s) return hipSuccess;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->capture) return hipErrorStreamCaptureUnsupported;
    s->cv.wait(lk, [&] { return s->q.empty() && !s->running; });
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    if (!s) return hipSuccess;
    (void)hipStreamSynchronize(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->worker.join();
    delete s;
    return hipSuccess;
}

hipError_t hipMallocAsync(void **p, size_t bytes, hipStream_t s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->capture) {
        if (std::this_thread::get_id() != s->capture_thread) return hipErrorStreamCaptureUnsupported;
        // graph-owned: one address for every replay, contents undefined at
        // each allocation
        void *q = dev_alloc(bytes);
        s->capture->owned.push_back({q, bytes});
        s->capture->ops.push_back([q, bytes] { std::memset(q, 0xA5, bytes); });
        *p = q;
        return hipSuccess;
    }
    lk.unlock();
    *p = dev_alloc(bytes);
    return hipSuccess;
}

hipError_t hipFreeAsync(void *p, hipStream_t s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->capture) {
        if (std::this_thread::get_id() != s->capture_thread) return hipErrorStreamCaptureUnsupported;
        size_t bytes = 0;
        bool found = false;
        for (const Buffer &b : s->capture->owned)
            if (b.p == p) {
                bytes = b.bytes;
                found = true;
            }
        if (!found) return hipErrorInvalidValue;  // freeing memory the graph does not own
        s->capture->ops.push_back([p, bytes] { std::memset(p, 0x5A, bytes); });
        return hipSuccess;
    }
    lk.unlock();
    return enqueue(s, [p] { dev_free(p); });
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s)
{
    return enqueue(s, [dst, src, bytes] { std::memcpy(dst, src, bytes); });
}

// FAKE_HOSTFN_TAIL_US=t keeps a host-function operation running t
// microseconds after the function returns (a runtime that finishes its own
// bookkeeping of the command after the callback), to widen that window.
hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void *arg)
{
    static const long tail_us = [] {
        const char *v = std::getenv("FAKE_HOSTFN_TAIL_US");
        return v ? std::atol(v) : 0L;
    }();
    return enqueue(s, [fn, arg] {
        fn(arg);
        if (tail_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(tail_us));
    });
}

hipError_t fake_enqueue(hipStream_t s, std::function<void()> fn) { return enqueue(s, std::move(fn)); }

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->capture) return hipErrorIllegalState;
    {
        std::lock_guard<std::mutex> g(g_mu);
        ++g_captures;
        if (!s->q.empty() || s->running) ++g_busy_captures;
    }
    s->capture = new FakeGraph();
    s->capture_thread = std::this_thread::get_id();
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->capture) return hipErrorIllegalState;
    *g = s->capture;
    s->capture = nullptr;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    // the executable takes over the graph's operations and owned memory
    FakeGraph *e = new FakeGraph();
    e->ops = g->ops;
    e->owned.swap(g->owned);
    *exec = e;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    if (!g) return hipSuccess;
    for (const Buffer &b : g->owned) dev_free(b.p);
    delete g;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t e) { return hipGraphDestroy(e); }

hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s)
{
    {
        std::lock_guard<std::mutex> g(g_mu);
        ++g_graph_launches;
    }
    return enqueue(s, [e] {
        for (auto &op : e->ops) op();
    });
}

FakeStats fake_stats()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return FakeStats{g_ops, g_graph_launches, g_captures, g_busy_captures, g_max_live};
}
