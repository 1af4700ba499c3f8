// Caching device allocator and small host/device helpers.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace nair {

void fail(nair_status code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        nair_status code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? NAIR_ENOMEM : NAIR_EDEVICE;
        fail(code, std::string(what) + ": " + hipGetErrorString(e));
    }
}

namespace {

// Size classes: multiples of 256 B up to 64 KiB, then 8 classes per power of two
// (at most 12.5% slack).  Freed blocks are kept per (device, class).
size_t size_class(size_t bytes) {
    if (bytes <= 65536) return (bytes + 255) & ~static_cast<size_t>(255);
    int lg = 63 - __builtin_clzll(bytes);
    size_t step = static_cast<size_t>(1) << (lg - 3);
    return (bytes + step - 1) / step * step;
}

struct Pool {
    std::mutex mu;
    std::unordered_map<void *, std::pair<int, size_t>> live;         // ptr -> (device, class)
    std::map<std::pair<int, size_t>, std::vector<void *>> free_list;  // (device, class) -> ptrs
    std::unordered_map<void *, std::pair<const ExtAlloc *, void *>> ext_live;   // caller's blocks -> (allocator, stream)
};

thread_local const ExtAlloc *g_ext = nullptr;
thread_local void *g_ext_stream = nullptr;

Pool &pool() {
    static Pool *p = new Pool();   // never destroyed: frees at exit would race the runtime teardown
    return *p;
}

}  // namespace

AllocScope::AllocScope(const ExtAlloc *e, void *stream) : prev(g_ext), prev_stream(g_ext_stream) {
    g_ext = e;
    g_ext_stream = stream;
}

AllocScope::~AllocScope() {
    g_ext = prev;
    g_ext_stream = prev_stream;
}

void *pool_alloc(size_t bytes) {
    if (g_ext) {   // the handle's caller-supplied allocator
        const size_t n = bytes ? bytes : 1;
        void *p = g_ext->a.alloc(n, g_ext_stream, g_ext->a.ctx);
        if (!p) fail(NAIR_ENOMEM, "the caller's allocator returned no memory for " + std::to_string(n) + " bytes");
        Pool &P = pool();
        std::lock_guard<std::mutex> lk(P.mu);
        P.ext_live[p] = {g_ext, g_ext_stream};
        return p;
    }
    int dev = 0;
    NAIR_HIP(hipGetDevice(&dev));
    size_t cls = size_class(bytes ? bytes : 1);
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.free_list.find({dev, cls});
        if (it != P.free_list.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            P.live[p] = {dev, cls};
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
        // release cached blocks and retry once
        (void)hipGetLastError();
        pool_trim();
        e = hipMalloc(&p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(NAIR_ENOMEM, "device allocation of " + std::to_string(cls) + " bytes failed");
        }
    }
    std::lock_guard<std::mutex> lk(P.mu);
    P.live[p] = {dev, cls};
    return p;
}

void pool_free(void *p) {
    if (!p) return;
    Pool &P = pool();
    std::unique_lock<std::mutex> lk(P.mu);
    auto xt = P.ext_live.find(p);
    if (xt != P.ext_live.end()) {
        const ExtAlloc *e = xt->second.first;
        void *stream = xt->second.second;
        P.ext_live.erase(xt);
        lk.unlock();
        e->a.free(p, stream, e->a.ctx);
        return;
    }
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    P.free_list[it->second].push_back(p);
    P.live.erase(it);
}

void pool_trim() {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : P.free_list) {
        (void)hipSetDevice(kv.first.first);
        for (void *p : kv.second) (void)hipFree(p);
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

// ------------------------------------------------------------ kernel timer

thread_local int g_timer_level = 0;
thread_local bool g_matrix_cores = true;
thread_local bool g_capturing = false;
thread_local bool g_timer_off = false;

namespace {
struct Timer {
    std::mutex mu;
    int kernel = -1, level = -1;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<int> pending_count;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;
    int64_t launches = 0;
    double total_ms = 0.0;
};
Timer &timer() {
    static Timer *t = new Timer();
    return *t;
}
}  // namespace

TimerScope::TimerScope(int kernel, int level, hipStream_t stream, int launches) : on(false), s(stream) {
    if (g_capturing || g_timer_off) return;
    Timer &T = timer();
    if (T.kernel != kernel || (T.level >= 0 && T.level != level)) return;
    std::lock_guard<std::mutex> lk(T.mu);
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!T.spare.empty()) {
        ev = T.spare.back();
        T.spare.pop_back();
    } else {
        NAIR_HIP(hipEventCreate(&ev.first));
        NAIR_HIP(hipEventCreate(&ev.second));
    }
    NAIR_HIP(hipEventRecord(ev.first, s));
    T.pending.push_back(ev);
    T.pending_count.push_back(launches);
    on = true;
}

TimerScope::~TimerScope() {
    if (!on) return;
    Timer &T = timer();
    std::lock_guard<std::mutex> lk(T.mu);
    (void)hipEventRecord(T.pending.back().second, s);
}

void timer_select(int kernel, int level) {
    Timer &T = timer();
    std::lock_guard<std::mutex> lk(T.mu);
    T.kernel = kernel;
    T.level = level;
}

void timer_read(int64_t *launches, double *total_ms) {
    Timer &T = timer();
    std::lock_guard<std::mutex> lk(T.mu);
    for (size_t k = 0; k < T.pending.size(); ++k) {
        auto &ev = T.pending[k];
        NAIR_HIP(hipEventSynchronize(ev.second));
        float ms = 0.0f;
        NAIR_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
        T.total_ms += ms;
        T.launches += T.pending_count[k];
        T.spare.push_back(ev);
    }
    T.pending.clear();
    T.pending_count.clear();
    if (launches) *launches = T.launches;
    if (total_ms) *total_ms = T.total_ms;
    T.launches = 0;
    T.total_ms = 0.0;
}

namespace {

// Small device-to-host reads go through one pinned staging buffer: a copy
// into pageable memory is staged and waited for one by one, a copy into
// pinned memory is a plain transfer the stream runs in order.
constexpr size_t kStageBytes = 64 * 1024;

struct Stage {
    std::mutex mu;
    char *buf = nullptr;
};

Stage &stage() {
    static Stage st;
    return st;
}

}  // namespace

void read_device(const ReadItem *items, size_t nitems, hipStream_t s) {
    size_t total = 0;
    for (size_t k = 0; k < nitems; ++k) total += (items[k].bytes + 7) & ~static_cast<size_t>(7);
    if (total > kStageBytes) {   // large reads copy directly
        for (size_t k = 0; k < nitems; ++k)
            if (items[k].bytes)
                NAIR_HIP(hipMemcpyAsync(items[k].host, items[k].dev, items[k].bytes, hipMemcpyDeviceToHost, s));
        NAIR_HIP(hipStreamSynchronize(s));
        return;
    }
    Stage &st = stage();
    std::lock_guard<std::mutex> lk(st.mu);
    if (!st.buf) NAIR_HIP(hipHostMalloc(reinterpret_cast<void **>(&st.buf), kStageBytes, hipHostMallocPortable));
    size_t off = 0;
    for (size_t k = 0; k < nitems; ++k) {
        if (items[k].bytes)
            NAIR_HIP(hipMemcpyAsync(st.buf + off, items[k].dev, items[k].bytes, hipMemcpyDeviceToHost, s));
        off += (items[k].bytes + 7) & ~static_cast<size_t>(7);
    }
    NAIR_HIP(hipStreamSynchronize(s));
    off = 0;
    for (size_t k = 0; k < nitems; ++k) {
        if (items[k].bytes) std::memcpy(items[k].host, st.buf + off, items[k].bytes);
        off += (items[k].bytes + 7) & ~static_cast<size_t>(7);
    }
}

void read_device(std::initializer_list<ReadItem> items, hipStream_t s) { read_device(items.begin(), items.size(), s); }

int read_int(const int *dptr, hipStream_t s) {
    int v = 0;
    read_device({{dptr, &v, sizeof(int)}}, s);
    return v;
}

void read_ints(const int *dptr, int *host, int n, hipStream_t s) {
    read_device({{dptr, host, sizeof(int) * static_cast<size_t>(n)}}, s);
}

}  // namespace nair
