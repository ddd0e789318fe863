// c3x_common.hip -- errors, device memory cache, version strings.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "c3x_host.h"

namespace c3x {

static thread_local char g_err[512] = "";

c3x_status fail(c3x_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

c3x_status fail_hip(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(C3X_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(C3X_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err[0] = 0; }

// ---------------------------------------------------------------------------- memory cache

namespace {
struct Cache {
    std::mutex mu;
    // (device, size class) -> free blocks
    std::multimap<std::pair<int, size_t>, void *> free_;
    std::map<void *, std::pair<int, size_t>> live;
};
Cache &cache()
{
    static Cache *c = new Cache();  // never destroyed: outlives static teardown
    return *c;
}
size_t size_class(size_t n)
{
    if (n <= 4096) return 4096;
    if (n <= (1u << 20)) {
        size_t c = 4096;
        while (c < n) c <<= 1;
        return c;
    }
    // above 1 MiB: round up to 1/8 of the next power of two
    size_t p = 1u << 20;
    while (p < n) p <<= 1;
    size_t step = p >> 3;
    return (n + step - 1) / step * step;
}
}  // namespace

// Test hook: the k-th device allocation from the moment it is armed fails
// (C3X_DEBUG_FAIL_ALLOC=k arms it at the first allocation of the process;
// c3x_debug_fail_alloc(k) arms it at any time, 0 disarms).
static std::mutex g_fail_mu;
static int g_fail_left = -1;  // -1: not yet read from the environment

static int fail_alloc_countdown()
{
    std::lock_guard<std::mutex> g(g_fail_mu);
    if (g_fail_left < 0) {
        const char *e = getenv("C3X_DEBUG_FAIL_ALLOC");
        g_fail_left = e ? std::max(0, atoi(e)) : 0;
    }
    if (g_fail_left > 0 && --g_fail_left == 0) return 1;
    return 0;
}

void *dev_alloc(size_t bytes)
{
    if (fail_alloc_countdown()) return nullptr;
    int dev = 0;
    (void)hipGetDevice(&dev);
    size_t c = size_class(bytes);
    Cache &k = cache();
    {
        std::lock_guard<std::mutex> g(k.mu);
        auto it = k.free_.find({dev, c});
        if (it != k.free_.end()) {
            void *p = it->second;
            k.free_.erase(it);
            k.live[p] = {dev, c};
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
        // drop cached blocks of this device and retry once
        std::vector<void *> drop;
        {
            std::lock_guard<std::mutex> g(k.mu);
            for (auto it = k.free_.begin(); it != k.free_.end();) {
                if (it->first.first == dev) {
                    drop.push_back(it->second);
                    it = k.free_.erase(it);
                } else {
                    ++it;
                }
            }
        }
        for (void *q : drop) (void)hipFree(q);
        (void)hipGetLastError();
        if (hipMalloc(&p, c) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> g(k.mu);
    k.live[p] = {dev, c};
    return p;
}

// Pinned host staging for a call's small read-backs (counters, sizes): a
// pinned destination lets the copy go straight to host memory. One buffer
// per host thread, kept for the process; null if it cannot be had.
uint8_t *pinned_stage(size_t bytes)
{
    thread_local uint8_t *p = nullptr;
    thread_local size_t cap = 0;
    if (cap < bytes) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        if (hipHostMalloc((void **)&p, bytes) == hipSuccess) cap = bytes;
        else p = nullptr;
        (void)hipGetLastError();
    }
    return p;
}

void dev_free(void *p)
{
    if (!p) return;
    Cache &k = cache();
    std::lock_guard<std::mutex> g(k.mu);
    auto it = k.live.find(p);
    if (it == k.live.end()) return;
    k.free_.insert({it->second, p});
    k.live.erase(it);
}

}  // namespace c3x

extern "C" {

const char *c3x_last_error(void) { return c3x::g_err; }
const char *c3x_version(void) { return "c3x 0.1 (gfx950)"; }
int c3x_abi_version(void) { return C3X_ABI_VERSION; }

// Arms the allocation-failure hook: the k-th device allocation from now
// fails (0 disarms). Not part of the public header; used by tests.
void c3x_debug_fail_alloc(int k)
{
    std::lock_guard<std::mutex> g(c3x::g_fail_mu);
    c3x::g_fail_left = k > 0 ? k : 0;
}

// Number of device blocks handed out and not yet returned to the cache (not
// part of the public header; used by tests that check for leaks).
int c3x_debug_live_blocks(void)
{
    c3x::Cache &k = c3x::cache();
    std::lock_guard<std::mutex> g(k.mu);
    return (int)k.live.size();
}

}
