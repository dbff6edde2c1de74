// Caching device-memory pool with an optional HBM budget.
//
// Blocks are rounded to size classes (powers of two up to 1 MiB, then whole
// MiB) and kept on a free list after release, so repeated create/destroy
// cycles and the server's per-request buffers do not pay for hipMalloc.  The
// budget (bytes; 0 = unlimited, initialised from the environment variable
// OSC_HBM_BUDGET) bounds the bytes handed out at any time.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "osc_internal.h"

namespace osc {
namespace {

struct Block {
    size_t bytes;
    int device;
};

std::mutex g_mu;
std::multimap<size_t, std::pair<void *, int>> g_free;   // size -> (ptr, device)
std::unordered_map<void *, Block> g_live;
size_t g_in_use = 0;
size_t g_budget = [] {
    const char *e = std::getenv("OSC_HBM_BUDGET");
    return e ? (size_t)std::strtoull(e, nullptr, 10) : (size_t)0;
}();

size_t size_class(size_t b) {
    if (b == 0) b = 1;
    const size_t mib = size_t(1) << 20;
    if (b >= mib) return (b + mib - 1) / mib * mib;
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}

void trim_locked() {
    for (auto &kv : g_free) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(kv.second.second);
        (void)hipFree(kv.second.first);
        (void)hipSetDevice(cur);
    }
    g_free.clear();
}

}  // namespace

size_t pool_size_class(size_t bytes) { return size_class(bytes); }

void *pool_alloc(size_t bytes) {
    const size_t c = size_class(bytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_budget && g_in_use + c > g_budget) return nullptr;
    for (auto it = g_free.lower_bound(c); it != g_free.end() && it->first < 2 * c; ++it) {
        if (it->second.second != dev) continue;
        void *p = it->second.first;
        const size_t got = it->first;
        g_free.erase(it);
        g_live[p] = Block{got, dev};
        g_in_use += got;
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        trim_locked();
        if (hipMalloc(&p, c) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    g_live[p] = Block{c, dev};
    g_in_use += c;
    return p;
}

void pool_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    g_in_use -= it->second.bytes;
    g_free.emplace(it->second.bytes, std::make_pair(p, it->second.device));
    g_live.erase(it);
}

size_t pool_in_use() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_in_use;
}

size_t pool_budget() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_budget;
}

void pool_set_budget(size_t bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_budget = bytes;
}

void pool_trim() {
    std::lock_guard<std::mutex> lk(g_mu);
    trim_locked();
}

}  // namespace osc
