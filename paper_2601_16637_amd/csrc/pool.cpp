// Caching device allocator behind every library-owned buffer (DevBuf) that is
// not carved from a serving region.
//
// A Davidson solve at 1e8 determinants holds some 30 GB of subspace vectors,
// staging and sigma workspace; handing those back to the driver after every
// solve and asking for them again at the next one makes each call pay for the
// driver's page mapping and clearing of tens of gigabytes, with a cost that
// varies from call to call.  Released blocks are therefore kept per device
// and handed out again to requests of about the same size (the successive
// solves of one workload ask for the same sizes every time).
//
// A block enters the cache only after the device has synchronised, exactly
// as hipFree would have waited, so no kernel still in flight can see its
// memory handed to another owner.  When hipMalloc fails, the cache is emptied
// and the allocation retried once.  sbd_release_cached_memory() returns
// every cached block to the driver.
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace sbd {
namespace {

constexpr size_t kSmallGrain = 256;
constexpr size_t kLargeGrain = 2u << 20;  // 2 MiB
constexpr size_t kLarge = 1u << 20;

size_t round_size(size_t n) {
    const size_t g = n >= kLarge ? kLargeGrain : kSmallGrain;
    return (n + g - 1) / g * g;
}

// A cached block of `size` serves a request of `n` (rounded) when it wastes
// at most a quarter of the request plus one large grain.
bool fits(size_t size, size_t n) { return size >= n && size - n <= n / 4 + kLargeGrain; }

struct DevicePool {
    std::multimap<size_t, void*> free_blocks;  // size -> pointer
    std::map<void*, size_t> live;              // pointer -> block size, handed out
    size_t cached = 0, in_use = 0;
};

struct Pool {
    std::mutex mu;
    std::map<int, DevicePool> dev;
};

Pool& pool() {
    static Pool* p = new Pool();  // never destroyed: the HIP runtime may be gone at exit
    return *p;
}

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) d = 0;
    return d;
}

// Free every cached block of device d (caller holds the lock; d is current).
void trim(DevicePool& P) {
    if (P.free_blocks.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& b : P.free_blocks) (void)hipFree(b.second);
    P.free_blocks.clear();
    P.cached = 0;
}

}  // namespace

hipError_t pool_alloc(size_t n, void** out) {
    *out = nullptr;
    if (n == 0) return hipSuccess;
    const size_t want = round_size(n);
    Pool& G = pool();
    std::lock_guard<std::mutex> g(G.mu);
    DevicePool& P = G.dev[current_device()];
    auto it = P.free_blocks.lower_bound(want);
    if (it != P.free_blocks.end() && fits(it->first, want)) {
        *out = it->second;
        P.live[it->second] = it->first;
        P.cached -= it->first;
        P.in_use += it->first;
        P.free_blocks.erase(it);
        return hipSuccess;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        trim(P);
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) return e;
    *out = p;
    P.live[p] = want;
    P.in_use += want;
    return hipSuccess;
}

void pool_free(void* p) {
    if (!p) return;
    Pool& G = pool();
    std::lock_guard<std::mutex> g(G.mu);
    for (auto& d : G.dev) {
        auto it = d.second.live.find(p);
        if (it == d.second.live.end()) continue;
        const size_t size = it->second;
        d.second.live.erase(it);
        d.second.in_use -= size;
        // as hipFree would: nothing in flight on the device may still use the block
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != d.first) (void)hipSetDevice(d.first);
        (void)hipDeviceSynchronize();
        if (cur != d.first) (void)hipSetDevice(cur);
        d.second.free_blocks.emplace(size, p);
        d.second.cached += size;
        return;
    }
    (void)hipFree(p);  // not from the pool (cannot happen through DevBuf)
}

void pool_stats(size_t* cached, size_t* in_use) {
    Pool& G = pool();
    std::lock_guard<std::mutex> g(G.mu);
    const auto it = G.dev.find(current_device());
    *cached = it == G.dev.end() ? 0 : it->second.cached;
    *in_use = it == G.dev.end() ? 0 : it->second.in_use;
}

void pool_release_cached() {
    Pool& G = pool();
    std::lock_guard<std::mutex> g(G.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& d : G.dev) {
        if (d.second.free_blocks.empty()) continue;
        (void)hipSetDevice(d.first);
        trim(d.second);
    }
    (void)hipSetDevice(cur);
}

}  // namespace sbd

extern "C" int sbd_release_cached_memory(void) {
    sbd::pool_release_cached();
    return SBD_OK;
}

extern "C" int sbd_memory_stats(size_t* cached_bytes, size_t* in_use_bytes) {
    if (!cached_bytes || !in_use_bytes) return sbd::fail(SBD_ERR_ARG, "null argument");
    sbd::pool_stats(cached_bytes, in_use_bytes);
    return SBD_OK;
}
