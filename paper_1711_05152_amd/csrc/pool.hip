// Caching device allocator behind every DevMem of the library.
//
// Plans and the steps of the sparse FFT allocate and free work areas of up to tens of GB.  Once
// device memory has been through a few such cycles, the driver's hipMalloc / hipFree of those sizes
// take 50 ms to seconds per call (measured: single hipMalloc calls of 2.4 s, hipFree calls of
// 50-110 ms, against a few ms of kernels per step).  Freed blocks are therefore kept mapped, per
// device, in size classes and handed out again:
//   * classes: powers of two up to 2 MiB; above, eight classes per octave rounded to 2 MiB (at most
//     12.5 % slack); a request takes the smallest cached block of its class or of a class at most
//     1.5 times larger (the sizes of consecutive sparse-FFT steps drift by tens of percent);
//   * a freed block may still be read or written by work queued before the free (hipFree waited
//     for the device, the cache does not), so it is "pending" until the next device-wide
//     synchronisation; the cache synchronises only when a request finds no fitting ready block but
//     a fitting pending one;
//   * idle bytes per device are capped (default a quarter of the device's memory, see
//     mr1l_memory_cache); a free beyond the cap goes back to the driver;
//   * a hipMalloc that fails for lack of memory empties the device's cache and is retried once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "runtime.h"

namespace mr1l {
namespace {

// size classes and the ready / pending bookkeeping live in host_logic.h (host::BlockCache)
using DevCache = host::BlockCache;
using host::size_class;

std::mutex g_mu;
std::vector<DevCache> g_cache;

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// caller holds g_mu
DevCache& cache_of(int dev) {
    if ((int)g_cache.size() <= dev) g_cache.resize(dev + 1);
    DevCache& C = g_cache[dev];
    if (C.limit < 0) {
        DeviceScope ds(dev);   // the memory size of this device, whichever is current
        size_t fr = 0, tot = 0;
        C.limit = hipMemGetInfo(&fr, &tot) == hipSuccess ? (int64_t)(tot / 4) : 0;
    }
    return C;
}

// caller holds g_mu; returns the bytes given back to the driver
size_t trim_locked(int dev) {
    DevCache& C = cache_of(dev);
    if (C.ready.empty() && C.pending.empty()) return 0;
    DeviceScope ds(dev);
    (void)hipDeviceSynchronize();
    return C.release_all([](void* p, size_t) { (void)hipFree(p); });
}

}  // namespace

hipError_t pool_alloc(void** p, size_t bytes, int* dev_out, size_t* block_out) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    *dev_out = dev;
    const size_t c = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DevCache& C = cache_of(dev);
        DevCache::Find r = C.take(c, p, block_out);
        if (r == DevCache::NEEDS_DRAIN) {
            // every pending block becomes reusable once the device has drained
            e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            C.drained();
            r = C.take(c, p, block_out);
        }
        if (r == DevCache::HIT) return hipSuccess;
    }
    e = hipMalloc(p, c);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_mu);
            trim_locked(dev);
        }
        e = hipMalloc(p, c);
    }
    if (e != hipSuccess) *p = nullptr;
    else *block_out = c;
    return e;
}

// c: the size of the block as handed out by pool_alloc
void pool_free(void* p, size_t c, int dev) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (cache_of(dev).give_back(p, c)) return;
    }
    // work queued before the free may still use the block
    DeviceScope ds(dev);
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
}

hipError_t TableStager::add(DevMem& dst, const void* src, size_t bytes) {
    hipError_t e = dst.alloc(bytes);
    if (e != hipSuccess || bytes == 0) return e;
    const size_t off = (host.size() + 255) & ~(size_t)255;
    host.resize(off + bytes);
    std::memcpy(host.data() + off, src, bytes);
    items.push_back(Item{&dst, off, bytes});
    return hipSuccess;
}

namespace {
constexpr int kCopySegs = 16;
struct CopyBatch {
    const char* src[kCopySegs];
    char* dst[kCopySegs];
    uint64_t bytes[kCopySegs];
};

// segment blockIdx.y of the batch; the blocks of a segment stride over it
__global__ __launch_bounds__(256) void k_copy_segments(CopyBatch b) {
    const int i = blockIdx.y;
    const char* s = b.src[i];
    char* d = b.dst[i];
    const uint64_t n = b.bytes[i];
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t head = 0;
    if ((((uintptr_t)s | (uintptr_t)d) & 15) == 0) {
        head = n / 16 * 16;
        for (uint64_t q = t; q < n / 16; q += step) ((uint4*)d)[q] = ((const uint4*)s)[q];
    }
    for (uint64_t q = head + t; q < n; q += step) d[q] = s[q];
}
}  // namespace

hipError_t copy_segments(const CopySeg* segs, int n, hipStream_t st) {
    for (int i0 = 0; i0 < n; i0 += kCopySegs) {
        CopyBatch b{};
        const int m = std::min(kCopySegs, n - i0);
        uint64_t most = 0;
        for (int i = 0; i < m; ++i) {
            b.src[i] = (const char*)segs[i0 + i].src;
            b.dst[i] = (char*)segs[i0 + i].dst;
            b.bytes[i] = segs[i0 + i].bytes;
            most = std::max(most, b.bytes[i]);
        }
        if (most == 0) continue;
        // one 16-byte move per thread and sweep; at most 64 blocks per segment
        const uint64_t blocks = std::min<uint64_t>(64, (most + 4095) / 4096);
        hipLaunchKernelGGL(k_copy_segments, dim3((unsigned)blocks, (unsigned)m), dim3(256), 0, st, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
// per thread and slot: the pinned buffer, and an event after the copy of the last flush that has
// not been waited for yet.  A kernel reads the pinned buffer, so it is allocated coherent and a
// buffer that has grown too small is retired, not freed (process lifetime).
thread_local void* t_pinned[2] = {nullptr, nullptr};
thread_local size_t t_cap[2] = {0, 0};
thread_local hipEvent_t t_done[2] = {nullptr, nullptr};
thread_local bool t_pending[2] = {false, false};
}  // namespace

hipError_t TableStager::settle(Slot slot) {
    if (!t_pending[slot]) return hipSuccess;
    t_pending[slot] = false;
    return hipEventSynchronize(t_done[slot]);
}

hipError_t TableStager::flush(hipStream_t st) {
    void** pinned = t_pinned;
    size_t* cap = t_cap;
    hipEvent_t* done = t_done;
    if (items.empty()) return hipSuccess;
    {
        hipError_t e = settle(slot);
        if (e != hipSuccess) return e;
    }
    if (!done[slot]) {
        hipError_t e = hipEventCreateWithFlags(&done[slot], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (cap[slot] < host.size()) {
        pinned[slot] = nullptr;
        cap[slot] = 0;
        const size_t want = std::max<size_t>(host.size(), (size_t)1 << 20);
        hipError_t e = hipHostMalloc(&pinned[slot], want, hipHostMallocCoherent | hipHostMallocPortable);
        if (e != hipSuccess) return e;
        cap[slot] = want;
    }
    std::memcpy(pinned[slot], host.data(), host.size());
    std::vector<CopySeg> segs;
    segs.reserve(items.size());
    for (const Item& it : items) segs.push_back(CopySeg{(const char*)pinned[slot] + it.off, it.dst->p, it.bytes});
    hipError_t e = copy_segments(segs.data(), (int)segs.size(), st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(done[slot], st);
    if (e != hipSuccess) return e;
    t_pending[slot] = true;
    items.clear();
    host.clear();
    return hipSuccess;
}

}  // namespace mr1l

using namespace mr1l;

extern "C" mr1l_status mr1l_memory_cache(int device, int64_t max_idle_bytes, int64_t* released) {
    clear_error();
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        set_error("invalid device for mr1l_memory_cache");
        return MR1L_ERR_ARG;
    }
    filter_cache_clear(device);   // its blocks return to the cache's idle lists first
    std::lock_guard<std::mutex> lk(g_mu);
    const size_t freed = trim_locked(device);
    if (max_idle_bytes >= 0) cache_of(device).limit = max_idle_bytes;
    if (released) *released = (int64_t)freed;
    return MR1L_OK;
}
