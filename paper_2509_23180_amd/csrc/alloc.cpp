// Caching allocators for device memory and mapped host memory.
//
// Solving allocates a workspace per problem (Krylov basis, scratch, task
// records); a request stream or a benchmark loop would otherwise call
// hipMalloc / hipFree (and hipHostMalloc for the completion flags) for every
// solve.  Released blocks are kept per device, ordered by size, and a request
// takes the smallest kept block that holds it with at most a quarter (and at
// most 256 MiB) to spare: request sizes vary continuously on a served stream,
// so exact size classes were rarely reused, and every miss cost a hipMalloc
// and, once the cache was full, a hipFree, which waits for the whole device.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

#include "runtime.h"

namespace fds {

namespace {

// size classes: powers of two up to 1 MiB, then multiples of 2 MiB
size_t size_class(size_t bytes) {
  if (bytes <= (1u << 20)) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  const size_t g = 2u << 20;
  return (bytes + g - 1) / g * g;
}

size_t cache_limit() {
  static const size_t lim = [] {
    const char* e = std::getenv("FDS_CACHE_BYTES");
    // (a hipMalloc that runs out of memory gives the kept blocks back first;
    // allocations of other libraries in the process do not, hence the cap)
    return e ? (size_t)std::strtoull(e, nullptr, 10) : ((size_t)64 << 30);
  }();
  return lim;
}

struct DeviceCache {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> unused;   // unused blocks per device, by capacity
  std::map<void*, int> owner;     // block -> device
  size_t cached = 0;
  std::multimap<size_t, void*> host_free;   // mapped host blocks by size
  std::map<void*, void*> host_dev;          // host block -> device pointer
};

// Never destroyed: buffers owned by objects that outlive static destruction
// (plans freed during interpreter shutdown) still return here.
DeviceCache& cache() {
  static DeviceCache* c = new DeviceCache();
  return *c;
}

}  // namespace

void* device_cache_alloc(size_t bytes, size_t* capacity) {
  int dev = 0;
  FDS_HIP(hipGetDevice(&dev));
  const size_t c = size_class(bytes);
  DeviceCache& dc = cache();
  {
    std::lock_guard<std::mutex> lk(dc.mu);
    auto it = dc.unused.find(dev);
    if (it != dc.unused.end()) {
      const size_t slack = std::min(c / 4, (size_t)256 << 20);
      auto b = it->second.lower_bound(c);
      if (b != it->second.end() && b->first <= c + slack) {
        void* p = b->second;
        const size_t cap = b->first;
        it->second.erase(b);
        dc.cached -= cap;
        *capacity = cap;
        return p;
      }
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, c);
  if (e == hipErrorOutOfMemory) {
    // give the cached blocks of this device back and retry once
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(dc.mu);
    auto it = dc.unused.find(dev);
    if (it != dc.unused.end()) {
      for (auto& b : it->second) {
        (void)hipFree(b.second);
        dc.owner.erase(b.second);
        dc.cached -= b.first;
      }
      it->second.clear();
    }
    e = hipMalloc(&p, c);
  }
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? FDS_E_NOMEM : FDS_E_DEVICE,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> lk(dc.mu);
    dc.owner[p] = dev;
  }
  *capacity = c;
  return p;
}

void device_cache_free(void* p, size_t capacity) {
  if (!p) return;
  DeviceCache& dc = cache();
  std::lock_guard<std::mutex> lk(dc.mu);
  auto o = dc.owner.find(p);
  const int dev = o == dc.owner.end() ? 0 : o->second;
  if (dc.cached + capacity > cache_limit()) {
    (void)hipFree(p);
    if (o != dc.owner.end()) dc.owner.erase(o);
    return;
  }
  dc.unused[dev].emplace(capacity, p);
  dc.cached += capacity;
}

void* host_mapped_alloc(size_t bytes, void** device_ptr) {
  DeviceCache& dc = cache();
  {
    std::lock_guard<std::mutex> lk(dc.mu);
    auto it = dc.host_free.lower_bound(bytes);
    if (it != dc.host_free.end() && it->first < 2 * bytes + 4096) {
      void* p = it->second;
      dc.host_free.erase(it);
      *device_ptr = dc.host_dev[p];
      return p;
    }
  }
  void* p = nullptr;
  FDS_HIP(hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent));
  void* d = nullptr;
  FDS_HIP(hipHostGetDevicePointer(&d, p, 0));
  std::lock_guard<std::mutex> lk(dc.mu);
  dc.host_dev[p] = d;
  *device_ptr = d;
  return p;
}

void host_mapped_free(void* p, size_t bytes) {
  if (!p) return;
  DeviceCache& dc = cache();
  std::lock_guard<std::mutex> lk(dc.mu);
  dc.host_free.emplace(bytes, p);
}

}  // namespace fds
