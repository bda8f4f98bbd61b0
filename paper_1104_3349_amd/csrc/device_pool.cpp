// Caching device allocator for the library's buffers (DevBuf).  A released
// block goes to its device's pool instead of hipFree (which synchronises the
// device and costs tens of microseconds); an allocation takes the smallest
// pooled block of at least the requested size and at most twice it.  A block
// is handed out again only after a device synchronisation that followed its
// release (pool_sync, called at the start of the allocating entry points),
// so no kernel queued before the release can still be using it, whatever
// stream it ran on.  Cached bytes per device are capped (a quarter of the
// device memory); beyond the cap a release goes to hipFree.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "precond.h"

namespace addns {
namespace {

struct Block {
  void* p;
  size_t cap;
};

struct DevicePool {
  std::multimap<size_t, void*> ready;  // capacity -> block, reusable
  std::vector<Block> pending;          // released since the last synchronisation
  size_t cached = 0;                   // bytes in ready + pending
  size_t limit = 0;
};

// Never destroyed: a handle released during process exit, after the static
// destructors have run, still finds its pool.
struct State {
  std::mutex mu;
  std::map<int, DevicePool> pools;
};
State& st() {
  static State* s = new State();
  return *s;
}

DevicePool& pool_of(int dev) {
  DevicePool& d = st().pools[dev];
  if (d.limit == 0) {
    size_t total = 0;
    if (hipDeviceTotalMem(&total, dev) != hipSuccess || total == 0) total = size_t(16) << 30;
    d.limit = total / 4;
  }
  return d;
}

}  // namespace

void* pool_alloc(size_t n, size_t* cap, int* dev) {
  ADDNS_HIP(hipGetDevice(dev));
  {
    std::lock_guard<std::mutex> lk(st().mu);
    DevicePool& d = pool_of(*dev);
    auto it = d.ready.lower_bound(n);
    if (it != d.ready.end() && it->first <= 2 * n) {
      void* p = it->second;
      *cap = it->first;
      d.cached -= it->first;
      d.ready.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pool_trim();  // give the cached blocks back and try once more
    ADDNS_HIP(hipMalloc(&p, n));
  }
  *cap = n;
  return p;
}

void pool_free(void* p, size_t cap, int dev) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(st().mu);
    DevicePool& d = pool_of(dev);
    if (d.cached + cap <= d.limit) {
      d.pending.push_back(Block{p, cap});
      d.cached += cap;
      return;
    }
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != dev) (void)hipSetDevice(dev);
  (void)hipFree(p);
  if (cur != dev) (void)hipSetDevice(cur);
}

void pool_sync() {
  int dev = 0;
  ADDNS_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(st().mu);
    if (pool_of(dev).pending.empty()) return;
  }
  ADDNS_HIP(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(st().mu);
  DevicePool& d = pool_of(dev);
  for (const Block& b : d.pending) d.ready.emplace(b.cap, b.p);
  d.pending.clear();
}

size_t pool_trim() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  std::lock_guard<std::mutex> lk(st().mu);
  size_t freed = 0;
  for (auto& kv : st().pools) {
    DevicePool& d = kv.second;
    if (d.ready.empty() && d.pending.empty()) continue;
    (void)hipSetDevice(kv.first);
    (void)hipDeviceSynchronize();
    for (auto& b : d.ready) (void)hipFree(b.second);
    for (const Block& b : d.pending) (void)hipFree(b.p);
    freed += d.cached;
    d.ready.clear();
    d.pending.clear();
    d.cached = 0;
  }
  (void)hipSetDevice(cur);
  return freed;
}

}  // namespace addns
