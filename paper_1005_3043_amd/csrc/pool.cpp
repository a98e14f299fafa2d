// Cache of device allocations.  A multigrid context on a large lattice holds
// some hundred GB in a few dozen buffers, and hipMalloc of buffers that size
// takes from 0.1 s to several seconds per call, growing as a process creates
// and destroys contexts.  Freed buffers are therefore kept per device and
// handed to the next request of the same rounded size (a context built with
// the same lattice and parameters gets all of its buffers back), up to a cap
// of cached bytes per device (60 % of the device's memory); beyond it the
// oldest cached blocks are freed.  A failed hipMalloc empties the device's
// cache and is tried once more.  mg_release_cached_memory frees the cache.
// Blocks are only cached after the device has finished its queued work.
#include <mutex>
#include <vector>

#include "solver.h"

namespace mg {

namespace {
constexpr size_t GRAIN = 2u << 20;  // blocks of 2 MiB or more are sized in 2 MiB steps
constexpr int MAX_DEV = 64;

struct Block {
  void *p;
  size_t bytes;
};
struct DevCache {
  std::vector<Block> free;  // oldest first
  size_t cached = 0, cap = 0;
};
std::mutex mu;
DevCache cache[MAX_DEV];

size_t rounded(size_t bytes) { return bytes >= GRAIN ? (bytes + GRAIN - 1) / GRAIN * GRAIN : bytes; }

void trim(DevCache &d, size_t keep) {
  while (d.cached > keep && !d.free.empty()) {
    (void)hipFree(d.free.front().p);
    d.cached -= d.free.front().bytes;
    d.free.erase(d.free.begin());
  }
}
}  // namespace

hipError_t pool_alloc(void **out, size_t bytes) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t n = rounded(bytes);
  if (dev >= 0 && dev < MAX_DEV) {
    std::lock_guard<std::mutex> lk(mu);
    DevCache &d = cache[dev];
    for (size_t i = d.free.size(); i-- > 0;) {
      if (d.free[i].bytes == n) {
        *out = d.free[i].p;
        d.cached -= n;
        d.free.erase(d.free.begin() + (long)i);
        return hipSuccess;
      }
    }
  }
  e = hipMalloc(out, n);
  if (e == hipErrorOutOfMemory && dev >= 0 && dev < MAX_DEV) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(mu);
      trim(cache[dev], 0);
    }
    e = hipMalloc(out, n);
  }
  return e;
}

void pool_free(void *p, size_t bytes) {
  if (!p) return;
  // As hipFree does, wait for the device's queued work, which may still use
  // the block, before it can be handed out again.
  (void)hipDeviceSynchronize();
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) {
    (void)hipFree(p);
    return;
  }
  const size_t n = rounded(bytes);
  std::lock_guard<std::mutex> lk(mu);
  DevCache &d = cache[dev];
  if (d.cap == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) d.cap = tot / 10 * 6;
    else d.cap = 1;
  }
  if (n > d.cap) {
    (void)hipFree(p);
    return;
  }
  d.free.push_back(Block{p, n});
  d.cached += n;
  trim(d, d.cap);
}

void pool_release(int dev) {
  if (dev < 0 || dev >= MAX_DEV) return;
  std::lock_guard<std::mutex> lk(mu);
  trim(cache[dev], 0);
}

size_t pool_cached(int dev) {
  if (dev < 0 || dev >= MAX_DEV) return 0;
  std::lock_guard<std::mutex> lk(mu);
  return cache[dev].cached;
}

}  // namespace mg

extern "C" int mg_release_cached_memory(size_t *released) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MG_EHIP;
  if (released) *released = mg::pool_cached(dev);
  mg::pool_release(dev);
  return MG_OK;
}
