// Device memory cache of libmfs.
//
// A solve holds tens of GB for a few hundred milliseconds (the stored near
// field, the Krylov bases, the periodizer's arenas) and a serving loop or a
// benchmark repeats that many times.  Returning such blocks to the driver
// and asking for them again costs far more than the work itself on some
// steps (the driver clears and maps freed device memory before it hands it
// out again), so every buffer of at least kPoolMin bytes goes through a
// per-device cache: a released block is kept and handed to the next request
// of about its size.  Smaller buffers go straight to hipMalloc / hipFree.
//
// Ordering.  hipFree waits for the device to finish the work queued before
// it, which is what makes releasing a buffer that a queued kernel still
// reads safe.  A cached block keeps that rule: its release synchronises the
// device before the block becomes available again, so a later request on
// any stream never sees it while earlier work still uses it.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mfs {

namespace {

constexpr size_t kPoolMin = (size_t)1 << 20;     // smaller blocks are not cached
constexpr size_t kPoolGrain = (size_t)2 << 20;   // cached sizes are multiples of this

struct Pool {
  std::mutex mu;
  std::multimap<size_t, void *> idle;   // size -> block, not in use
  size_t idle_bytes = 0;
  size_t cap = 0;                       // largest idle total kept (0: not yet read)
  size_t in_use = 0, peak = 0;          // bytes of live DevBufs (cached blocks at their block size)
};

void note_alloc(Pool &p, size_t n) {   // p.mu held
  p.in_use += n;
  if (p.in_use > p.peak) p.peak = p.in_use;
}

// One pool per device, created on first use and never destroyed: blocks
// still cached at process exit are returned by the driver with the process.
Pool &pool_of(int dev) {
  static std::mutex mu;
  static std::vector<Pool *> pools;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)pools.size() <= dev) pools.resize(dev + 1, nullptr);
  if (!pools[dev]) pools[dev] = new Pool;
  return *pools[dev];
}

int current_device() {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  return dev;
}

// Free idle blocks of p (largest first) until at most `keep` bytes stay idle.
// Called with p.mu held.
void trim_locked(Pool &p, size_t keep) {
  while (p.idle_bytes > keep && !p.idle.empty()) {
    auto it = std::prev(p.idle.end());
    (void)hipFree(it->second);
    p.idle_bytes -= it->first;
    p.idle.erase(it);
  }
}

}  // namespace

void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) return;
  dev = current_device();
  Pool &pl = pool_of(dev);
  if (n < kPoolMin) {
    if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{MFS_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
    cached = 0;
    std::lock_guard<std::mutex> lk(pl.mu);
    note_alloc(pl, n);
    return;
  }
  const size_t want = (n + kPoolGrain - 1) / kPoolGrain * kPoolGrain;
  {
    std::lock_guard<std::mutex> lk(pl.mu);
    // the smallest idle block that fits, if it wastes at most 1/8 of it
    auto it = pl.idle.lower_bound(want);
    if (it != pl.idle.end() && it->first - want <= want / 8) {
      p = it->second;
      cached = it->first;
      pl.idle_bytes -= it->first;
      pl.idle.erase(it);
      bytes = n;
      note_alloc(pl, cached);
      return;
    }
  }
  void *q = nullptr;
  if (hipMalloc(&q, want) != hipSuccess) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(pl.mu);
      trim_locked(pl, 0);
    }
    if (hipMalloc(&q, want) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{MFS_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed"};
    }
  }
  p = q;
  cached = want;
  bytes = n;
  std::lock_guard<std::mutex> lk(pl.mu);
  note_alloc(pl, want);
}

void DevBuf::release() {
  if (!p) return;
  if (!cached) {
    (void)hipFree(p);
    Pool &pl = pool_of(dev);
    std::lock_guard<std::mutex> lk(pl.mu);
    pl.in_use -= bytes;
  } else {
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
    // the rule hipFree keeps: nothing queued before this point may still
    // be using the block when it is handed out again
    (void)hipDeviceSynchronize();
    Pool &pl = pool_of(dev);
    {
      std::lock_guard<std::mutex> lk(pl.mu);
      if (pl.cap == 0) {
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        pl.cap = tot / 2;   // keep at most half of the device idle in the cache
      }
      pl.idle.emplace(cached, p);
      pl.idle_bytes += cached;
      pl.in_use -= cached;
      trim_locked(pl, pl.cap);
    }
    if (prev != dev) (void)hipSetDevice(prev);
  }
  p = nullptr;
  bytes = 0;
  cached = 0;
}

size_t pool_idle_bytes(int dev) {
  Pool &pl = pool_of(dev);
  std::lock_guard<std::mutex> lk(pl.mu);
  return pl.idle_bytes;
}

void pool_trim(int dev) {
  Pool &pl = pool_of(dev);
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != dev) (void)hipSetDevice(dev);
  {
    std::lock_guard<std::mutex> lk(pl.mu);
    trim_locked(pl, 0);
  }
  if (prev != dev) (void)hipSetDevice(prev);
}

void pool_stats(int dev, size_t *in_use, size_t *peak, size_t *idle) {
  Pool &pl = pool_of(dev);
  std::lock_guard<std::mutex> lk(pl.mu);
  if (in_use) *in_use = pl.in_use;
  if (peak) *peak = pl.peak;
  if (idle) *idle = pl.idle_bytes;
}

void pool_reset_peak(int dev) {
  Pool &pl = pool_of(dev);
  std::lock_guard<std::mutex> lk(pl.mu);
  pl.peak = pl.in_use;
}

size_t device_free_bytes() {
  size_t fr = 0, tot = 0;
  HIP_CHECK(hipMemGetInfo(&fr, &tot));
  return fr + pool_idle_bytes(current_device());
}

}  // namespace mfs
