// Device memory for the library: a per-device cache of freed blocks.
//
// A context's life allocates and frees tens of GB (integral blocks, batched
// transients, DIIS histories); mapping and unmapping that much memory costs
// tens of milliseconds per GB.  Freed blocks are therefore kept and handed to
// later requests of similar size, in this context or the next.  A block is
// cached only after a device synchronization, so no stream can still be using
// it when it is reused.  A failing allocation first returns the cache to the
// device and retries; lrcc_trim_memory returns it on request.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>

#include "common.h"
#include "devmem.h"

namespace lrcc {

namespace {

struct Block {
  size_t bytes;
  int device;
};

std::mutex g_mu;
std::unordered_map<void*, Block> g_live;          // pointer -> size, device
std::map<int, std::multimap<size_t, void*>> g_free;  // device -> (size -> pointer)
std::map<int, size_t> g_cached;                    // device -> cached bytes

size_t round_up(size_t b) {
  const size_t g = b > (size_t(1) << 20) ? (size_t(2) << 20) : 512;
  return (std::max<size_t>(b, 16) + g - 1) / g * g;
}

size_t cache_limit(int dev) {
  static std::map<int, size_t> lim;
  auto it = lim.find(dev);
  if (it != lim.end()) return it->second;
  size_t fr = 0, tot = 0;
  size_t l = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 2 : 0;
  lim[dev] = l;
  return l;
}

void trim_device(int dev) {  // caller holds g_mu
  auto& fl = g_free[dev];
  for (auto& kv : fl) (void)hipFree(kv.second);
  fl.clear();
  g_cached[dev] = 0;
}

}  // namespace

void* dev_alloc(size_t bytes) {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  const size_t b = round_up(bytes);
  std::lock_guard<std::mutex> g(g_mu);
  auto& fl = g_free[dev];
  auto it = fl.lower_bound(b);
  if (it != fl.end() && it->first <= b + b / 4 + (size_t(4) << 20)) {  // close enough in size
    void* p = it->second;
    g_live[p] = Block{it->first, dev};
    g_cached[dev] -= it->first;
    fl.erase(it);
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, b);
  if (e == hipErrorOutOfMemory && !fl.empty()) {
    (void)hipGetLastError();
    trim_device(dev);
    e = hipMalloc(&p, b);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? LRCC_E_NOMEM : LRCC_E_HIP,
                "hipMalloc(" + std::to_string(b) + " bytes): " + hipGetErrorString(e));
  }
  g_live[p] = Block{b, dev};
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) {  // not ours
    (void)hipFree(p);
    return;
  }
  const Block blk = it->second;
  g_live.erase(it);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != blk.device) (void)hipSetDevice(blk.device);
  // every stream on the device is done with the block before it can be reused
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && g_cached[blk.device] + blk.bytes <= cache_limit(blk.device)) {
    g_free[blk.device].emplace(blk.bytes, p);
    g_cached[blk.device] += blk.bytes;
  } else {
    (void)hipFree(p);
  }
  if (cur != blk.device) (void)hipSetDevice(cur);
}

void dev_trim() {
  std::lock_guard<std::mutex> g(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_free) {
    if (kv.second.empty()) continue;
    (void)hipSetDevice(kv.first);
    (void)hipDeviceSynchronize();
    trim_device(kv.first);
  }
  (void)hipSetDevice(cur);
}

size_t dev_cached_bytes() {
  std::lock_guard<std::mutex> g(g_mu);
  size_t s = 0;
  for (auto& kv : g_cached) s += kv.second;
  return s;
}

}  // namespace lrcc
