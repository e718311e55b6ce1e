// Device memory for the library: a per-device cache of freed blocks.
//
// A context's life allocates and frees tens of GB (integral blocks, batched
// transients, DIIS histories); mapping and unmapping that much memory costs
// tens of milliseconds per GB.  Freed blocks are therefore kept and handed to
// later requests of similar size, in this context or the next.  A block is
// cached only after a device synchronization, so no stream can still be using
// it when it is reused.  A failing allocation first returns the cache to the
// device and retries; lrcc_trim_memory returns it on request.
//
// A context given a caller-owned workspace (lrcc_set_workspace) takes all
// its memory from that buffer instead, through an Arena active on the
// calling thread for the duration of each of its entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
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

thread_local Arena* t_arena = nullptr;

}  // namespace

// ---------------------------------------------------------------- arena
Arena::Arena(void* base, size_t bytes) : base_((char*)base), size_(bytes) {
  // the usable range starts at the first 256-byte boundary
  const size_t skew = (256 - ((uintptr_t)base_ & 255)) & 255;
  if (bytes > skew) free_[skew] = bytes - skew;
  used_ = std::min(skew, bytes);
}

void* Arena::alloc(size_t bytes) {
  const size_t b = (std::max<size_t>(bytes, 16) + 255) / 256 * 256;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < b) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > b) free_[off + b] = len - b;
    void* p = base_ + off;
    live_[p] = b;
    used_ += b;
    peak_ = std::max(peak_, used_);
    return p;
  }
  throw Error(LRCC_E_NOMEM, "workspace too small: " + std::to_string(b) + " bytes requested, " +
                                std::to_string(largest_free()) + " in the largest free range");
}

bool Arena::owns(const void* p) const { return p >= base_ && p < base_ + size_; }

void Arena::free(void* p) {
  auto it = live_.find(p);
  if (it == live_.end()) return;
  size_t off = (char*)p - base_, len = it->second;
  live_.erase(it);
  used_ -= len;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && off + len == nx->first) {  // merge with the next range
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // merge with the previous range
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      pv->second += len;
      return;
    }
  }
  free_[off] = len;
}

size_t Arena::largest_free() const {
  size_t m = 0;
  for (auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

ArenaScope::ArenaScope(Arena* a) : prev_(t_arena) { t_arena = a; }
ArenaScope::~ArenaScope() { t_arena = prev_; }
Arena* current_arena() { return t_arena; }

// ---------------------------------------------------------------- device memory
void* dev_alloc(size_t bytes) {
  if (t_arena) return t_arena->alloc(bytes);
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
  if (t_arena && t_arena->owns(p)) {  // stream-ordered reuse within the context
    t_arena->free(p);
    return;
  }
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

size_t dev_available() {
  if (t_arena) return t_arena->free_bytes();
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
  return fr + dev_cached_bytes();
}

size_t dev_cached_bytes() {
  std::lock_guard<std::mutex> g(g_mu);
  size_t s = 0;
  for (auto& kv : g_cached) s += kv.second;
  return s;
}

}  // namespace lrcc
