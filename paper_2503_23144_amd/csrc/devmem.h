// Device memory for the library (see devmem.hip).
#pragma once
#include <cstddef>
#include <map>
#include <unordered_map>

namespace lrcc {

// A caller-owned device buffer that one context sub-allocates from
// (first fit, 256-byte aligned, coalescing free list).
class Arena {
 public:
  Arena(void* base, size_t bytes);
  void* alloc(size_t bytes);  // throws Error(LRCC_E_NOMEM) when no free range fits
  bool owns(const void* p) const;
  void free(void* p);
  size_t free_bytes() const { return size_ - used_; }
  size_t largest_free() const;
  size_t peak() const { return peak_; }

 private:
  char* base_;
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;            // offset -> length
  std::unordered_map<const void*, size_t> live_;  // pointer -> length
};

// Allocations made while an ArenaScope is active on this thread come from
// its arena (the ABI entry points of a context with a workspace set one).
class ArenaScope {
 public:
  explicit ArenaScope(Arena* a);
  ~ArenaScope();

 private:
  Arena* prev_;
};
Arena* current_arena();

void* dev_alloc(size_t bytes);  // on the current device (or the current arena); throws Error on failure
void dev_free(void* p);         // arena blocks return to the arena; others are cached after a device sync
void dev_trim();                // return every cached block to its device
size_t dev_cached_bytes();
size_t dev_available();         // bytes a new allocation can get: the arena's free bytes, else free + cached

}  // namespace lrcc
