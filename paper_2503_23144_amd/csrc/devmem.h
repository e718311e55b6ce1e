// Cached device allocation (see devmem.hip).
#pragma once
#include <cstddef>

namespace lrcc {

void* dev_alloc(size_t bytes);  // on the current device; throws Error on failure
void dev_free(void* p);         // synchronizes the block's device, then caches or frees it
void dev_trim();                // return every cached block to its device
size_t dev_cached_bytes();

}  // namespace lrcc
