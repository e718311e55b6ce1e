// Integral-block assembly on the GPU from density-fitting factors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "common.h"

namespace lrcc {

// dst[p][q][r][s] = <pq||rs> for the classes in spec (e.g. "ovvo"); B on the
// device as FP64 complex [naux][nmo][nmo].
void build_block(const void* Bdev, int64_t naux, int64_t o, int64_t v, const std::string& spec, void* dst,
                 hipStream_t st);
// W[P(a,b)][P(e,f)] = <ab||ef>, a<b, e<f (FP64).
void build_packed_vvvv(const void* Bdev, int64_t naux, int64_t o, int64_t v, void* W, hipStream_t st);
// packed[x][y][P(e,f)] = full[x][y][e][f] for e < f (FP64).
void pack_last_pair(const void* full, int64_t n0, int64_t n1, int64_t n, void* packed, hipStream_t st);

}  // namespace lrcc
