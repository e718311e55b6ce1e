// Integral-block assembly on the GPU from density-fitting factors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "common.h"

namespace lrcc {

// dst[p][q][r][s] = <pq||rs> for the classes in spec (e.g. "ovvo"); B on the
// device as FP64 complex [naux][nmo][nmo].  With pack_last (r and s of one
// class) dst is packed over r < s instead: dst[p][q][P(r,s)], formed in
// chunks of p so that the dense block never exists whole.
void build_block(const void* Bdev, int64_t naux, int64_t o, int64_t v, const std::string& spec, void* dst,
                 hipStream_t st, bool pack_last = false);
// W[P(a,b)][P(e,f)] = <ab||ef>, a<b, e<f (FP64).
void build_packed_vvvv(const void* Bdev, int64_t naux, int64_t o, int64_t v, void* W, hipStream_t st);
// Upper triangle of W in row blocks: block j holds rows [R(b_j),
// R(b_{j+1})) and columns [R(b_j), V) of W, R(b) = b(b-1)/2, row length
// V - R(b_j), at offs[j] complex elements into `dst` (precision TO; the rows
// are formed in FP64 and rounded once).  bnd: b_0 = 1 < ... < b_nb = v;
// bnd = {1, v}, offs = {0} gives the whole W.  Lvv: the virtual-virtual
// block of B, [naux][v][v] FP64.
template <typename TO>
void build_vvvv_triangle(const void* Lvv, int64_t naux, int64_t v, const std::vector<int64_t>& bnd,
                         const std::vector<int64_t>& offs, void* dst, hipStream_t st);
// packed[x][y][P(e,f)] = full[x][y][e][f] for e < f (FP64).
void pack_last_pair(const void* full, int64_t n0, int64_t n1, int64_t n, void* packed, hipStream_t st);

}  // namespace lrcc
