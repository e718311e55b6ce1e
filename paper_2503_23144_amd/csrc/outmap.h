// Output address map of the GEMM epilogue (device and host).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lrcc {

// Output address map of a GEMM: element (m, n) of the product is stored at
// C + row(m) + col(n), with row(m) = sum_k digit_k(m) * mstr[k] over the
// mixed-radix digits of m (radices mdim[0..nm), the last varying fastest),
// and col(n) likewise.  This writes a product straight into a tensor whose
// index order interleaves the M and N indices (no permutation pass).
constexpr int kMapRank = 4;
struct OutMap {
  int nm = 1, nn = 1;
  int64_t mdim[kMapRank] = {1, 1, 1, 1}, mstr[kMapRank] = {0, 0, 0, 0};
  int64_t ndim[kMapRank] = {1, 1, 1, 1}, nstr[kMapRank] = {1, 0, 0, 0};
  static OutMap plain(int64_t ldc) {  // row-major with leading dimension ldc
    OutMap o;
    o.mstr[0] = ldc;
    o.mdim[0] = INT64_MAX;
    o.ndim[0] = INT64_MAX;
    return o;
  }
  __host__ __device__ static int64_t off(int64_t x, int nd, const int64_t* dim, const int64_t* str) {
    if (nd == 1) return x * str[0];
    int64_t o = 0;
    if (x < INT32_MAX) {  // 32-bit digit decode: far cheaper than 64-bit division on the GPU
      uint32_t y = (uint32_t)x;
      for (int k = nd - 1; k >= 0; --k) {
        const uint32_t dk = dim[k] > (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)dim[k];
        const uint32_t q = y / dk;
        o += (int64_t)(y - q * dk) * str[k];
        y = q;
      }
      return o;
    }
    for (int k = nd - 1; k >= 0; --k) {
      const int64_t q = x / dim[k];
      o += (x - q * dim[k]) * str[k];
      x = q;
    }
    return o;
  }
  __host__ __device__ int64_t row(int64_t m) const { return off(m, nm, mdim, mstr); }
  __host__ __device__ int64_t col(int64_t n) const { return off(n, nn, ndim, nstr); }
};

}  // namespace lrcc
