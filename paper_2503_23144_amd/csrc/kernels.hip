// Streaming kernels of the lrcc runtime (gfx950): index permutation, pair
// (un)packing with antisymmetry, reductions with wavefront shuffles, solver
// updates and integral-block assembly.  These are HBM-bound; each reads and
// writes every element once, with the output linear index driving the
// thread mapping so that stores are coalesced.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <algorithm>

#include <cmath>

#include "common.h"
#include "kernels.h"

namespace lrcc {

template <typename T>
struct cplx2;
template <>
struct cplx2<double> {
  using type = double2;
};
template <>
struct cplx2<float> {
  using type = float2;
};

static inline unsigned nblocks(int64_t total, int threads = 256, int64_t cap = 1 << 20) {
  int64_t b = (total + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

#define LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// ---------------------------------------------------------------- permute
template <typename T, typename I>
__global__ void __launch_bounds__(256) permute_kernel(const typename cplx2<T>::type* __restrict__ in,
                                                      typename cplx2<T>::type* __restrict__ out, PermDesc d,
                                                      I total, T are, T aim, T bre, T bim, int use_beta) {
  for (I lin = (I)blockIdx.x * blockDim.x + threadIdx.x; lin < total; lin += (I)gridDim.x * blockDim.x) {
    I rem = lin;
    int64_t off = 0;
    for (int k = d.rank - 1; k >= 0; --k) {
      I dk = (I)d.dims[k];
      I q = rem / dk;
      off += (int64_t)(rem - q * dk) * d.istride[k];
      rem = q;
    }
    auto x = in[off];
    T re = are * x.x - aim * x.y;
    T im = are * x.y + aim * x.x;
    if (use_beta) {
      auto y = out[lin];
      re += bre * y.x - bim * y.y;
      im += bre * y.y + bim * y.x;
    }
    out[lin] = {re, im};
  }
}

// Permutations whose input-contiguous dimension p is not the output's last
// one: the naive kernel above then reads with a stride between neighbouring
// lanes.  Here each 32 x 32 tile over (dim p, last dim) is read with lanes
// along p (contiguous in the input), staged in LDS, and written with lanes
// along the last dim (contiguous in the output).  The remaining dimensions
// index the tiles; istride[p] must be 1.
template <typename T>
__global__ void __launch_bounds__(256) transpose_kernel(const typename cplx2<T>::type* __restrict__ in,
                                                        typename cplx2<T>::type* __restrict__ out, PermDesc d,
                                                        int p, int64_t ntiles, int64_t tp, int64_t tl, T are, T aim,
                                                        T bre, T bim, int use_beta) {
  using C = typename cplx2<T>::type;
  __shared__ C tile[32][33];
  const int L = d.rank - 1;
  const int64_t np = d.dims[p], nl = d.dims[L], sl = d.istride[L];
  int64_t ostr[kMaxRank];
  ostr[L] = 1;
  for (int k = L - 1; k >= 0; --k) ostr[k] = ostr[k + 1] * d.dims[k + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int64_t rest = t / (tp * tl);
    const int64_t rem = t - rest * (tp * tl);
    const int64_t ip0 = (rem / tl) * 32, il0 = (rem % tl) * 32;
    int64_t ib = 0, ob = 0;
    for (int k = L - 1; k >= 0; --k) {
      if (k == p) continue;
      const int64_t q = rest / d.dims[k];
      const int64_t dk = rest - q * d.dims[k];
      rest = q;
      ib += dk * d.istride[k];
      ob += dk * ostr[k];
    }
    for (int j = ty; j < 32; j += 8) {
      const int64_t ip = ip0 + tx, il = il0 + j;
      if (ip < np && il < nl) tile[j][tx] = in[ib + ip + il * sl];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
      const int64_t ip = ip0 + j, il = il0 + tx;
      if (ip < np && il < nl) {
        const C x = tile[tx][j];
        T re = are * x.x - aim * x.y;
        T im = are * x.y + aim * x.x;
        C* o = out + ob + ip * ostr[p] + il;
        if (use_beta) {
          const C y = *o;
          re += bre * y.x - bim * y.y;
          im += bre * y.y + bim * y.x;
        }
        *o = C{re, im};
      }
    }
    __syncthreads();
  }
}

template <typename T>
void launch_permute(const void* in, void* out, const PermDesc& d, double are, double aim, double bre, double bim,
                    hipStream_t st) {
  int64_t total = 1;
  for (int k = 0; k < d.rank; ++k) total *= d.dims[k];
  if (total == 0) return;
  using C = typename cplx2<T>::type;
  int ub = (bre != 0.0 || bim != 0.0) ? 1 : 0;
  static const bool trace = [] {
    const char* e = std::getenv("LRCC_TRACE_PERMUTE");
    return e && e[0] == '1';
  }();
  if (trace) {  // LRCC_TRACE_PERMUTE=1: shape of every launch on stderr
    fprintf(stderr, "[lrcc permute] %s beta=%d total=%lld dims", sizeof(T) == 8 ? "c128" : "c64", ub,
            (long long)total);
    for (int k = 0; k < d.rank; ++k) fprintf(stderr, " %lld", (long long)d.dims[k]);
    fprintf(stderr, " istride");
    for (int k = 0; k < d.rank; ++k) fprintf(stderr, " %lld", (long long)d.istride[k]);
    fprintf(stderr, "\n");
  }
  // tiled transpose when the input-contiguous dimension is not the last one
  int p = -1;
  for (int k = 0; k < d.rank; ++k)
    if (d.istride[k] == 1 && d.dims[k] > 1) p = k;
  const int L = d.rank - 1;
  if (p >= 0 && p != L && d.dims[L] > 1) {
    const int64_t tp = (d.dims[p] + 31) / 32, tl = (d.dims[L] + 31) / 32;
    const int64_t ntiles = total / (d.dims[p] * d.dims[L]) * tp * tl;
    const unsigned blocks = (unsigned)std::min<int64_t>(ntiles, int64_t(1) << 20);
    hipLaunchKernelGGL(transpose_kernel<T>, dim3(blocks), dim3(256), 0, st, (const C*)in, (C*)out, d, p, ntiles,
                       tp, tl, (T)are, (T)aim, (T)bre, (T)bim, ub);
    LAUNCH_CHECK();
    return;
  }
  if (total < (int64_t(1) << 31))
    hipLaunchKernelGGL((permute_kernel<T, uint32_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)in,
                       (C*)out, d, (uint32_t)total, (T)are, (T)aim, (T)bre, (T)bim, ub);
  else
    hipLaunchKernelGGL((permute_kernel<T, int64_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)in,
                       (C*)out, d, total, (T)are, (T)aim, (T)bre, (T)bim, ub);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- pair index
__device__ inline void decode_pair(int64_t P, int64_t& p, int64_t& q) {
  int64_t qq = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)P)) * 0.5);
  while (qq * (qq - 1) / 2 > P) --qq;
  while ((qq + 1) * qq / 2 <= P) ++qq;
  q = qq;
  p = P - qq * (qq - 1) / 2;
}

// ---------------------------------------------------------------- pack
// I: index type of the element decode (uint32_t when every size fits; the
// 64-bit divisions otherwise dominate these memory-bound kernels).
template <typename T, typename I>
__global__ void __launch_bounds__(256) pack_kernel(const typename cplx2<T>::type* __restrict__ full,
                                                   typename cplx2<T>::type* __restrict__ packed, PackDesc d,
                                                   I total, T are, T aim, int acc) {
  for (I lin = (I)blockIdx.x * blockDim.x + threadIdx.x; lin < total; lin += (I)gridDim.x * blockDim.x) {
    I rem = lin;
    int64_t off = 0;
    int np = 0;
    int64_t o1[2] = {0, 0}, o2[2] = {0, 0};
    int md[2] = {0, 0};
    for (int k = d.rank - 1; k >= 0; --k) {
      const I dk = (I)d.dims[k];
      const I q = rem / dk;
      const int64_t i = (int64_t)(rem - q * dk);
      rem = q;
      if (d.pair[k]) {
        int64_t a, b;
        decode_pair(i, a, b);
        o1[np] = a * d.fp[k] + b * d.fq[k];
        o2[np] = b * d.fp[k] + a * d.fq[k];
        md[np] = d.mode[k];
        ++np;
      } else {
        off += i * d.fstride[k];
      }
    }
    T re = 0, im = 0;
    for (int mask = 0; mask < (1 << np); ++mask) {
      bool ok = true;
      int64_t o = off;
      T s = 1;
      for (int j = 0; j < np; ++j) {
        if (mask & (1 << j)) {
          if (!md[j]) ok = false;
          o += o2[j];
          s = -s;
        } else {
          o += o1[j];
        }
      }
      if (!ok) continue;
      auto x = full[o];
      re += s * x.x;
      im += s * x.y;
    }
    T rr = are * re - aim * im, ii = are * im + aim * re;
    if (acc) {
      auto y = packed[lin];
      rr += y.x;
      ii += y.y;
    }
    packed[lin] = {rr, ii};
  }
}

template <typename T, typename I>
__global__ void __launch_bounds__(256) unpack_kernel(const typename cplx2<T>::type* __restrict__ packed,
                                                     typename cplx2<T>::type* __restrict__ full, PackDesc d,
                                                     I total, T are, T aim, int acc) {
  for (I lin = (I)blockIdx.x * blockDim.x + threadIdx.x; lin < total; lin += (I)gridDim.x * blockDim.x) {
    I rem = lin;
    int64_t pidx[kMaxRank], qidx[kMaxRank], plain[kMaxRank];
    for (int k = d.frank - 1; k >= 0; --k) {
      const I dk = (I)d.fdims[k];
      const I q = rem / dk;
      const int64_t i = (int64_t)(rem - q * dk);
      rem = q;
      int j = d.fmap[k];
      if (d.fsec[k] < 0)
        plain[j] = i;
      else if (d.fsec[k] == 0)
        pidx[j] = i;
      else
        qidx[j] = i;
    }
    int64_t off = 0;
    T s = 1;
    bool zero = false;
    for (int j = 0; j < d.rank; ++j) {
      if (!d.pair[j]) {
        off += plain[j] * d.pstride[j];
        continue;
      }
      int64_t p = pidx[j], q = qidx[j];
      if (p == q) {
        zero = true;
      } else if (p < q) {
        off += (q * (q - 1) / 2 + p) * d.pstride[j];
      } else if (d.mode[j]) {
        off += (p * (p - 1) / 2 + q) * d.pstride[j];
        s = -s;
      } else {
        zero = true;
      }
    }
    T re = 0, im = 0;
    if (!zero) {
      auto x = packed[off];
      re = s * (are * x.x - aim * x.y);
      im = s * (are * x.y + aim * x.x);
    }
    if (acc) {
      auto y = full[lin];
      re += y.x;
      im += y.y;
    }
    full[lin] = {re, im};
  }
}

// Unpack of the common layout: the packed tensor's last dim is a pair
// (a < b) whose two full dims are the full tensor's last two, an n x n
// row-major block per outer row.  A workgroup (32 x 8 threads) writes up to
// TPB consecutive 32 x 32 tiles of one outer row's block.  The packed entries
// P(a,b) = b(b-1)/2 + a run along a, so a tile's a < b entries are staged in
// LDS as [b][a]: the packed reads (along a) and the full writes (along b) are
// both coalesced.  The a > b entries, -P(b,a) when the pair is antisymmetric
// (mode 1), run along b and are read directly; the diagonal and, for mode 0,
// the a > b part are 0.
constexpr int UT = 32, TPB = 4, PTPB = 1;  // tile edge; tiles per workgroup (unpack, pack)

template <typename T, typename I>
__global__ void __launch_bounds__(256) unpack_tail_pair_kernel(const typename cplx2<T>::type* __restrict__ packed,
                                                               typename cplx2<T>::type* __restrict__ full,
                                                               PackDesc d, I rows, int n, int nt, T are, T aim,
                                                               int acc) {
  using C = typename cplx2<T>::type;
  constexpr int NY = 256 / UT;
  __shared__ C tile[UT][UT + 1];
  const int in = d.rank - 1;
  const int mode = d.mode[in];
  const int tx = threadIdx.x % UT, ty = threadIdx.x / UT;
  const int tiles = nt * nt, chunks = (tiles + TPB - 1) / TPB;
  const int64_t nblk = (int64_t)rows * chunks;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const I r = (I)(blk / chunks);
    const int c = (int)(blk % chunks);
    // packed offset and sign of outer row r, in one pass over the outer full
    // dims (the second index of a pair is the dim right after its first)
    I rem = r;
    int64_t off = 0, qsec = 0;
    T s = 1;
    bool zero = false;
    for (int k = d.frank - 3; k >= 0; --k) {
      const I dk = (I)d.fdims[k];
      const I q = rem / dk;
      const int64_t i = (int64_t)(rem - q * dk);
      rem = q;
      const int j = d.fmap[k];
      if (d.fsec[k] < 0) {
        off += i * d.pstride[j];
      } else if (d.fsec[k] == 1) {
        qsec = i;
      } else if (i == qsec) {
        zero = true;
      } else if (i < qsec) {
        off += (qsec * (qsec - 1) / 2 + i) * d.pstride[j];
      } else if (d.mode[j]) {
        off += (i * (i - 1) / 2 + qsec) * d.pstride[j];
        s = -s;
      } else {
        zero = true;
      }
    }
    const C* prow = packed + off;
    C* frow = full + (int64_t)r * n * n;
    const int t1 = min(tiles, (c + 1) * TPB);
    for (int t = c * TPB; t < t1; ++t) {
      const int ta = t / nt, tb = t % nt;
      const int a0 = ta * UT, b0 = tb * UT;
      if (!zero && ta <= tb) {
        for (int y = ty; y < UT; y += NY) {
          const int b = b0 + y, a = a0 + tx;
          if (b < n && a < b) tile[y][tx] = prow[(int64_t)b * (b - 1) / 2 + a];
        }
      }
      __syncthreads();
      for (int y = ty; y < UT; y += NY) {
        const int a = a0 + y, b = b0 + tx;
        if (a < n && b < n) {
          T re = 0, im = 0;
          if (!zero && a != b && (a < b || mode)) {
            C x;
            T sg = s;
            if (a < b) {
              x = tile[b - b0][a - a0];
            } else {
              x = prow[(int64_t)a * (a - 1) / 2 + b];
              sg = -sg;
            }
            re = sg * (are * x.x - aim * x.y);
            im = sg * (are * x.y + aim * x.x);
          }
          C* f = frow + (int64_t)a * n + b;
          if (acc) {
            const C yv = *f;
            re += yv.x;
            im += yv.y;
          }
          *f = C{re, im};
        }
      }
      __syncthreads();  // the tile is rewritten for the next one
    }
  }
}

// Pack of the same layout (the last packed dim a pair (a < b) over the full
// tensor's last two dims, fp = n, fq = 1; at most two outer pairs).  A
// workgroup forms the packed entries of up to PTPB tiles ta <= tb of the n x n
// block of one outer packed row.  For each order of the outer pairs (summed
// in the order of pack_kernel), full[a][b] is staged in LDS as [a][b] (read
// along b) and read back along a, and -full[b][a] (mode 1) is read along a
// directly, so the packed writes P(a,b) = b(b-1)/2 + a (along a) and every
// read are coalesced.
template <typename T, typename I>
__global__ void __launch_bounds__(256) pack_tail_pair_kernel(const typename cplx2<T>::type* __restrict__ full,
                                                             typename cplx2<T>::type* __restrict__ packed,
                                                             PackDesc d, I rows, int n, int nt, T are, T aim,
                                                             int acc) {
  using C = typename cplx2<T>::type;
  constexpr int NY = 256 / UT, EPT = UT / NY;  // thread rows, outputs per thread
  __shared__ C tile[UT][UT + 1];
  const int in = d.rank - 1;
  const int mode = d.mode[in];
  const int tx = threadIdx.x % UT, ty = threadIdx.x / UT;
  const int tiles = nt * (nt + 1) / 2, chunks = (tiles + PTPB - 1) / PTPB;
  const int64_t npk = (int64_t)n * (n - 1) / 2, nblk = (int64_t)rows * chunks;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const I r = (I)(blk / chunks);
    const int c = (int)(blk % chunks);
    // outer packed row r: plain offset and both orders of each outer pair
    I rem = r;
    int64_t off = 0, o1a = 0, o2a = 0, o1b = 0, o2b = 0;
    int np = 0, mda = 0, mdb = 0;
    for (int k = in - 1; k >= 0; --k) {
      const I dk = (I)d.dims[k];
      const I q = rem / dk;
      const int64_t i = (int64_t)(rem - q * dk);
      rem = q;
      if (d.pair[k]) {
        int64_t pa, pb;
        decode_pair(i, pa, pb);
        const int64_t x1 = pa * d.fp[k] + pb * d.fq[k], x2 = pb * d.fp[k] + pa * d.fq[k];
        if (np == 0) {
          o1a = x1, o2a = x2, mda = d.mode[k];
        } else {
          o1b = x1, o2b = x2, mdb = d.mode[k];
        }
        ++np;
      } else {
        off += i * d.fstride[k];
      }
    }
    // order mo: bit 0 swaps the first outer pair found (innermost), bit 1 the second
    int64_t co[4];
    T cs[4];
    bool cok[4];
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      const bool ba = (mo & 1) != 0, bb = (mo & 2) != 0;
      cok[mo] = mo < (1 << np) && (!ba || mda) && (!bb || mdb);
      co[mo] = off + (np > 0 ? (ba ? o2a : o1a) : 0) + (np > 1 ? (bb ? o2b : o1b) : 0);
      cs[mo] = (ba != bb) ? T(-1) : T(1);
    }
    C* prow = packed + (int64_t)r * npk;
    const int t1 = min(tiles, (c + 1) * PTPB);
    for (int t = c * PTPB; t < t1; ++t) {
      // tile t -> (ta <= tb), t = tb (tb + 1) / 2 + ta
      int tb = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while (tb * (tb + 1) / 2 > t) --tb;
      while ((tb + 1) * (tb + 2) / 2 <= t) ++tb;
      const int ta = t - tb * (tb + 1) / 2;
      const int a0 = ta * UT, b0 = tb * UT;
      T re[EPT], im[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) re[e] = im[e] = 0;
#pragma unroll
      for (int mo = 0; mo < 4; ++mo) {
        if (!cok[mo]) continue;  // uniform over the workgroup
        const C* fb = full + co[mo];
        const T sm = cs[mo];
        for (int y = ty; y < UT; y += NY) {  // full[a][b] for a = a0 + y, along b
          const int a = a0 + y, b = b0 + tx;
          if (a < n && b < n) tile[y][tx] = fb[(int64_t)a * n + b];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int a = a0 + tx, b = b0 + ty + NY * e;
          if (a < b && b < n) {
            const C x = tile[tx][b - b0];
            re[e] += sm * x.x;
            im[e] += sm * x.y;
            if (mode) {
              const C z = fb[(int64_t)b * n + a];
              re[e] += -sm * z.x;
              im[e] += -sm * z.y;
            }
          }
        }
        __syncthreads();  // the tile is rewritten for the next order
      }
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int a = a0 + tx, b = b0 + ty + NY * e;
        if (a < b && b < n) {
          T rr = are * re[e] - aim * im[e], ii = are * im[e] + aim * re[e];
          C* pp = prow + (int64_t)b * (b - 1) / 2 + a;
          if (acc) {
            const C yv = *pp;
            rr += yv.x;
            ii += yv.y;
          }
          *pp = C{rr, ii};
        }
      }
    }
  }
}

template <typename T>
void launch_pack(const void* full, void* packed, const PackDesc& d, double are, double aim, bool acc,
                 hipStream_t st) {
  int64_t total = 1;
  for (int k = 0; k < d.rank; ++k) total *= d.dims[k];
  if (total == 0) return;
  using C = typename cplx2<T>::type;
  const int in = d.rank - 1;
  int outer_pairs = 0;
  for (int k = 0; k < in; ++k) outer_pairs += d.pair[k] ? 1 : 0;
  if (in >= 0 && d.pair[in] && d.npair[in] >= 2 && d.npair[in] < 46341 && d.fp[in] == d.npair[in] &&
      d.fq[in] == 1 && outer_pairs <= 2) {
    const int64_t n = d.npair[in], rows = total / d.dims[in], nt = (n + UT - 1) / UT;
    const int64_t chunks = (nt * (nt + 1) / 2 + PTPB - 1) / PTPB;
    const int64_t blocks = std::min<int64_t>(rows * chunks, int64_t(1) << 24);
    if (total < (int64_t(1) << 31))
      hipLaunchKernelGGL((pack_tail_pair_kernel<T, uint32_t>), dim3((unsigned)blocks), dim3(256), 0, st,
                         (const C*)full, (C*)packed, d, (uint32_t)rows, (int)n, (int)nt, (T)are, (T)aim,
                         acc ? 1 : 0);
    else
      hipLaunchKernelGGL((pack_tail_pair_kernel<T, int64_t>), dim3((unsigned)blocks), dim3(256), 0, st,
                         (const C*)full, (C*)packed, d, rows, (int)n, (int)nt, (T)are, (T)aim, acc ? 1 : 0);
    LAUNCH_CHECK();
    return;
  }
  if (total < (int64_t(1) << 31))
    hipLaunchKernelGGL((pack_kernel<T, uint32_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)full,
                       (C*)packed, d, (uint32_t)total, (T)are, (T)aim, acc ? 1 : 0);
  else
    hipLaunchKernelGGL((pack_kernel<T, int64_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)full,
                       (C*)packed, d, total, (T)are, (T)aim, acc ? 1 : 0);
  LAUNCH_CHECK();
}

template <typename T>
void launch_unpack(const void* packed, void* full, const PackDesc& d, double are, double aim, bool acc,
                   hipStream_t st) {
  int64_t total = d.full_elems;
  if (total == 0) return;
  using C = typename cplx2<T>::type;
  const int in = d.rank - 1;
  // every pair's second full dim must follow its first (one-pass row decode)
  bool adjacent = true;
  for (int k = 0; k < d.frank; ++k)
    if (d.fsec[k] == 0) adjacent = adjacent && k + 1 < d.frank && d.fsec[k + 1] == 1 && d.fmap[k + 1] == d.fmap[k];
  if (in >= 0 && d.frank >= 2 && adjacent && d.pair[in] && d.fmap[d.frank - 2] == in && d.fsec[d.frank - 2] == 0 &&
      d.fmap[d.frank - 1] == in && d.fsec[d.frank - 1] == 1 && d.pstride[in] == 1) {
    const int64_t n = d.npair[in];
    if (n >= 2 && n < 46341 && d.fdims[d.frank - 2] == n && d.fdims[d.frank - 1] == n) {
      const int64_t rows = total / (n * n), nt = (n + UT - 1) / UT;
      const int64_t blocks = std::min<int64_t>(rows * ((nt * nt + TPB - 1) / TPB), int64_t(1) << 24);
      if (total < (int64_t(1) << 31))
        hipLaunchKernelGGL((unpack_tail_pair_kernel<T, uint32_t>), dim3((unsigned)blocks), dim3(256), 0, st,
                           (const C*)packed, (C*)full, d, (uint32_t)rows, (int)n, (int)nt, (T)are, (T)aim,
                           acc ? 1 : 0);
      else
        hipLaunchKernelGGL((unpack_tail_pair_kernel<T, int64_t>), dim3((unsigned)blocks), dim3(256), 0, st,
                           (const C*)packed, (C*)full, d, rows, (int)n, (int)nt, (T)are, (T)aim, acc ? 1 : 0);
      LAUNCH_CHECK();
      return;
    }
  }
  if (total < (int64_t(1) << 31))
    hipLaunchKernelGGL((unpack_kernel<T, uint32_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)packed,
                       (C*)full, d, (uint32_t)total, (T)are, (T)aim, acc ? 1 : 0);
  else
    hipLaunchKernelGGL((unpack_kernel<T, int64_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)packed,
                       (C*)full, d, total, (T)are, (T)aim, acc ? 1 : 0);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- summed permutes
// One workgroup per 32 x 32 tile of the trailing p x q block of one row r;
// each thread owns four outputs (p = p0 + ty + 8e, q = q0 + tx).  Sources in
// the output's order are read along q directly; exchanged sources are staged
// through LDS (read along p) so that every global access is coalesced.
struct SumArgs {
  int n;
  const void* p[4];
  int swap[4];
  int virt[4];
  double re[4], im[4];
  int nouter;
  const void* U[2];
  const void* V[2];
  int64_t ustride[2], vstride[2];
  double ore[2], oim[2];
  int64_t ni, nj;
};

template <typename T, typename I>
__global__ void __launch_bounds__(256) sum_swap_kernel(SumArgs s, typename cplx2<T>::type* __restrict__ out,
                                                       int acc, I rows, int np, int nq, int ntp, int ntq) {
  using C = typename cplx2<T>::type;
  constexpr int NY = 256 / UT, EPT = UT / NY;
  __shared__ C tile[UT][UT + 1];
  __shared__ C fac[2][4][UT];  // outer-product factors of in-place sources
  static_assert(2 * 4 * UT == 256, "one factor entry per thread");
  const int tx = threadIdx.x % UT, ty = threadIdx.x / UT;
  const I per_row = (I)ntp * (I)ntq, nblk = rows * per_row;
  const int64_t blk_elems = (int64_t)np * nq;
  const I nj = (I)s.nj, ni = (I)s.ni;
  for (I blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const I r = blk / per_row;
    const int t = (int)(blk - r * per_row), p0 = (t / ntq) * UT, q0 = (t % ntq) * UT;
    const int64_t base = r * blk_elems;
    bool hv = false;
    for (int k = 0; k < s.n; ++k) hv = hv || s.virt[k] != 0;
    T re[EPT], im[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int p = p0 + ty + NY * e, q = q0 + tx;
      re[e] = im[e] = 0;
      if (acc && p < np && q < nq) {
        const C y = out[base + (int64_t)p * nq + q];
        re[e] = y.x;
        im[e] = y.y;
      }
    }
    // Outer-product factors of this tile for in-place sources, staged in
    // LDS by one load per thread (beta folded into U): fac[c][0] = beta
    // U_c[b][i][p0 + x], [1] = V_c[b][j][p0 + x], [2] = beta U_c[b][i][q0 + x],
    // [3] = V_c[b][j][q0 + x], x < 32.
    if (hv) {
      const I rj = r / nj, rb = rj / ni;
      const int64_t j = (int64_t)(r - rj * nj), i = (int64_t)(rj - rb * ni), b = (int64_t)rb;
      const int cc = threadIdx.x / (4 * UT), w = (threadIdx.x / UT) % 4, x = threadIdx.x % UT;
      const int idx = (w < 2 ? p0 : q0) + x;
      C val = C{0, 0};
      if (cc < s.nouter && idx < np) {
        if (w % 2 == 0) {
          const C u = ((const C*)s.U[cc])[b * s.ustride[cc] + i * np + idx];
          const T br = (T)s.ore[cc], bi = (T)s.oim[cc];
          val = C{br * u.x - bi * u.y, br * u.y + bi * u.x};
        } else {
          val = ((const C*)s.V[cc])[b * s.vstride[cc] + j * nq + idx];
        }
      }
      fac[cc][w][x] = val;
      __syncthreads();
    }
    for (int k = 0; k < s.n; ++k) {  // uniform over the workgroup
      const C* src = (const C*)s.p[k];
      const T ar = (T)s.re[k], ai = (T)s.im[k];
      if (s.virt[k]) {
        // tt[p][q] = sum_c beta_c U_c[i][p] V_c[j][q]; exchanged: tt[q][p]
        const bool sw = s.swap[k] != 0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          T tr = 0, ti = 0;
#pragma unroll
          for (int cc = 0; cc < 2; ++cc) {
            const C u = sw ? fac[cc][2][tx] : fac[cc][0][ty + NY * e];
            const C v = sw ? fac[cc][1][ty + NY * e] : fac[cc][3][tx];
            tr += u.x * v.x - u.y * v.y;
            ti += u.x * v.y + u.y * v.x;
          }
          re[e] += ar * tr - ai * ti;
          im[e] += ar * ti + ai * tr;
        }
      } else if (!s.swap[k]) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int p = p0 + ty + NY * e, q = q0 + tx;
          if (p < np && q < nq) {
            const C x = src[base + (int64_t)p * nq + q];
            re[e] += ar * x.x - ai * x.y;
            im[e] += ar * x.y + ai * x.x;
          }
        }
      } else {
        for (int y = ty; y < UT; y += NY) {  // src[r][q][p], rows q, along p
          const int q = q0 + y, p = p0 + tx;
          if (q < nq && p < np) tile[y][tx] = src[base + (int64_t)q * np + p];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int p = p0 + ty + NY * e, q = q0 + tx;
          if (p < np && q < nq) {
            const C x = tile[tx][ty + NY * e];
            re[e] += ar * x.x - ai * x.y;
            im[e] += ar * x.y + ai * x.x;
          }
        }
        __syncthreads();  // the tile is rewritten by the next exchanged source
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int p = p0 + ty + NY * e, q = q0 + tx;
      if (p < np && q < nq) out[base + (int64_t)p * nq + q] = C{re[e], im[e]};
    }
    if (hv) __syncthreads();  // fac is rewritten for the next tile
  }
}

template <typename T>
void launch_sum_swap(const SumSources& s, void* out, bool acc, int64_t rows, int64_t np, int64_t nq,
                     hipStream_t st) {
  if (rows <= 0 || np <= 0 || nq <= 0) return;
  LRCC_REQUIRE(s.n >= 1 && s.n <= 4 && np < (int64_t(1) << 30) && nq < (int64_t(1) << 30), LRCC_E_INTERNAL,
               "summed permute: bad sources or sizes");
  LRCC_REQUIRE(s.nouter >= 0 && s.nouter <= 2, LRCC_E_INTERNAL, "summed permute: bad outer products");
  SumArgs a{};
  a.n = s.n;
  for (int k = 0; k < s.n; ++k) {
    a.p[k] = s.p[k];
    a.swap[k] = s.swap[k];
    a.virt[k] = s.virt[k];
    a.re[k] = s.re[k];
    a.im[k] = s.im[k];
    LRCC_REQUIRE(!s.virt[k] || (s.nouter > 0 && np == nq && s.ni > 0 && s.nj > 0), LRCC_E_INTERNAL,
                 "summed permute: a virtual source needs its outer products");
  }
  a.nouter = s.nouter;
  for (int c = 0; c < s.nouter; ++c) {
    a.U[c] = s.U[c];
    a.V[c] = s.V[c];
    a.ustride[c] = s.ustride[c];
    a.vstride[c] = s.vstride[c];
    a.ore[c] = s.ore[c];
    a.oim[c] = s.oim[c];
  }
  a.ni = s.ni;
  a.nj = s.nj;
  const int64_t ntp = (np + UT - 1) / UT, ntq = (nq + UT - 1) / UT;
  const int64_t blocks = std::min<int64_t>(rows * ntp * ntq, int64_t(1) << 24);
  using C = typename cplx2<T>::type;
  if (rows * ntp * ntq < (int64_t(1) << 31) && s.ni < (int64_t(1) << 31) && s.nj < (int64_t(1) << 31))
    hipLaunchKernelGGL((sum_swap_kernel<T, uint32_t>), dim3((unsigned)blocks), dim3(256), 0, st, a, (C*)out,
                       acc ? 1 : 0, (uint32_t)rows, (int)np, (int)nq, (int)ntp, (int)ntq);
  else
    hipLaunchKernelGGL((sum_swap_kernel<T, int64_t>), dim3((unsigned)blocks), dim3(256), 0, st, a, (C*)out,
                       acc ? 1 : 0, rows, (int)np, (int)nq, (int)ntp, (int)ntq);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- fill
template <typename T>
__global__ void fill_zero_kernel(typename cplx2<T>::type* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = {T(0), T(0)};
}

template <typename T>
void launch_fill_zero(void* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel<T>, dim3(nblocks(n)), dim3(256), 0, st, (typename cplx2<T>::type*)p, n);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- reductions
// Block-wide sum of a complex double over 256 threads (4 wavefronts of 64):
// shuffle within the wavefront, then one LDS slot per wavefront.
__device__ inline double2 block_sum(double re, double im) {
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_down(re, o, 64);
    im += __shfl_down(im, o, 64);
  }
  __shared__ double2 part[4];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = {re, im};
  __syncthreads();
  double2 s = {0.0, 0.0};
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      s.x += part[k].x;
      s.y += part[k].y;
    }
  return s;
}

template <typename T>
__global__ void __launch_bounds__(256) dot_partial_kernel(const typename cplx2<T>::type* __restrict__ x, int64_t ldx,
                                                          const typename cplx2<T>::type* __restrict__ y, int64_t ldy,
                                                          int64_t n, int conjx, double2* __restrict__ part) {
  int64_t r = blockIdx.y;
  const auto* xr = x + r * ldx;
  const auto* yr = y + r * ldy;
  double re = 0, im = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double ar = xr[i].x, ai = conjx ? -(double)xr[i].y : (double)xr[i].y;
    double br = yr[i].x, bi = yr[i].y;
    re += ar * br - ai * bi;
    im += ar * bi + ai * br;
  }
  double2 s = block_sum(re, im);
  if (threadIdx.x == 0) part[r * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) reduce_rows_kernel(const double2* __restrict__ part, int nparts,
                                                          double2* __restrict__ out) {
  int64_t r = blockIdx.x;
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    re += part[r * nparts + i].x;
    im += part[r * nparts + i].y;
  }
  double2 s = block_sum(re, im);
  if (threadIdx.x == 0) out[r] = s;
}

template <typename T>
void launch_batched_dot(int64_t nvec, int64_t n, const void* x, int64_t ldx, const void* y, int64_t ldy,
                        bool conjx, void* out, void* work, hipStream_t st) {
  if (nvec <= 0) return;
  int nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 4095) / 4096));
  using C = typename cplx2<T>::type;
  hipLaunchKernelGGL(dot_partial_kernel<T>, dim3(nparts, (unsigned)nvec), dim3(256), 0, st, (const C*)x, ldx,
                     (const C*)y, ldy, n, conjx ? 1 : 0, (double2*)work);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)nvec), dim3(256), 0, st, (const double2*)work, nparts,
                     (double2*)out);
  LAUNCH_CHECK();
}

__global__ void __launch_bounds__(256) gram_partial_kernel(const double2* __restrict__ h, int64_t hs, int m,
                                                           const double2* __restrict__ e, int64_t n,
                                                           double2* __restrict__ part) {
  int64_t rk = blockIdx.y;
  int64_t r = rk / m, k = rk - r * m;
  const double2* hr = h + (r * hs + k) * n;
  const double2* er = e + r * n;
  double re = 0, im = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = hr[i], b = er[i];
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  double2 s = block_sum(re, im);
  if (threadIdx.x == 0) part[rk * gridDim.x + blockIdx.x] = s;
}

void launch_gram(int64_t nvec, int m, int64_t n, const void* h, int64_t hs, const void* e, void* out, void* work,
                 hipStream_t st) {
  if (nvec <= 0 || m <= 0) return;
  int nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 4095) / 4096));
  hipLaunchKernelGGL(gram_partial_kernel, dim3(nparts, (unsigned)(nvec * m)), dim3(256), 0, st, (const double2*)h,
                     hs, m, (const double2*)e, n, (double2*)work);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)(nvec * m)), dim3(256), 0, st, (const double2*)work, nparts,
                     (double2*)out);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- solver updates
template <typename Ts>
__global__ void __launch_bounds__(256) residual_kernel(int64_t n, const typename cplx2<Ts>::type* sig,
                                                       const double* __restrict__ shift, const double2* X,
                                                       const double2* b, int64_t bstride, double2* R,
                                                       const double* __restrict__ D) {
  int64_t r = blockIdx.y;
  double s = shift ? shift[r] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = r * n + i;
    double re = sig ? (double)sig[k].x : 0.0, im = sig ? (double)sig[k].y : 0.0;
    if (X) {
      double f = s + (D ? D[i] : 0.0);
      re += f * X[k].x;
      im += f * X[k].y;
    }
    if (b) {
      re += b[r * bstride + i].x;
      im += b[r * bstride + i].y;
    }
    R[k] = {re, im};
  }
}

template <typename Ts>
void launch_residual(int64_t nvec, int64_t n, const void* sig, const double* shift_dev, const void* X,
                     const void* b, int64_t bstride, void* R, hipStream_t st, const double* D) {
  if (nvec <= 0) return;
  unsigned gx = nblocks(n, 256, 4096);
  using C = typename cplx2<Ts>::type;
  hipLaunchKernelGGL(residual_kernel<Ts>, dim3(gx, (unsigned)nvec), dim3(256), 0, st, n, (const C*)sig, shift_dev,
                     (const double2*)X, (const double2*)b, bstride, (double2*)R, D);
  LAUNCH_CHECK();
}

template <typename T>
__global__ void zero_diag_kernel(typename cplx2<T>::type* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i * (n + 1)] = {T(0), T(0)};
}

template <typename T>
void launch_zero_diag(void* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_diag_kernel<T>, dim3(nblocks(n)), dim3(256), 0, st, (typename cplx2<T>::type*)p, n);
  LAUNCH_CHECK();
}

__global__ void __launch_bounds__(256) jacobi_kernel(int64_t n, const double* __restrict__ D,
                                                     const double* __restrict__ shift, const double2* __restrict__ X,
                                                     const double2* __restrict__ R, double2* __restrict__ Xn,
                                                     double2* __restrict__ E, const int* __restrict__ out_rows,
                                                     double2* __restrict__ E2, const int* __restrict__ active) {
  const int64_t r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t ro = out_rows ? (int64_t)out_rows[r] : r;
  double s = shift ? shift[r] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = r * n + i, ko = ro * n + i;
    double inv = 1.0 / (D[i] + s);
    double2 d = {-R[k].x * inv, -R[k].y * inv};
    if (Xn) Xn[ko] = X ? double2{X[k].x + d.x, X[k].y + d.y} : d;
    if (E) E[ko] = d;
    if (E2) E2[k] = d;
  }
}

void launch_jacobi(int64_t nvec, int64_t n, const double* D, const double* shift_dev, const void* X, const void* R,
                   void* Xn, void* E, hipStream_t st, const int* out_rows, void* E2, const int* active) {
  if (nvec <= 0) return;
  unsigned gx = nblocks(n, 256, 4096);
  hipLaunchKernelGGL(jacobi_kernel, dim3(gx, (unsigned)nvec), dim3(256), 0, st, n, D, shift_dev, (const double2*)X,
                     (const double2*)R, (double2*)Xn, (double2*)E, out_rows, (double2*)E2, active);
  LAUNCH_CHECK();
}

__global__ void __launch_bounds__(256) combine_kernel(int64_t n, int m, const double2* __restrict__ c,
                                                      const double2* __restrict__ H, int64_t hs,
                                                      double2* __restrict__ X, const int* __restrict__ active) {
  int64_t r = blockIdx.y;
  if (active && !active[r]) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double re = 0, im = 0;
    for (int k = 0; k < m; ++k) {
      double2 a = c[r * m + k], h = H[(r * hs + k) * n + i];
      re += a.x * h.x - a.y * h.y;
      im += a.x * h.y + a.y * h.x;
    }
    X[r * n + i] = {re, im};
  }
}

void launch_combine(int64_t nvec, int m, int64_t n, const void* c, const void* H, int64_t hs, void* X,
                    hipStream_t st, const int* active) {
  if (nvec <= 0) return;
  unsigned gx = nblocks(n, 256, 4096);
  hipLaunchKernelGGL(combine_kernel, dim3(gx, (unsigned)nvec), dim3(256), 0, st, n, m, (const double2*)c,
                     (const double2*)H, hs, (double2*)X, active);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- device-resident DIIS
__global__ void diis_check_kernel(int64_t nvec, const double2* __restrict__ dots, double tol, int stall, int m,
                                  DiisSlot* __restrict__ q, int* __restrict__ active, int* __restrict__ hrow) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nvec || !active[r]) return;
  DiisSlot s = q[r];
  const double rn = sqrt(fmax(0.0, dots[r].x));
  s.rn = rn;
  s.itc += 1;
  if (!isfinite(rn)) {
    s.bad = 1;
    active[r] = 0;
    q[r] = s;
    return;
  }
  if (s.bnorm < 0) s.bnorm = rn > 0 ? rn : 1.0;
  if (rn < 0.7 * s.best) {
    s.best = rn;
    s.best_it = s.itc - 1;
  }
  const bool conv = rn <= tol * s.bnorm;
  const bool stalled = stall > 0 && (s.itc - 1) - s.best_it >= stall;
  if (conv || stalled) {
    s.conv = conv ? 1 : 0;
    active[r] = 0;
  } else {
    s.iters += 1;
    if (m > 0) hrow[r] = (int)r * m + s.next;
  }
  q[r] = s;
}

void launch_diis_check(int64_t nvec, const void* dots, double tol, int stall, int m, DiisSlot* st_dev, int* active,
                       int* hrow, hipStream_t st) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(diis_check_kernel, dim3((unsigned)((nvec + 63) / 64)), dim3(64), 0, st, nvec,
                     (const double2*)dots, tol, stall, m, st_dev, active, hrow);
  LAUNCH_CHECK();
}

__device__ inline double2 cmul(double2 a, double2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ inline double cabs2(double2 a) { return hypot(a.x, a.y); }

constexpr int kDiisMax = 32;  // lrcc_config.diis_size is at most 32

// One workgroup per slot; its first thread solves the small system in LDS.
__global__ void diis_coef_kernel(int m, const double2* __restrict__ gram, DiisSlot* __restrict__ q,
                                 const int* __restrict__ active, double2* __restrict__ Gall,
                                 double2* __restrict__ coef) {
  const int64_t r = blockIdx.x;
  if (!active[r] || threadIdx.x != 0) return;
  __shared__ double2 A[(kDiisMax + 1) * (kDiisMax + 1)];
  __shared__ double2 bvec[kDiisMax + 1], xv[kDiisMax + 1];
  __shared__ int idx[kDiisMax];
  DiisSlot s = q[r];
  double2* G = Gall + r * m * m;
  double2* c = coef + r * m;
  const int p = s.next;
  s.cnt = min(s.cnt + 1, m);
  s.next = (s.next + 1) % m;
  for (int k = 0; k < m; ++k) {
    const double2 g = gram[r * m + k];
    G[k * m + p] = g;
    G[p * m + k] = {g.x, -g.y};
  }
  const int cnt = s.cnt, N = cnt + 1;
  for (int k = 0; k < cnt; ++k) idx[k] = ((s.next - cnt + k) % m + m) % m;
  double sc = 0;
  for (int i = 0; i < cnt; ++i) sc = fmax(sc, cabs2(G[idx[i] * m + idx[i]]));
  bool ok = sc > 0;
  if (ok) {
    for (int i = 0; i < cnt; ++i) {
      for (int j = 0; j < cnt; ++j) {
        const double2 g = G[idx[i] * m + idx[j]];
        A[i * N + j] = {g.x / sc, g.y / sc};
      }
      A[i * N + cnt] = {1.0, 0.0};
      A[cnt * N + i] = {1.0, 0.0};
      bvec[i] = {0.0, 0.0};
    }
    A[cnt * N + cnt] = {0.0, 0.0};
    bvec[cnt] = {1.0, 0.0};
    for (int k = 0; k < N && ok; ++k) {
      int piv = k;
      for (int i = k + 1; i < N; ++i)
        if (cabs2(A[i * N + k]) > cabs2(A[piv * N + k])) piv = i;
      if (cabs2(A[piv * N + k]) < 1e-14) {
        ok = false;
        break;
      }
      if (piv != k) {
        for (int j = 0; j < N; ++j) {
          const double2 t = A[k * N + j];
          A[k * N + j] = A[piv * N + j];
          A[piv * N + j] = t;
        }
        const double2 t = bvec[k];
        bvec[k] = bvec[piv];
        bvec[piv] = t;
      }
      for (int i = k + 1; i < N; ++i) {
        const double2 f = cdiv(A[i * N + k], A[k * N + k]);
        for (int j = k; j < N; ++j) {
          const double2 t = cmul(f, A[k * N + j]);
          A[i * N + j] = {A[i * N + j].x - t.x, A[i * N + j].y - t.y};
        }
        const double2 t = cmul(f, bvec[k]);
        bvec[i] = {bvec[i].x - t.x, bvec[i].y - t.y};
      }
    }
  }
  for (int k = 0; k < m; ++k) c[k] = {0.0, 0.0};
  if (ok) {
    for (int i = N - 1; i >= 0; --i) {
      double2 t = bvec[i];
      for (int j = i + 1; j < N; ++j) {
        const double2 u = cmul(A[i * N + j], xv[j]);
        t = {t.x - u.x, t.y - u.y};
      }
      xv[i] = cdiv(t, A[i * N + i]);
    }
    for (int i = 0; i < cnt; ++i) c[idx[i]] = xv[i];
  } else {  // restart the subspace from the newest entry
    s.cnt = 1;
    c[p] = {1.0, 0.0};
  }
  q[r] = s;
}

void launch_diis_coef(int64_t nvec, int m, const void* gram, DiisSlot* st_dev, const int* active, void* G,
                      void* coef, hipStream_t st) {
  if (nvec <= 0 || m <= 0) return;
  LRCC_REQUIRE(m <= kDiisMax, LRCC_E_INVALID, "DIIS subspace larger than 32");
  hipLaunchKernelGGL(diis_coef_kernel, dim3((unsigned)nvec), dim3(64), 0, st, m, (const double2*)gram, st_dev,
                     active, (double2*)G, (double2*)coef);
  LAUNCH_CHECK();
}

__global__ void d2s_kernel(int64_t n, const double2* __restrict__ in, float2* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = {(float)in[i].x, (float)in[i].y};
}
__global__ void s2d_kernel(int64_t n, const float2* __restrict__ in, double2* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = {(double)in[i].x, (double)in[i].y};
}
void launch_d2s(int64_t n, const void* in, void* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(d2s_kernel, dim3(nblocks(n)), dim3(256), 0, st, n, (const double2*)in, (float2*)out);
  LAUNCH_CHECK();
}
void launch_s2d(int64_t n, const void* in, void* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(s2d_kernel, dim3(nblocks(n)), dim3(256), 0, st, n, (const float2*)in, (double2*)out);
  LAUNCH_CHECK();
}

template <typename Ti, typename To>
__global__ void copy_rows_kernel(int64_t w, const typename cplx2<Ti>::type* __restrict__ src, int64_t sld,
                                 typename cplx2<To>::type* __restrict__ dst, int64_t dld) {
  int64_t r = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < w; i += (int64_t)gridDim.x * blockDim.x) {
    auto x = src[r * sld + i];
    dst[r * dld + i] = {(To)x.x, (To)x.y};
  }
}

template <typename Ti, typename To>
void launch_copy_rows(int64_t rows, int64_t w, const void* src, int64_t sld, void* dst, int64_t dld,
                      hipStream_t st) {
  if (rows <= 0 || w <= 0) return;
  LRCC_REQUIRE(rows < 65536, LRCC_E_INVALID, "too many rows");
  hipLaunchKernelGGL((copy_rows_kernel<Ti, To>), dim3(nblocks(w, 256, 8192), (unsigned)rows), dim3(256), 0, st, w,
                     (const typename cplx2<Ti>::type*)src, sld, (typename cplx2<To>::type*)dst, dld);
  LAUNCH_CHECK();
}
template void launch_copy_rows<double, double>(int64_t, int64_t, const void*, int64_t, void*, int64_t, hipStream_t);
template void launch_copy_rows<double, float>(int64_t, int64_t, const void*, int64_t, void*, int64_t, hipStream_t);
template void launch_copy_rows<float, float>(int64_t, int64_t, const void*, int64_t, void*, int64_t, hipStream_t);
template void launch_copy_rows<float, double>(int64_t, int64_t, const void*, int64_t, void*, int64_t, hipStream_t);

__global__ void denominators_kernel(int64_t o, int64_t v, const double* __restrict__ eps, double* __restrict__ D) {
  int64_t n1 = o * v, V = v * (v - 1) / 2, O = o * (o - 1) / 2;
  int64_t n = n1 + O * V;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    if (k < n1) {
      int64_t i = k / v, a = k - i * v;
      D[k] = eps[o + a] - eps[i];
    } else {
      int64_t q = k - n1;
      int64_t I = q / V, A = q - I * V;
      int64_t i, j, a, b;
      decode_pair(I, i, j);
      decode_pair(A, a, b);
      D[k] = eps[o + a] + eps[o + b] - eps[i] - eps[j];
    }
  }
}

void launch_denominators(int64_t o, int64_t v, const double* eps, double* D, hipStream_t st) {
  int64_t n = o * v + (o * (o - 1) / 2) * (v * (v - 1) / 2);
  hipLaunchKernelGGL(denominators_kernel, dim3(nblocks(n)), dim3(256), 0, st, o, v, eps, D);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- integral assembly
template <typename T>
__global__ void __launch_bounds__(256) pack_vvvv_kernel(int64_t v, int64_t a0, int64_t b0,
                                                        const typename cplx2<T>::type* __restrict__ C,
                                                        typename cplx2<T>::type* __restrict__ W) {
  // grid.y: (a - a0) * v + b ; grid.x * 256: E
  int64_t ab = blockIdx.y;
  int64_t al = ab / v, b = ab - al * v;
  int64_t a = a0 + al;
  if (b <= a) return;
  int64_t V = v * (v - 1) / 2;
  int64_t row = b * (b - 1) / 2 + a;
  int64_t ld = (v - b0) * v;
  const auto* Ca = C + al * v * ld + (b - b0) * v;  // C[al][e][b][f] at Ca[e*ld + f]
  for (int64_t E = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; E < V; E += (int64_t)gridDim.x * blockDim.x) {
    int64_t e, f;
    decode_pair(E, e, f);
    auto x = Ca[e * ld + f];
    auto y = Ca[f * ld + e];
    W[row * V + E] = {x.x - y.x, x.y - y.y};
  }
}

template <typename T>
void launch_pack_vvvv(int64_t v, int64_t a0, int64_t a1, int64_t b0, const void* C, void* W, hipStream_t st) {
  int64_t V = v * (v - 1) / 2;
  if (V == 0 || a1 <= a0) return;
  using Cx = typename cplx2<T>::type;
  unsigned gx = nblocks(V, 256, 64);
  hipLaunchKernelGGL(pack_vvvv_kernel<T>, dim3(gx, (unsigned)((a1 - a0) * v)), dim3(256), 0, st, v, a0, b0,
                     (const Cx*)C, (Cx*)W);
  LAUNCH_CHECK();
}

template <typename T>
__global__ void __launch_bounds__(256) pack_wrows_kernel(int64_t v, int64_t b0, int64_t b1,
                                                         const typename cplx2<T>::type* __restrict__ C,
                                                         typename cplx2<T>::type* __restrict__ Wc) {
  // grid.y: row offset from P(0, b0); grid.x * 256: E = P(e, f)
  const int64_t V = v * (v - 1) / 2;
  int64_t a, b;
  decode_pair(b0 * (b0 - 1) / 2 + blockIdx.y, a, b);
  const int64_t ld = b1 * v;
  const auto* Cr = C + (b - b0) * v * ld + a * v;  // (ae|bf) at Cr[f * ld + e]
  for (int64_t E = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; E < V; E += (int64_t)gridDim.x * blockDim.x) {
    int64_t e, f;
    decode_pair(E, e, f);
    const auto x = Cr[f * ld + e];
    const auto y = Cr[e * ld + f];
    Wc[(int64_t)blockIdx.y * V + E] = {x.x - y.x, x.y - y.y};
  }
}

template <typename T>
void launch_pack_wrows(int64_t v, int64_t b0, int64_t b1, const void* C, void* Wc, hipStream_t st) {
  const int64_t V = v * (v - 1) / 2, nr = b1 * (b1 - 1) / 2 - b0 * (b0 - 1) / 2;
  if (V == 0 || nr <= 0) return;
  using Cx = typename cplx2<T>::type;
  hipLaunchKernelGGL(pack_wrows_kernel<T>, dim3(nblocks(V, 256, 64), (unsigned)nr), dim3(256), 0, st, v, b0, b1,
                     (const Cx*)C, (Cx*)Wc);
  LAUNCH_CHECK();
}

// Per-block maxima of |X[q][p][r] - conj X[q][r][p]| and |X[q][p][r]| over
// nq square n x n complex matrices (Hermiticity check of the DF factors).
__global__ void __launch_bounds__(256) herm_defect_kernel(int64_t nq, int64_t n, const double2* __restrict__ X,
                                                          double* __restrict__ part) {
  const int64_t total = nq * n * n;
  double dmax = 0, amax = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i % n, t = i / n, p = t % n, q = t / n;
    const double2 x = X[i], y = X[(q * n + r) * n + p];
    dmax = fmax(dmax, hypot(x.x - y.x, x.y + y.y));
    amax = fmax(amax, hypot(x.x, x.y));
  }
  __shared__ double sd[256], sa[256];
  sd[threadIdx.x] = dmax;
  sa[threadIdx.x] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
      sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sa[0];
  }
}

void launch_herm_defect(int64_t nq, int64_t n, const void* X, void* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(herm_defect_kernel, dim3(nparts), dim3(256), 0, st, nq, n, (const double2*)X, (double*)part);
  LAUNCH_CHECK();
}

__global__ void gather_block_kernel(int64_t naux, int64_t nmo, int64_t p0, int64_t np, int64_t r0, int64_t nr,
                                    const double2* __restrict__ src, double2* __restrict__ dst) {
  int64_t total = naux * np * nr;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = i % nr, t = i / nr;
    int64_t p = t % np, x = t / np;
    dst[i] = src[(x * nmo + p0 + p) * nmo + r0 + r];
  }
}

void launch_gather_block(int64_t naux, int64_t nmo, int64_t p0, int64_t np, int64_t r0, int64_t nr, const void* src,
                         void* dst, hipStream_t st) {
  int64_t total = naux * np * nr;
  if (total == 0) return;
  hipLaunchKernelGGL(gather_block_kernel, dim3(nblocks(total)), dim3(256), 0, st, naux, nmo, p0, np, r0, nr,
                     (const double2*)src, (double2*)dst);
  LAUNCH_CHECK();
}

// ---------------------------------------------------------------- materialize
template <typename T, typename I>
__global__ void __launch_bounds__(256) materialize_kernel(const typename cplx2<T>::type* __restrict__ src,
                                                          typename cplx2<T>::type* __restrict__ out, MatDesc d,
                                                          I total, T are, T aim, int acc) {
  for (I lin = (I)blockIdx.x * blockDim.x + threadIdx.x; lin < total; lin += (I)gridDim.x * blockDim.x) {
    I rem = lin;
    int64_t off = 0, p = -1, q = -1;
    for (int k = d.rank - 1; k >= 0; --k) {
      const I dk = (I)d.dims[k];
      const I qt = rem / dk;
      const int64_t i = (int64_t)(rem - qt * dk) + d.shift[k];
      rem = qt;
      if (d.pairpos[k] < 0)
        off += i * d.str[k];
      else if (d.pairpos[k] == 0)
        p = i;
      else
        q = i;
    }
    T s = 1;
    bool zero = false;
    if (p >= 0) {
      if (p == q) {
        zero = true;
      } else if (p < q) {
        off += (q * (q - 1) / 2 + p) * d.pstride;
      } else {
        off += (p * (p - 1) / 2 + q) * d.pstride;
        s = -s;
      }
    }
    T re = 0, im = 0;
    if (!zero) {
      const auto x = src[off];
      const T xr = x.x, xi = d.conj ? -x.y : x.y;
      re = s * (are * xr - aim * xi);
      im = s * (are * xi + aim * xr);
    }
    if (acc) {
      const auto y = out[lin];
      re += y.x;
      im += y.y;
    }
    out[lin] = {re, im};
  }
}

template <typename T>
void launch_materialize(const void* src, void* out, const MatDesc& d, double are, double aim, bool acc,
                        hipStream_t st) {
  int64_t total = 1;
  for (int k = 0; k < d.rank; ++k) total *= d.dims[k];
  if (total == 0) return;
  using C = typename cplx2<T>::type;
  if (total < (int64_t(1) << 31))
    hipLaunchKernelGGL((materialize_kernel<T, uint32_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)src,
                       (C*)out, d, (uint32_t)total, (T)are, (T)aim, acc ? 1 : 0);
  else
    hipLaunchKernelGGL((materialize_kernel<T, int64_t>), dim3(nblocks(total)), dim3(256), 0, st, (const C*)src,
                       (C*)out, d, total, (T)are, (T)aim, acc ? 1 : 0);
  LAUNCH_CHECK();
}

// explicit instantiations
#define INST(T)                                                                                               \
  template void launch_permute<T>(const void*, void*, const PermDesc&, double, double, double, double,       \
                                  hipStream_t);                                                              \
  template void launch_pack<T>(const void*, void*, const PackDesc&, double, double, bool, hipStream_t);      \
  template void launch_unpack<T>(const void*, void*, const PackDesc&, double, double, bool, hipStream_t);    \
  template void launch_fill_zero<T>(void*, int64_t, hipStream_t);                                            \
  template void launch_sum_swap<T>(const SumSources&, void*, bool, int64_t, int64_t, int64_t, hipStream_t);   \
  template void launch_batched_dot<T>(int64_t, int64_t, const void*, int64_t, const void*, int64_t, bool,    \
                                      void*, void*, hipStream_t);                                            \
  template void launch_residual<T>(int64_t, int64_t, const void*, const double*, const void*, const void*,   \
                                   int64_t, void*, hipStream_t, const double*);                              \
  template void launch_zero_diag<T>(void*, int64_t, hipStream_t);                                            \
  template void launch_pack_vvvv<T>(int64_t, int64_t, int64_t, int64_t, const void*, void*, hipStream_t);    \
  template void launch_pack_wrows<T>(int64_t, int64_t, int64_t, const void*, void*, hipStream_t);           \
  template void launch_materialize<T>(const void*, void*, const MatDesc&, double, double, bool, hipStream_t);
INST(double)
INST(float)

}  // namespace lrcc
