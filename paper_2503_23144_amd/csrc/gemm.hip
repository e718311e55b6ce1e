// Complex GEMM on CDNA4 matrix cores (gfx950).
//
//   C = alpha op(A) op(B) + beta C,  op = identity or transpose (no conjugate)
//
// FP64: complex product by 4 real products on v_mfma_f64_16x16x4_f64,
//       (Ar + i Ai)(Br + i Bi) = (ArBr - AiBi) + i (ArBi + AiBr).
// FP32: 3 real products (Gauss / Karatsuba) on v_mfma_f32_16x16x4_f32 with
//       FP32 accumulation:  P1 = ArBr, P2 = AiBi, P3 = (Ar+Ai)(Br+Bi),
//       Re = P1 - P2, Im = P3 - P1 - P2.  The pre-added planes (Ar+Ai),
//       (Br+Bi) are formed once per element when a tile is staged to LDS.
//
// Tiling: a 256-thread workgroup (4 wavefronts of 64 lanes, 2 x 2) owns a
// BM x BN tile of C; each wavefront owns (BM/2) x (BN/2) made of 16 x 16
// MFMA blocks.  K advances in BK-deep slabs staged in LDS as real planes
// laid out [k][row] so that the MFMA operand read (lane l takes row l%16 at
// k = l/16) is a contiguous 16-element run per k.  The next slab is
// prefetched to registers while the current one is consumed.  Blocks are
// remapped so that consecutive workgroups on one XCD walk the M tiles of the
// same N column (reuse of the B slab in that XCD's L2).
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace lrcc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct cpx;
// Output row of accumulator register r in lane group g = lane/16 (column
// lane%16): the FP64 instruction interleaves rows across lane groups, the
// FP32 one gives each lane group four consecutive rows.
template <>
struct cpx<double> {
  using type = double2;
  using acc = d4;
  static constexpr int planes = 2;
  static __device__ constexpr int row(int g, int r) { return g + 4 * r; }
};
template <>
struct cpx<float> {
  using type = float2;
  using acc = f4;
  static constexpr int planes = 3;
  static __device__ constexpr int row(int g, int r) { return 4 * g + r; }
};

__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int WM = BM / 2, WN = BN / 2;      // wavefront tile
constexpr int TI = WM / 16, TJ = WN / 16;    // MFMA blocks per wavefront
constexpr int LOADS = BM * BK / NT;          // complex elements per thread per operand slab

// Map a linear workgroup id to (tile_m, tile_n).  Hardware dispatches
// consecutive ids round-robin over the 8 XCDs; regroup so that each XCD sees
// a contiguous run of ids, which walk M fastest inside one N column.
__device__ inline void tile_of(int64_t bid, int64_t nbm, int64_t nbn, int64_t& tm, int64_t& tn) {
  int64_t total = nbm * nbn;
  int64_t id = bid;
  if (total >= 64 && total % 8 == 0) {
    int64_t per = total / 8;
    id = (bid % 8) * per + bid / 8;
  }
  tm = id % nbm;
  tn = id / nbm;
}

// KIND only separates kernel symbols (0: general contraction, 1: the packed
// vvvv ladder), so that profiles attribute time to the ladder.
template <typename T, bool TA, bool TB, int KIND>
__global__ void __launch_bounds__(NT) zgemm_kernel(int64_t M, int64_t N, int64_t K, T are, T aim,
                                                  const typename cpx<T>::type* __restrict__ A, int64_t lda,
                                                  const typename cpx<T>::type* __restrict__ B, int64_t ldb, T bre,
                                                  T bim, typename cpx<T>::type* __restrict__ C, int64_t ldc) {
  using V2 = typename cpx<T>::type;
  using ACC = typename cpx<T>::acc;
  constexpr int NP = cpx<T>::planes;
  __shared__ T As[NP][BK][BM];
  __shared__ T Bs[NP][BK][BN];

  const int64_t nbm = (M + BM - 1) / BM, nbn = (N + BN - 1) / BN;
  int64_t tm, tn;
  tile_of(blockIdx.x, nbm, nbn, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int r16 = lane & 15, kq = lane >> 4;

  // per-thread load coordinates (tile-local)
  int la_r[LOADS], la_k[LOADS], lb_c[LOADS], lb_k[LOADS];
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    if (!TA) {  // A[m][k]: thread walks 4 consecutive k
      la_r[q] = tid >> 2;
      la_k[q] = (tid & 3) * 4 + q;
    } else {  // A stored [k][m]: 4 consecutive m
      la_k[q] = tid >> 4;
      la_r[q] = (tid & 15) * 4 + q;
    }
    if (!TB) {  // B[k][n]: 4 consecutive n
      lb_k[q] = tid >> 4;
      lb_c[q] = (tid & 15) * 4 + q;
    } else {  // B stored [n][k]: 4 consecutive k
      lb_c[q] = tid >> 2;
      lb_k[q] = (tid & 3) * 4 + q;
    }
  }

  V2 ra[LOADS], rb[LOADS];
  auto load_slab = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      int64_t gm = m0 + la_r[q], gk = k0 + la_k[q];
      V2 z = {T(0), T(0)};
      if (gm < M && gk < K) z = TA ? A[gk * lda + gm] : A[gm * lda + gk];
      ra[q] = z;
      int64_t gn = n0 + lb_c[q], gk2 = k0 + lb_k[q];
      V2 w = {T(0), T(0)};
      if (gn < N && gk2 < K) w = TB ? B[gn * ldb + gk2] : B[gk2 * ldb + gn];
      rb[q] = w;
    }
  };
  auto store_slab = [&]() {
#pragma unroll
    for (int q = 0; q < LOADS; ++q) {
      As[0][la_k[q]][la_r[q]] = ra[q].x;
      As[1][la_k[q]][la_r[q]] = ra[q].y;
      Bs[0][lb_k[q]][lb_c[q]] = rb[q].x;
      Bs[1][lb_k[q]][lb_c[q]] = rb[q].y;
      if constexpr (NP == 3) {
        As[2][la_k[q]][la_r[q]] = ra[q].x + ra[q].y;
        Bs[2][lb_k[q]][lb_c[q]] = rb[q].x + rb[q].y;
      }
    }
  };

  ACC acc[NP][TI][TJ];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[p][i][j] = ACC{0, 0, 0, 0};

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load_slab(0);
    store_slab();
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load_slab((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int k = ks * 4 + kq;
      T ar[TI], ai[TI], br[TJ], bi[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        ar[i] = As[0][k][wm + i * 16 + r16];
        ai[i] = As[1][k][wm + i * 16 + r16];
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        br[j] = Bs[0][k][wn + j * 16 + r16];
        bi[j] = Bs[1][k][wn + j * 16 + r16];
      }
      if constexpr (NP == 2) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            acc[0][i][j] = mfma(ar[i], br[j], acc[0][i][j]);
            acc[0][i][j] = mfma(-ai[i], bi[j], acc[0][i][j]);
            acc[1][i][j] = mfma(ar[i], bi[j], acc[1][i][j]);
            acc[1][i][j] = mfma(ai[i], br[j], acc[1][i][j]);
          }
      } else {
        T as[TI], bs[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) as[i] = As[2][k][wm + i * 16 + r16];
#pragma unroll
        for (int j = 0; j < TJ; ++j) bs[j] = Bs[2][k][wn + j * 16 + r16];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            acc[0][i][j] = mfma(ar[i], br[j], acc[0][i][j]);
            acc[1][i][j] = mfma(ai[i], bi[j], acc[1][i][j]);
            acc[2][i][j] = mfma(as[i], bs[j], acc[2][i][j]);
          }
      }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store_slab();
      __syncthreads();
    }
  }

  // epilogue: register r of a lane holds row cpx<T>::row(lane/16, r), column lane%16
  const bool use_beta = (bre != T(0) || bim != T(0));
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t gm = m0 + wm + i * 16 + cpx<T>::row(kq, r);
        int64_t gn = n0 + wn + j * 16 + r16;
        if (gm >= M || gn >= N) continue;
        T re, im;
        if constexpr (NP == 2) {
          re = acc[0][i][j][r];
          im = acc[1][i][j][r];
        } else {
          T p1 = acc[0][i][j][r], p2 = acc[1][i][j][r], p3 = acc[2][i][j][r];
          re = p1 - p2;
          im = p3 - p1 - p2;
        }
        T cr = are * re - aim * im, ci = are * im + aim * re;
        V2* c = C + gm * ldc + gn;
        if (use_beta) {
          V2 y = *c;
          cr += bre * y.x - bim * y.y;
          ci += bre * y.y + bim * y.x;
        }
        *c = V2{cr, ci};
      }
}

template <typename T>
void launch_gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double are, double aim, const void* A,
                 int64_t lda, const void* B, int64_t ldb, double bre, double bim, void* C, int64_t ldc,
                 hipStream_t st, int kind) {
  if (m <= 0 || n <= 0) return;
  using V2 = typename cpx<T>::type;
  int64_t nb = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
  LRCC_REQUIRE(nb < (int64_t(1) << 31), LRCC_E_INVALID, "gemm grid too large");
  dim3 grid((unsigned)nb), block(NT);
#define GO(TA_, TB_, K_)                                                                                     \
  hipLaunchKernelGGL((zgemm_kernel<T, TA_, TB_, K_>), grid, block, 0, st, m, n, k, (T)are, (T)aim, (const V2*)A, \
                     lda, (const V2*)B, ldb, (T)bre, (T)bim, (V2*)C, ldc)
  if (kind == 1 && !ta && tb)
    GO(false, true, 1);
  else if (kind == 1 && !ta && !tb)
    GO(false, false, 1);
  else if (!ta && !tb)
    GO(false, false, 0);
  else if (!ta && tb)
    GO(false, true, 0);
  else if (ta && !tb)
    GO(true, false, 0);
  else
    GO(true, true, 0);
#undef GO
  HIP_CHECK(hipGetLastError());
}

template void launch_gemm<double>(bool, bool, int64_t, int64_t, int64_t, double, double, const void*, int64_t,
                                  const void*, int64_t, double, double, void*, int64_t, hipStream_t, int);
template void launch_gemm<float>(bool, bool, int64_t, int64_t, int64_t, double, double, const void*, int64_t,
                                 const void*, int64_t, double, double, void*, int64_t, hipStream_t, int);

}  // namespace lrcc
