// Complex GEMM on CDNA4 matrix cores (gfx950).
//
//   C = alpha op(A) op(B) + beta C,  op = identity or transpose; B may be
//   conjugated (its imaginary plane is negated when staged)
//
// FP64: complex product by 4 real products on v_mfma_f64_16x16x4_f64,
//       (Ar + i Ai)(Br + i Bi) = (ArBr - AiBi) + i (ArBi + AiBr).
// FP32: 3 real products (Gauss / Karatsuba) on v_mfma_f32_16x16x4_f32 with
//       FP32 accumulation:  P1 = ArBr, P2 = AiBi, P3 = (Ar+Ai)(Br+Bi),
//       Re = P1 - P2, Im = P3 - P1 - P2.  The pre-added planes (Ar+Ai),
//       (Br+Bi) are formed in registers from the staged planes.
//
// Tiling: a workgroup of 4 wavefronts of 64 lanes (2 x 2) owns a BM x BN
// tile of C (64 x 64, 128 x 64, or 128 x 128 for FP32), or 8 wavefronts
// (2 x 4) own a 128 x 128 tile, or, for products at most 32 wide, 4
// wavefronts stacked along M own a 128 x 32 tile; the autotuner picks per
// shape.  Each
// wavefront owns a block of 16 x 16 MFMA outputs.  K advances in 16-deep
// slabs (32 for the FP32 128 x 128 tiles) staged in LDS as two real planes
// (re, im; the Gauss sums are formed in registers) whose layout follows the
// operand's global layout, padded so that the MFMA operand reads are free of
// bank conflicts.
// Global loads are lane-contiguous along the operand's contiguous dimension
// and unconditional (clamped addresses; the K tail is zeroed in LDS).  The
// next slab is fetched into registers while the current one is consumed;
// where LDS allows, it is double-buffered (one barrier per slab).  MFMA
// operand fragments are read from LDS one 4-deep step ahead.  Each XCD
// walks a contiguous run of tiles in groups of 8 tile rows, so both operand
// panels are shared in its L2.  The epilogue stores through an output map,
// so a product can land directly in a tensor of any index order; deep
// products with few tiles are split over K.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.h"
#include "devmem.h"
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
  static constexpr bool gauss = false;  // 4 real products
  static __device__ constexpr int row(int g, int r) { return g + 4 * r; }
};
template <>
struct cpx<float> {
  using type = float2;
  using acc = f4;
  static constexpr bool gauss = true;  // 3 real products
  static __device__ constexpr int row(int g, int r) { return 4 * g + r; }
};

__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// LDS padding (32 banks of 4 bytes).  MFMA operand reads take row l%16 at
// k = l/16 for lane l.  Row layout [row][k]: an FP32 read serves 32 lanes
// (16 rows x 2 k) at once, so the row stride must be twice an odd number;
// an FP64 read serves 16 lanes (16 rows, 2 banks each), so it must be odd.
// k-major layout [k][row]: the row stride is 16 mod 32, putting the two
// lane groups of a 32-lane FP32 read on disjoint halves of the banks.
template <typename T>
constexpr int padk() { return sizeof(T) == 4 ? 2 : 1; }
constexpr int PADR = 16;

// Map a linear workgroup id to (tile_m, tile_n).  Hardware dispatches
// consecutive ids round-robin over the 8 XCDs; regroup so that each XCD sees
// a contiguous run of ids (XCDs 0..r-1 take one tile more when the grid does
// not divide by 8).  Runs are then walked in groups of GM tile rows, M
// fastest: 32 consecutive tiles on one XCD cover 8 x 4 tiles, so A and B
// panels are both shared in that XCD's L2.
constexpr int64_t GM = 8;
// Products at most this wide (n) use the 128 x 32 tile.
constexpr int64_t kNarrow = 32;

// Split products run on the 128 x 32 tile when they are narrow or when its
// grid pads the m x n output at least 10 % less than the 64 x 64 grid (n = 150:
// 160 columns instead of 192).
static bool split_narrow(int64_t m, int64_t n) {
  if (n <= kNarrow) return true;
  const double p64 = (double)((m + 63) / 64 * 64) * (double)((n + 63) / 64 * 64);
  const double p32 = (double)((m + 127) / 128 * 128) * (double)((n + 31) / 32 * 32);
  return p32 < 0.9 * p64;
}
__device__ inline void tile_of(int64_t bid, int64_t nbm, int64_t nbn, int64_t& tm, int64_t& tn) {
  const int64_t total = nbm * nbn;
  int64_t id = bid;
  if (total >= 64) {
    const int64_t q = total / 8, r = total % 8, x = bid % 8, j = bid / 8;
    id = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
  }
  const int64_t width = GM * nbn;
  const int64_t first_m = (id / width) * GM;
  const int64_t gm = nbm - first_m < GM ? nbm - first_m : GM;
  const int64_t rem = id % width;
  tm = first_m + rem % gm;
  tn = rem / gm;
}

// Register staging of one operand tile: IN elements along the dimension
// that is contiguous in global memory, PER elements per thread, STEP rows of
// the other dimension per pass of the NT threads.
template <int ROWS, bool KMAJ, int BK, int NT>
struct Stage {
  static constexpr int IN = KMAJ ? ROWS : BK;
  static constexpr int PER = ROWS * BK / NT;
  static constexpr int STEP = NT / IN;
  static_assert(NT % IN == 0 && (ROWS * BK) % NT == 0, "tile does not split over the workgroup");
};

// LDS tile of one operand, one real plane per component.  The layout follows
// the operand's global layout, so lane-consecutive staging writes hit
// consecutive banks:
//   KMAJ (global contiguous along rows):  [k][row + PADR]
//   row layout (global contiguous along k): [row][k + padk]
template <typename T, int ROWS, bool KMAJ, int BK>
struct Tile {
  static constexpr int LD = KMAJ ? ROWS + PADR : BK + padk<T>();
  static constexpr int SIZE = KMAJ ? BK * LD : ROWS * LD;
  static __device__ inline int at(int row, int k) { return KMAJ ? k * LD + row : row * LD + k; }
};

// KIND only separates kernel symbols (0: general contraction, 1: the packed
// vvvv ladder, +2: autotuner probes of either), so that profiles attribute
// time to the ladder and never mix probes into it.  The workgroup
// (NW wavefronts, WGM x (NW/WGM)) owns a BM x BN tile of C.
//
// Split-K: blockIdx.y selects the depth range [y * kchunk, (y + 1) * kchunk)
// and the output C + y * cstride (partial products, reduced afterwards).
template <typename T, bool TA, bool TB, int KIND, int BM, int BN, int WGM, int BK, int NW>
__global__ void __launch_bounds__(64 * NW) zgemm_kernel(int64_t M, int64_t N, int64_t K, T are, T aim,
                                                  const typename cpx<T>::type* __restrict__ A, int64_t lda,
                                                  const typename cpx<T>::type* __restrict__ B, int64_t ldb, T bre,
                                                  T bim, typename cpx<T>::type* __restrict__ C, OutMap om,
                                                  int64_t kchunk, int64_t cstride, T bsgn) {
  using V2 = typename cpx<T>::type;
  constexpr int NT = 64 * NW;
  {
    const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
    K = (K < kbeg + kchunk ? K : kbeg + kchunk) - kbeg;
    A += TA ? kbeg * lda : kbeg;
    B += TB ? kbeg : kbeg * ldb;
    C += (int64_t)blockIdx.y * cstride;
  }
  using ACC = typename cpx<T>::acc;
  constexpr bool G3 = cpx<T>::gauss;
  constexpr int NA = G3 ? 3 : 2;  // accumulators per block
  constexpr int WGN = NW / WGM;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TI = WM / 16, TJ = WN / 16;
  using TA_ = Tile<T, BM, TA, BK>;   // A stored [k][m] when transposed
  using TB_ = Tile<T, BN, !TB, BK>;  // B stored [k][n] when not transposed
  // two real planes (re, im) per stage; the Gauss sums are formed in
  // registers.  Double-buffer when two stages still leave room for two
  // workgroups per CU (160 KB LDS), else stage once with two barriers.
  // Tiles that are register-bound to one workgroup per CU may use all of LDS.
  constexpr int STAGE_BYTES = 2 * (TA_::SIZE + TB_::SIZE) * (int)sizeof(T);
  constexpr bool ONE_PER_CU = NW == 8 || (sizeof(T) == 4 && BM * BN >= 128 * 128);
  constexpr int ST = (2 * STAGE_BYTES <= 81920 || (ONE_PER_CU && 2 * STAGE_BYTES <= 160 * 1024)) ? 2 : 1;
  __shared__ T As[ST][2][TA_::SIZE];
  __shared__ T Bs[ST][2][TB_::SIZE];

  const int64_t nbm = (M + BM - 1) / BM, nbn = (N + BN - 1) / BN;
  int64_t tm, tn;
  tile_of(blockIdx.x, nbm, nbn, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const int r16 = lane & 15, kq = lane >> 4;

  // Global -> register staging.  Consecutive lanes take consecutive
  // elements along the operand's contiguous dimension (IN), so one load
  // instruction of a wavefront covers whole cache lines.  Every load is
  // unconditional at a clamped in-range address: rows of A beyond M and
  // columns of B beyond N only feed outputs that are never stored, and in the
  // last, partial K slab the A tile's k >= K entries are zeroed in LDS, which
  // cancels whatever B holds there.
  using LA = Stage<BM, TA, BK, NT>;
  using LB = Stage<BN, !TB, BK, NT>;
  const int a_in = tid % LA::IN, a_out = tid / LA::IN;
  const int b_in = tid % LB::IN, b_out = tid / LB::IN;
  V2 ra[LA::PER], rb[LB::PER];
  auto load_slab = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < LA::PER; ++q) {
      const int o = a_out + LA::STEP * q;
      const int64_t gm = m0 + (TA ? a_in : o), gk = k0 + (TA ? o : a_in);
      const int64_t cm = gm < M ? gm : M - 1, ck = gk < K ? gk : K - 1;
      ra[q] = TA ? A[ck * lda + cm] : A[cm * lda + ck];
    }
#pragma unroll
    for (int q = 0; q < LB::PER; ++q) {
      const int o = b_out + LB::STEP * q;
      const int64_t gn = n0 + (TB ? o : b_in), gk = k0 + (TB ? b_in : o);
      const int64_t cn = gn < N ? gn : N - 1, ck = gk < K ? gk : K - 1;
      rb[q] = TB ? B[cn * ldb + ck] : B[ck * ldb + cn];
    }
  };
  auto zero_a_tail = [&](int s, int64_t k0) {
    const int kv = (int)(K - k0);  // valid depth of this slab, < BK
    for (int e = tid; e < BM * BK; e += NT) {
      const int row = e / BK, k = e % BK;
      if (k >= kv) {
        As[s][0][TA_::at(row, k)] = T(0);
        As[s][1][TA_::at(row, k)] = T(0);
      }
    }
  };
  auto store_slab = [&](int s) {
#pragma unroll
    for (int q = 0; q < LA::PER; ++q) {
      const int o = a_out + LA::STEP * q;
      const int x = TA ? TA_::at(a_in, o) : TA_::at(o, a_in);
      As[s][0][x] = ra[q].x;
      As[s][1][x] = ra[q].y;
    }
#pragma unroll
    for (int q = 0; q < LB::PER; ++q) {
      const int o = b_out + LB::STEP * q;
      const int x = TB ? TB_::at(o, b_in) : TB_::at(b_in, o);
      Bs[s][0][x] = rb[q].x;
      Bs[s][1][x] = rb[q].y * bsgn;  // bsgn = -1: conj(B)
    }
  };

  ACC acc[NA][TI][TJ];
#pragma unroll
  for (int p = 0; p < NA; ++p)
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[p][i][j] = ACC{0, 0, 0, 0};

  // MFMA operand fragments, double-buffered across the 4-deep k steps so the
  // LDS reads of step ks+1 are in flight during the products of step ks
  T ar[2][TI], ai[2][TI], br[2][TJ], bi[2][TJ];
  auto read_frag = [&](int f, int s, int ks) {
    const int k = ks * 4 + kq;
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const int x = TA_::at(wm + i * 16 + r16, k);
      ar[f][i] = As[s][0][x];
      ai[f][i] = As[s][1][x];
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int x = TB_::at(wn + j * 16 + r16, k);
      br[f][j] = Bs[s][0][x];
      bi[f][j] = Bs[s][1][x];
    }
  };
  auto products = [&](int f) {
    if constexpr (!G3) {
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          acc[0][i][j] = mfma(ar[f][i], br[f][j], acc[0][i][j]);
          acc[0][i][j] = mfma(-ai[f][i], bi[f][j], acc[0][i][j]);
          acc[1][i][j] = mfma(ar[f][i], bi[f][j], acc[1][i][j]);
          acc[1][i][j] = mfma(ai[f][i], br[f][j], acc[1][i][j]);
        }
    } else {
      T as[TI], bs[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) as[i] = ar[f][i] + ai[f][i];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bs[j] = br[f][j] + bi[f][j];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          acc[0][i][j] = mfma(ar[f][i], br[f][j], acc[0][i][j]);
          acc[1][i][j] = mfma(ai[f][i], bi[f][j], acc[1][i][j]);
          acc[2][i][j] = mfma(as[i], bs[j], acc[2][i][j]);
        }
    }
  };

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load_slab(0);
    store_slab(0);
    if (BK > K) {
      __syncthreads();  // the tail entries are written by other threads
      zero_a_tail(0, 0);
    }
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = ST == 2 ? (int)(kt & 1) : 0;
    if (kt + 1 < nk) load_slab((kt + 1) * BK);
    read_frag(0, cur, 0);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      if (ks + 1 < BK / 4) read_frag((ks + 1) & 1, cur, ks + 1);
      products(ks & 1);
    }
    if (kt + 1 < nk) {
      // with two stages the other one was last read before the previous
      // barrier; with one, wait until every wavefront is done reading it
      if constexpr (ST == 1) __syncthreads();
      store_slab(ST == 2 ? cur ^ 1 : 0);
      if ((kt + 2) * BK > K) {
        __syncthreads();  // the tail entries are written by other threads
        zero_a_tail(ST == 2 ? cur ^ 1 : 0, (kt + 1) * BK);
      }
    }
    __syncthreads();
  }

  // epilogue: register r of a lane holds row cpx<T>::row(lane/16, r), column
  // lane%16; element (m, n) goes to C + om.row(m) + om.col(n)
  const bool use_beta = (bre != T(0) || bim != T(0));
  int64_t coff[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int64_t gn = n0 + wn + j * 16 + r16;
    coff[j] = gn < N ? om.col(gn) : -1;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gm = m0 + wm + i * 16 + cpx<T>::row(kq, r);
      if (gm >= M) continue;
      const int64_t roff = om.row(gm);
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        if (coff[j] < 0) continue;
        T re, im;
        if constexpr (!G3) {
          re = acc[0][i][j][r];
          im = acc[1][i][j][r];
        } else {
          T p1 = acc[0][i][j][r], p2 = acc[1][i][j][r], p3 = acc[2][i][j][r];
          re = p1 - p2;
          im = p3 - p1 - p2;
        }
        T cr = are * re - aim * im, ci = are * im + aim * re;
        V2* c = C + roff + coff[j];
        if (use_beta) {
          V2 y = *c;
          cr += bre * y.x - bim * y.y;
          ci += bre * y.y + bim * y.x;
        }
        *c = V2{cr, ci};
      }
    }
}

// C = alpha * sum_s P[s] + beta * C over an m x n tile set (split-K reduction)
template <typename T>
__global__ void splitk_reduce_kernel(int64_t m, int64_t n, int splits, const typename cpx<T>::type* __restrict__ P,
                                     T are, T aim, T bre, T bim, typename cpx<T>::type* __restrict__ C, OutMap om) {
  const int64_t total = m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    T sr = 0, si = 0;
    for (int s = 0; s < splits; ++s) {
      const typename cpx<T>::type p = P[(int64_t)s * total + e];
      sr += p.x;
      si += p.y;
    }
    T cr = are * sr - aim * si, ci = are * si + aim * sr;
    typename cpx<T>::type* c = C + om.row(e / n) + om.col(e % n);
    if (bre != T(0) || bim != T(0)) {
      const typename cpx<T>::type y = *c;
      cr += bre * y.x - bim * y.y;
      ci += bre * y.y + bim * y.x;
    }
    *c = typename cpx<T>::type{cr, ci};
  }
}

template <typename T, int KIND, int BM, int BN, int WGM, int NW = 4>
static void go(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double are, double aim, const void* A, int64_t lda,
               const void* B, int64_t ldb, double bre, double bim, void* C, const OutMap& om, hipStream_t st,
               int splits = 1, void* ws = nullptr, bool conjb = false) {
  using V2 = typename cpx<T>::type;
  // deeper slabs for the FP32 128 x 128 tiles (one workgroup per CU: fewer
  // barriers and a longer prefetch distance)
  constexpr int BK = (sizeof(T) == 4 && BM == 128 && BN == 128) ? 32 : 16;
  constexpr int NT = 64 * NW;
  int64_t nb = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
  LRCC_REQUIRE(nb < (int64_t(1) << 31), LRCC_E_INVALID, "gemm grid too large");
  // split-K: equal depth ranges, multiples of the slab depth, none empty
  int64_t kchunk = k, cstride = 0;
  void* out = C;
  OutMap mo = om;
  double ar = are, ai = aim, br = bre, bi = bim;
  if (splits > 1) {
    kchunk = ((k + splits - 1) / splits + BK - 1) / BK * BK;
    splits = (int)((k + kchunk - 1) / kchunk);
    out = ws, mo = OutMap::plain(n), cstride = m * n;
    ar = 1, ai = 0, br = 0, bi = 0;
  }
#define GO_(TA_, TB_)                                                                                        \
  hipLaunchKernelGGL((zgemm_kernel<T, TA_, TB_, KIND, BM, BN, WGM, BK, NW>), dim3((unsigned)nb, (unsigned)splits), dim3(NT), \
                     0, st, m, n, k, (T)ar, (T)ai, (const V2*)A, lda, (const V2*)B, ldb, (T)br, (T)bi, (V2*)out, mo,  \
                     kchunk, cstride, (T)(conjb ? -1.0 : 1.0))
  if (!ta && !tb)
    GO_(false, false);
  else if (!ta && tb)
    GO_(false, true);
  else if (ta && !tb)
    GO_(true, false);
  else
    GO_(true, true);
#undef GO_
  HIP_CHECK(hipGetLastError());
  if (splits > 1) {
    const int64_t total = m * n;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3(blocks), dim3(256), 0, st, m, n, splits, (const V2*)ws, (T)are,
                       (T)aim, (T)bre, (T)bim, (V2*)C, om);
    HIP_CHECK(hipGetLastError());
  }
}

// ---------------------------------------------------------------- tile choice
// Candidate workgroup tiles: 0 = 64 x 64, 1 = 128 x 64, 2 = 128 x 128 (FP32),
// all with 4 wavefronts of (BM/2) x (BN/2); 3 = 128 x 128 with 8 wavefronts
// of 64 x 32 (two wavefronts per SIMD where tile 2 has one); 4 = 128 x 32
// with 4 wavefronts of 32 x 32 stacked along M, the heuristic's choice for
// products at most kNarrow wide, where a 64-wide tile would spend most of
// its matrix-core work on padding (N = 1 or o), and a candidate for any
// width (less padding when N is not a multiple of 64).
// The autotuner times every candidate once per GEMM shape (into a scratch
// output, so accumulating calls are not disturbed) and keeps the fastest;
// without it a size heuristic decides.  Results can persist in a text cache
// named by LRCC_AUTOTUNE_CACHE ("gfx950 prec ta tb kind m n k tile" lines,
// m n k bucketed as below).

template <typename T, int KIND>
static void dispatch(int cfgid, bool ta, bool tb, int64_t m, int64_t n, int64_t k, double are, double aim,
                     const void* A, int64_t lda, const void* B, int64_t ldb, double bre, double bim, void* C,
                     const OutMap& om, hipStream_t st, bool conjb) {
  if constexpr (sizeof(T) == 4) {  // 4 wavefronts of 64 x 64 FP64 would not fit the register file
    if (cfgid == 2)
      return go<T, KIND, 128, 128, 2>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, 1, nullptr,
                                      conjb);
  }
  if (cfgid == 3)
    return go<T, KIND, 128, 128, 2, 8>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, 1, nullptr,
                                       conjb);
  if (cfgid == 4)
    return go<T, KIND, 128, 32, 4>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, 1, nullptr,
                                   conjb);
  if (cfgid >= 1)
    go<T, KIND, 128, 64, 2>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, 1, nullptr, conjb);
  else
    go<T, KIND, 64, 64, 2>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, 1, nullptr, conjb);
}

namespace {
// Shapes are tuned per bucket: each of m, n, k above 64 is rounded down to
// its top three bits (four buckets per octave), so products within about
// 25 % of each other in every dimension share one choice.  Chunked
// contractions (the DF-direct ladder's row chunks, split virtual operands)
// produce hundreds of nearby shapes that would otherwise each be timed.
int64_t tune_bucket(int64_t x) {
  if (x <= 64) return x;
  int e = 63 - __builtin_clzll((unsigned long long)x);
  return (x >> (e - 2)) << (e - 2);
}

struct TuneKey {
  int prec, ta, tb, kind;
  int64_t m, n, k;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, ta, tb, kind, m, n, k) < std::tie(o.prec, o.ta, o.tb, o.kind, o.m, o.n, o.k);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_autotune = false;
bool g_cache_loaded = false;

std::string cache_path() {
  const char* p = std::getenv("LRCC_AUTOTUNE_CACHE");
  return p ? std::string(p) : std::string();
}

void load_cache() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  std::string path = cache_path();
  if (path.empty()) return;
  std::ifstream in(path);
  std::string arch;
  TuneKey key;
  int cfg;
  while (in >> arch >> key.prec >> key.ta >> key.tb >> key.kind >> key.m >> key.n >> key.k >> cfg)
    if (arch == "gfx950") g_tune[key] = cfg;
}

void save_entry(const TuneKey& key, int cfg) {
  std::string path = cache_path();
  if (path.empty()) return;
  std::ofstream out(path, std::ios::app);
  out << "gfx950 " << key.prec << " " << key.ta << " " << key.tb << " " << key.kind << " " << key.m << " " << key.n
      << " " << key.k << " " << cfg << "\n";
}
}  // namespace

void set_gemm_autotune(bool on) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_autotune = on;
}

int gemm_tuned_tile(int prec, bool ta, bool tb, int kind, int64_t m, int64_t n, int64_t k) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(TuneKey{prec, ta, tb, kind, tune_bucket(m), tune_bucket(n), tune_bucket(k)});
  return it == g_tune.end() ? -1 : it->second;
}

int gemm_tuned_shapes() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return (int)g_tune.size();
}

template <typename T>
static int heuristic_tile(int64_t m, int64_t n, int kind) {
  // Measured on MI355X: in FP32 the 64 x 64 tile (four workgroups per CU) is
  // the fastest on most large shapes; in FP64 the 8-wavefront 128 x 128 tile
  // is, once it still gives every CU several workgroups.  The ladder (kind 1,
  // K = V deep) runs as fast on the 8-wavefront 128 x 128 tile in FP32 too
  // (1004 against 990 ms at M = 3120, N = K = 79800) while its traffic below
  // the L2 is 6.5 times lower (0.54 against 3.6 TB per launch: four 64 x 64
  // tiles share a 128 x 128 tile's panels only while they stay in step),
  // so it takes that tile.  Narrow products take the 128 x 32 tile.
  if (n <= kNarrow) return 4;
  const int64_t big_tiles = ((m + 127) / 128) * ((n + 127) / 128);
  if ((sizeof(T) == 8 || kind == 1) && big_tiles >= 2048) return 3;
  return 0;
}

// LRCC_TRACE_GEMM=1 prints every launch's shape and tile choice to stderr.
static bool trace_on() {
  static const bool on = [] {
    const char* e = std::getenv("LRCC_TRACE_GEMM");
    return e && e[0] == '1';
  }();
  return on;
}

// A forced workgroup tile (0..4, -1 = automatic) for every unsplit launch,
// so that each tile can be tested and measured on its own; tile 2 runs as
// tile 1 in FP64.  The initial value comes from LRCC_GEMM_TILE.
static std::atomic<int> g_forced_tile{-2};
static int forced_tile() {
  int t = g_forced_tile.load(std::memory_order_relaxed);
  if (t == -2) {
    const char* e = std::getenv("LRCC_GEMM_TILE");
    t = (e && e[0] >= '0' && e[0] <= '4' && e[1] == 0) ? e[0] - '0' : -1;
    int expect = -2;
    if (!g_forced_tile.compare_exchange_strong(expect, t)) t = expect;
  }
  return t;
}

void set_gemm_tile(int tile) { g_forced_tile.store(tile >= 0 && tile <= 4 ? tile : -1); }

// Split-K for deep products whose tile grid (64 x 64, or 128 x 32 where
// split_narrow says so) fills the chip poorly.  The chip holds `slots` resident
// workgroups (64 x 64: four per CU in FP32, two in FP64; 128 x 32: three in
// FP32, two in FP64); a grid of w workgroups runs in ceil(w / slots) rounds,
// so its efficiency is w / (rounds * slots).  The depth is split s ways (at
// least 1024 deep each, at most 64 ways, partials of at most 256 MB) for
// the smallest s within 3 % of the best efficiency, and only when that
// gains at least 15 % over no split.
int gemm_splits(int64_t m, int64_t n, int64_t k, bool fp64) {
  if (k < 2048) return 1;
  const bool nar = split_narrow(m, n);
  const int64_t tiles = nar ? ((m + 127) / 128) * ((n + 31) / 32) : ((m + 63) / 64) * ((n + 63) / 64);
  const int64_t slots = nar ? (fp64 ? 512 : 768) : (fp64 ? 512 : 1024);
  const int64_t part = m * n * (fp64 ? 16 : 8);
  const int64_t smax = std::min<int64_t>({64, k / 1024, std::max<int64_t>(1, (int64_t(256) << 20) / part)});
  auto eff = [&](int64_t s) {
    const int64_t w = tiles * s, rounds = (w + slots - 1) / slots;
    return (double)w / (double)(rounds * slots);
  };
  double best = eff(1);
  for (int64_t s = 2; s <= smax; ++s) best = std::max(best, eff(s));
  int64_t pick = 1;
  for (int64_t s = 1; s <= smax; ++s)
    if (eff(s) >= 0.97 * best) {
      pick = s;
      break;
    }
  return eff(pick) >= 1.15 * eff(1) ? (int)pick : 1;
}

template <typename T>
size_t gemm_workspace_bytes(int64_t m, int64_t n, int64_t k) {
  const int s = gemm_splits(m, n, k, sizeof(T) == 8);
  return s > 1 ? (size_t)s * m * n * 2 * sizeof(T) : 0;
}

template <typename T>
void launch_gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double are, double aim, const void* A,
                 int64_t lda, const void* B, int64_t ldb, double bre, double bim, void* C, int64_t ldc,
                 hipStream_t st, int kind, void* ws, size_t ws_bytes, const OutMap* omap, bool conj_b,
                 bool allow_tune) {
  if (m <= 0 || n <= 0) return;
  const OutMap om = omap ? *omap : OutMap::plain(ldc);
  {
    const int splits = gemm_splits(m, n, k, sizeof(T) == 8);
    if (splits > 1 && ws && ws_bytes >= gemm_workspace_bytes<T>(m, n, k)) {
      if (trace_on())
        fprintf(stderr, "[lrcc gemm] %s ta=%d tb=%d kind=%d m=%lld n=%lld k=%lld tile=%d splits=%d\n",
                sizeof(T) == 8 ? "c128" : "c64", (int)ta, (int)tb, kind, (long long)m, (long long)n, (long long)k,
                split_narrow(m, n) ? 4 : 0, splits);
      if (split_narrow(m, n)) {
        if (kind == 1)
          go<T, 1, 128, 32, 4>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, splits, ws, conj_b);
        else
          go<T, 0, 128, 32, 4>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, splits, ws, conj_b);
      } else if (kind == 1) {
        go<T, 1, 64, 64, 2>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, splits, ws, conj_b);
      } else {
        go<T, 0, 64, 64, 2>(ta, tb, m, n, k, are, aim, A, lda, B, ldb, bre, bim, C, om, st, splits, ws, conj_b);
      }
      return;
    }
  }
  auto run = [&](int cfg, void* Cout, double br, double bi, bool probe) {
    if (probe) {  // plain layout into the scratch output
      const OutMap pm = OutMap::plain(n);
      if (kind == 1)
        dispatch<T, 3>(cfg, ta, tb, m, n, k, are, aim, A, lda, B, ldb, br, bi, Cout, pm, st, conj_b);
      else
        dispatch<T, 2>(cfg, ta, tb, m, n, k, are, aim, A, lda, B, ldb, br, bi, Cout, pm, st, conj_b);
    } else if (kind == 1) {
      dispatch<T, 1>(cfg, ta, tb, m, n, k, are, aim, A, lda, B, ldb, br, bi, Cout, om, st, conj_b);
    } else {
      dispatch<T, 0>(cfg, ta, tb, m, n, k, are, aim, A, lda, B, ldb, br, bi, Cout, om, st, conj_b);
    }
  };
  int cfg = heuristic_tile<T>(m, n, kind);
  bool tune = false;
  // no timing runs while the stream is being captured into a graph
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (st && hipStreamIsCapturing(st, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  const bool capturing = cap != hipStreamCaptureStatusNone;
  TuneKey key{sizeof(T) == 8 ? 64 : 32, ta, tb, kind, tune_bucket(m), tune_bucket(n), tune_bucket(k)};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (g_autotune) {
      load_cache();
      auto it = g_tune.find(key);
      if (it != g_tune.end())
        cfg = it->second;
      else
        tune = allow_tune && !capturing && forced_tile() < 0;
    }
  }
  const bool small = (double)m * n * k < 1e8;  // not worth timing
  if (tune && !small) {
    static const int cand32[] = {0, 1, 2, 3, 4}, cand64[] = {0, 1, 3, 4};
    const int* cand = sizeof(T) == 4 ? cand32 : cand64;
    const int ncand = sizeof(T) == 4 ? 5 : 4;
    void* scratch = nullptr;
    scratch = dev_alloc((size_t)m * n * 2 * sizeof(T));
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    const int heur = cfg;
    float best = 1e30f, heur_ms = 1e30f;
    for (int ci = 0; ci < ncand; ++ci) {
      const int c = cand[ci];
      float ms = 0;
      for (int rep = 0; rep < 2; ++rep) {  // a second, warm timing unless the first took long
        HIP_CHECK(hipEventRecord(e0, st));
        run(c, scratch, 0.0, 0.0, true);
        HIP_CHECK(hipEventRecord(e1, st));
        HIP_CHECK(hipEventSynchronize(e1));
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms > 50.0f) break;
      }
      if (c == heur) heur_ms = ms;
      if (ms < best) {
        best = ms;
        cfg = c;
      }
    }
    // near-ties (within 2 %, about the spread of repeated timings) keep the
    // heuristic's tile, so that the choice is the same from run to run
    if (heur_ms <= 1.02f * best) cfg = heur;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free(scratch);
  }
  if (tune) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = cfg;
    if (!small) save_entry(key, cfg);
  }
  if (forced_tile() >= 0) cfg = forced_tile();
  if (trace_on())
    fprintf(stderr, "[lrcc gemm] %s ta=%d tb=%d kind=%d m=%lld n=%lld k=%lld tile=%d splits=1\n",
            sizeof(T) == 8 ? "c128" : "c64", (int)ta, (int)tb, kind, (long long)m, (long long)n, (long long)k, cfg);
  run(cfg, C, bre, bim, false);
}

template void launch_gemm<double>(bool, bool, int64_t, int64_t, int64_t, double, double, const void*, int64_t,
                                  const void*, int64_t, double, double, void*, int64_t, hipStream_t, int, void*,
                                  size_t, const OutMap*, bool, bool);
template void launch_gemm<float>(bool, bool, int64_t, int64_t, int64_t, double, double, const void*, int64_t,
                                 const void*, int64_t, double, double, void*, int64_t, hipStream_t, int, void*,
                                 size_t, const OutMap*, bool, bool);
template size_t gemm_workspace_bytes<double>(int64_t, int64_t, int64_t);
template size_t gemm_workspace_bytes<float>(int64_t, int64_t, int64_t);

}  // namespace lrcc
