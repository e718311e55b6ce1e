// Launch wrappers of the HIP kernels (gfx950).  All complex data are
// interleaved {re, im} of T = double or float; all calls are asynchronous on
// `st`.  Sizes and strides are in complex elements.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "outmap.h"

namespace lrcc {

constexpr int kMaxRank = 8;

struct PermDesc {
  int rank;
  int64_t dims[kMaxRank];     // output dims (row-major)
  int64_t istride[kMaxRank];  // input stride for each output dim
};

// out = alpha * in[perm] + beta * out   (beta == 0: out is not read)
template <typename T>
void launch_permute(const void* in, void* out, const PermDesc& d, double are, double aim, double bre,
                    double bim, hipStream_t st);

// Pair-packing view.  The packed tensor has `rank` dims; dim k is either a
// plain dim (pair[k] == 0, size dims[k], full-tensor stride fstride[k]) or a
// packed pair of an n x n block (pair[k] == 1, n = npair[k], strides fp[k]
// (first index) and fq[k] (second index) in the full tensor, mode[k]).
struct PackDesc {
  int rank;
  int64_t dims[kMaxRank];     // packed dims
  int64_t fstride[kMaxRank];  // plain dims: stride in the full tensor
  int pair[kMaxRank];
  int64_t npair[kMaxRank];
  int64_t fp[kMaxRank], fq[kMaxRank];
  int mode[kMaxRank];
  int64_t full_elems;  // total full-tensor elements (unpack: output size)
  // unpack only: the full tensor's own dims and, per full dim, the packed
  // dim it belongs to and whether it is the first (0) or second (1) index
  int frank;
  int64_t fdims[kMaxRank];
  int fmap[kMaxRank];
  int fsec[kMaxRank];
  int64_t pstride[kMaxRank];  // packed stride of each packed dim
};

template <typename T>
void launch_pack(const void* full, void* packed, const PackDesc& d, double are, double aim, bool acc,
                 hipStream_t st);
template <typename T>
void launch_unpack(const void* packed, void* full, const PackDesc& d, double are, double aim, bool acc,
                   hipStream_t st);

// Dense tensor from a source that holds it up to a permutation, one
// antisymmetric packed pair and a complex conjugation:
//   out[t] (+)= (alpha * s) * X(src[off]),  X = conj if `conj` else identity,
// for every target multi-index t (row-major over dims[0..rank)), where index
// k of t (plus shift[k]) enters the source offset with stride str[k] (plain
// index) or as member pairpos[k] = 0 / 1 of the source's packed pair
// (offset P(p,q) * pstride with p < q, s = -1 when the members come as
// (q, p), zero when they are equal; pairpos[k] = -1 for plain indices).
struct MatDesc {
  int rank;
  int64_t dims[kMaxRank];
  int64_t shift[kMaxRank];
  int64_t str[kMaxRank];
  int pairpos[kMaxRank];
  int64_t pstride;
  int conj;
};
template <typename T>
void launch_materialize(const void* src, void* out, const MatDesc& d, double are, double aim, bool acc,
                        hipStream_t st);

template <typename T>
void launch_fill_zero(void* p, int64_t n, hipStream_t st);

// out[r][p][q] = (acc ? out : 0) + sum_s alpha_s * src_s[r][p][q] (swap[s] == 0)
// or alpha_s * src_s[r][q][p] (swap[s] == 1), in source order, r < rows,
// p < np, q < nq: a run of accumulations into one tensor whose sources are
// in its own index order or with its last two indices exchanged.  A source
// with virt[s] set is no tensor but the sum of outer products
// tt[b][i][j][p][q] = sum_c beta_c U_c[b][i][p] V_c[b][j][q], row r = (b ni + i) nj + j
// (U_c, V_c row-major, batch strides ustride/vstride elements, 0 = shared).
struct SumSources {
  int n;  // 1 .. 4
  const void* p[4];
  int swap[4];
  int virt[4];
  double re[4], im[4];
  int nouter;  // 0 .. 2 outer products
  const void* U[2];
  const void* V[2];
  int64_t ustride[2], vstride[2];
  double ore[2], oim[2];
  int64_t ni, nj;
};
template <typename T>
void launch_sum_swap(const SumSources& s, void* out, bool acc, int64_t rows, int64_t np, int64_t nq, hipStream_t st);

// out[r] = sum_k opx(x[r*ldx + k]) * y[r*ldy + k], r < nvec (FP64 result
// {re, im} in device memory).  conjx: conjugate x.  `work` holds at least
// nvec * 1024 * 16 bytes.
template <typename T>
void launch_batched_dot(int64_t nvec, int64_t n, const void* x, int64_t ldx, const void* y, int64_t ldy,
                        bool conjx, void* out, void* work, hipStream_t st);

// Gram rows: out[r*m + k] = sum_i conj(h[(r*hs + k)*n + i]) * e[r*n + i]
// (k < m) for r < nvec.  `work`: nvec*m*1024*16 bytes.
void launch_gram(int64_t nvec, int m, int64_t n, const void* h, int64_t hs, const void* e, void* out,
                 void* work, hipStream_t st);

// Dense complex GEMM C = alpha op(A) op(B) + beta C (no conjugation).
// FP64: 4 real MFMA products per complex product; FP32: 3 (Gauss).
// kind 1 marks the packed-vvvv ladder (a separate kernel symbol).  With a
// device workspace of gemm_workspace_bytes<T>(m, n, k) bytes, deep products
// with few output tiles are split over K (partials reduced in fixed order).
template <typename T>
void launch_gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double are, double aim, const void* A,
                 int64_t lda, const void* B, int64_t ldb, double bre, double bim, void* C, int64_t ldc,
                 hipStream_t st, int kind = 0, void* ws = nullptr, size_t ws_bytes = 0,
                 const OutMap* om = nullptr, bool conj_b = false,  // conj_b: use conj(B)
                 bool allow_tune = true);  // false: never time candidate tiles (no device allocation)
int gemm_splits(int64_t m, int64_t n, int64_t k, bool fp64);
template <typename T>
size_t gemm_workspace_bytes(int64_t m, int64_t n, int64_t k);

// Per-shape tile autotuning of launch_gemm (process-wide).
void set_gemm_autotune(bool on);
void set_gemm_tile(int tile);  // -1: automatic (autotuner or size heuristic)
int gemm_tuned_shapes();
// Tile the autotuner chose for a shape (kind 1: the ladder kernel), or -1.
int gemm_tuned_tile(int prec, bool ta, bool tb, int kind, int64_t m, int64_t n, int64_t k);

// Solver kernels (FP64 vectors, nvec right-hand sides of length n).
// R = sig + (D + s_r) X + b_r  (sig in Ts; D, shift, X, b may be null = 0).
template <typename Ts>
void launch_residual(int64_t nvec, int64_t n, const void* sig, const double* shift_dev, const void* X,
                     const void* b, int64_t bstride, void* R, hipStream_t st, const double* D = nullptr);
// p[i*(n+1)] = 0 for i < n (diagonal of an n x n complex matrix)
template <typename T>
void launch_zero_diag(void* p, int64_t n, hipStream_t st);
// Xn = X - R / (D + s_r);  E = Xn - X  (either output may be null).  With
// out_rows (device, nvec entries) row r of Xn and E is their row out_rows[r]
// (e.g. a slot of a history ring); E2, when given, receives E at row r too.
// With `active` (device, nvec flags) rows whose flag is 0 are left untouched.
void launch_jacobi(int64_t nvec, int64_t n, const double* D, const double* shift_dev, const void* X,
                   const void* R, void* Xn, void* E, hipStream_t st, const int* out_rows = nullptr,
                   void* E2 = nullptr, const int* active = nullptr);
// X[r] = sum_k c[r*m + k] * H[(r*hs + k)*n + ...]  (rows with active[r] == 0 untouched)
void launch_combine(int64_t nvec, int m, int64_t n, const void* c, const void* H, int64_t hs, void* X,
                    hipStream_t st, const int* active = nullptr);

// Per right-hand-side state of the device-resident DIIS iteration.
struct DiisSlot {
  double rn;     // last residual norm
  double bnorm;  // reference norm (< 0: taken from the first residual)
  double best;   // best residual norm by a factor 0.7 so far, and the evaluation it came at
  int best_it;
  int itc;       // residual evaluations so far
  int iters;     // updates applied (evaluations that left the slot active)
  int cnt;       // DIIS entries stored (<= m), ring position of the next one
  int next;
  int conv;      // 1: converged (residual <= tol * bnorm)
  int bad;       // 1: residual not finite
};
// After the residual norms dots[r] = ||R_r||^2 of nvec active-or-not slots:
// updates each active slot's state, deactivates it when converged or when
// `stall` > 0 evaluations passed without a 0.7x improvement, and sets the
// history row hrow[r] = r * m + next of the slots that stay active.
void launch_diis_check(int64_t nvec, const void* dots, double tol, int stall, int m, DiisSlot* st_dev, int* active,
                       int* hrow, hipStream_t st);
// DIIS extrapolation coefficients of every active slot, on the device: the
// new Gram row gram[r*m + k] = <e_k, e_new> enters the slot's Hermitian Gram
// matrix G[r] (m x m) at the ring position, and [G 1; 1^T 0][c; l] = [0; 1]
// over the stored entries is solved by Gaussian elimination with partial
// pivoting on G / max|G_kk|; coef[r*m + k] = c_k (0 for empty positions).
// A singular system restarts the slot's subspace from its newest entry.
void launch_diis_coef(int64_t nvec, int m, const void* gram, DiisSlot* st_dev, const int* active, void* G,
                      void* coef, hipStream_t st);
// dst[r*dld + i] = (To) src[r*sld + i], i < w, r < rows (complex; strided row copy)
template <typename Ti, typename To>
void launch_copy_rows(int64_t rows, int64_t w, const void* src, int64_t sld, void* dst, int64_t dld,
                      hipStream_t st);
// D[n]: D1[i][a] = e_a - e_i, D2[P(i,j)][P(a,b)] = e_a + e_b - e_i - e_j (eps on device, FP64 real)
void launch_denominators(int64_t o, int64_t v, const double* eps, double* D, hipStream_t st);
// precision conversion (complex)
void launch_d2s(int64_t n, const void* in, void* out, hipStream_t st);
void launch_s2d(int64_t n, const void* in, void* out, hipStream_t st);

// Integral builder: W[P(a,b)][P(e,f)] = C[a-a0][e][b-b0][f] - C[a-a0][f][b-b0][e]
// for a in [a0, a1), b in (a, v), e < f; C holds (ae|bf) for b >= b0
// (row (a-a0)*v + e, column (b-b0)*v + f, row length (v-b0)*v).
template <typename T>
void launch_pack_vvvv(int64_t v, int64_t a0, int64_t a1, int64_t b0, const void* C, void* W, hipStream_t st);
// Rows of the same W for b in [b0, b1): Wc[P(a,b) - P(0,b0)][P(e,f)] =
// C[b-b0][f][a][e] - C[b-b0][e][a][f], where C[(b-b0)*v + f][a*v + e] = (ae|bf)
// (row length b1*v).
template <typename T>
void launch_pack_wrows(int64_t v, int64_t b0, int64_t b1, const void* C, void* Wc, hipStream_t st);
// part[2b], part[2b+1] (b < nparts): maxima of |X[q][p][r] - conj X[q][r][p]|
// and of |X[q][p][r]| over nq complex FP64 n x n matrices, per block b
void launch_herm_defect(int64_t nq, int64_t n, const void* X, void* part, int nparts, hipStream_t st);
// dst[x][p][r] = src[x][p0 + p][r0 + r] (sub-block gather), p < np, r < nr
void launch_gather_block(int64_t naux, int64_t nmo, int64_t p0, int64_t np, int64_t r0, int64_t nr,
                         const void* src, void* dst, hipStream_t st);

}  // namespace lrcc
