// Perturbation-sensitive frozen natural spinors (FNS++), Section II.C.
//
//  1. MP2 doubles t_ij^ab = <ab||ij> / (e_i + e_j - e_a - e_b)         (Eq. 39)
//  2. Hbar_ii = F_ii + 1/2 sum t_in^ef <in||ef>,
//     Hbar_aa = F_aa - 1/2 sum t_mn^fa <mn||fa>                          (Eqs. 49-50)
//  3. per direction A: Abar_i^a, Abar_ij^ac (Eq. 48, singles projection
//     A_ai + sum_me A_me t_im^ae), divided by the Hbar denominators + w
//     (Eqs. 46-47, with +w as printed)
//  4. D_ab = <1/2 sum_ijc t(A)_ij^ac conj t(A)_ij^bc + sum_i t(A)_i^a conj t(A)_i^b>
//     averaged over directions and the frequency grid              (Eq. 45)
//  5. D V = V n, keep |n| > thresh or the `keep` largest             (Eq. 41)
//  6. F~ = V~^H F_vv V~, F~ Z~ = Z~ e~, U = V~ Z~                      (Eqs. 42-44)
//  7. B, F and mu are rotated with C = diag(1_occ, U) on the device and the
//     integral blocks are rebuilt in the truncated space.
// The two Hermitian eigenproblems use rocSOLVER (zheevd).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>

#include "context.h"
#include "kernels.h"

namespace lrcc {

namespace {

// t[i][j][a][b] = <ab||ij> / (e_i + e_j - e_a - e_b) = conj <ij||ab> / (...)
// (g = <ij||ab>, [i][j][a][b]; the factors are Hermitian)
__global__ void mp2_kernel(int64_t o, int64_t v, const double2* __restrict__ g, const double* __restrict__ eps,
                           double2* __restrict__ t) {
  int64_t n = o * o * v * v;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = k % v, r = k / v;
    int64_t a = r % v;
    r /= v;
    int64_t j = r % o, i = r / o;
    double d = eps[i] + eps[j] - eps[o + a] - eps[o + b];
    double2 x = g[k];
    t[k] = (i == j || a == b) ? double2{0.0, 0.0} : double2{x.x / d, -x.y / d};
  }
}

// tA1[i][a] = s1[i][a] / (Haa[a] - Hii[i] + w)
__global__ void fnspp_singles_kernel(int64_t o, int64_t v, const double* __restrict__ Hii,
                                     const double* __restrict__ Haa, double w, const double2* __restrict__ s1,
                                     double2* __restrict__ t1) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < o * v; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / v, a = k % v;
    const double d = Haa[a] - Hii[i] + w;
    t1[k] = {s1[k].x / d, s1[k].y / d};
  }
}

// One chunk of pairs p = i*o + j in [p0, p0 + np) of a doubles tensor
// s[p][a][c], written as X[a][p - p0][c] and Xc = conj X: the row layout in
// which D[a][b] += sum_(p,c) X[a][(p,c)] Xc[b][(p,c)] is one GEMM.  With
// Hii set, the values are first divided by Haa[a] + Haa[c] - Hii[i] - Hii[j] + w
// (tA2, zero where i = j or a = c).
__global__ void pair_chunk_kernel(int64_t o, int64_t v, int64_t p0, int64_t np, const double2* __restrict__ s,
                                  const double* __restrict__ Hii, const double* __restrict__ Haa, double w,
                                  double2* __restrict__ X, double2* __restrict__ Xc) {
  const int64_t n = np * v * v;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = k % v, r = k / v;
    const int64_t pp = r % np, a = r / np;
    const int64_t p = p0 + pp;
    double2 x = s[(p * v + a) * v + c];
    if (Hii) {
      const int64_t i = p / o, j = p % o;
      if (i == j || a == c) {
        x = {0.0, 0.0};
      } else {
        const double d = Haa[a] + Haa[c] - Hii[i] - Hii[j] + w;
        x = {x.x / d, x.y / d};
      }
    }
    X[k] = x;
    Xc[k] = {x.x, -x.y};
  }
}

// part[y][a] = Re sum_{r = y, y + gridDim.y, ...} x[r][a] y[r][a] (rows x cols)
__global__ void col_dot_kernel(int64_t rows, int64_t cols, const double2* __restrict__ x,
                               const double2* __restrict__ y, double* __restrict__ part) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= cols) return;
  double acc = 0.0;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const double2 p = x[r * cols + a], q = y[r * cols + a];
    acc += p.x * q.x - p.y * q.y;
  }
  part[(int64_t)blockIdx.y * cols + a] = acc;
}

// out[a] = base[a] + scale * sum_y part[y][a]
__global__ void col_sum_kernel(int64_t nparts, int64_t cols, const double* __restrict__ part,
                               const double* __restrict__ base, double scale, double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= cols) return;
  double acc = 0.0;
  for (int64_t y = 0; y < nparts; ++y) acc += part[y * cols + a];
  out[a] = base[a] + scale * acc;
}

__global__ void conj_kernel(int64_t n, const double2* __restrict__ x, double2* __restrict__ y) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = {x[k].x, -x[k].y};
}

unsigned grid_of(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1 << 20); }

void conj_copy(int64_t n, const void* x, void* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(conj_kernel, dim3(grid_of(n)), dim3(256), 0, st, n, (const double2*)x, (double2*)y);
  HIP_CHECK(hipGetLastError());
}

// Row-major permute of a 2-D or grouped tensor via the generic kernel.
void permute(const void* in, void* out, std::initializer_list<int64_t> dims, std::initializer_list<int64_t> istr,
             hipStream_t st, double bre = 0.0) {
  PermDesc d{};
  d.rank = (int)dims.size();
  int k = 0;
  for (int64_t x : dims) d.dims[k++] = x;
  k = 0;
  for (int64_t x : istr) d.istride[k++] = x;
  launch_permute<double>(in, out, d, 1.0, 0.0, bre, 0.0, st);
}

struct Solver {
  rocblas_handle h = nullptr;
  explicit Solver(hipStream_t st) {
    LRCC_REQUIRE(rocblas_create_handle(&h) == rocblas_status_success, LRCC_E_INTERNAL, "rocblas_create_handle");
    rocblas_set_stream(h, st);
  }
  ~Solver() {
    if (h) rocblas_destroy_handle(h);
  }
  // Eigen-decomposition of a Hermitian n x n matrix held row-major on the
  // device.  Returns eigenvalues (ascending) and, in V (row-major, host),
  // the eigenvectors as columns: H V = V diag(w).
  void eigh(int n, const void* Hdev, std::vector<double>& w, std::vector<cplx>& V, hipStream_t st) {
    DevBuf A, Dv, Ev, info;
    A.ensure((size_t)n * n * 16);
    Dv.ensure(n * 8);
    Ev.ensure(n * 8);
    info.ensure(16);
    // a row-major Hermitian H read column-major is conj(H); its eigenvectors
    // are the conjugates of those of H
    HIP_CHECK(hipMemcpyAsync(A.p, Hdev, (size_t)n * n * 16, hipMemcpyDeviceToDevice, st));
    rocblas_status s = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, n,
                                        (rocblas_double_complex*)A.p, n, Dv.as<double>(), Ev.as<double>(),
                                        (rocblas_int*)info.p);
    LRCC_REQUIRE(s == rocblas_status_success, LRCC_E_INTERNAL, "rocsolver_zheevd failed");
    int inf = 0;
    w.resize(n);
    std::vector<cplx> R((size_t)n * n);
    HIP_CHECK(hipMemcpyAsync(&inf, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(w.data(), Dv.p, n * 8, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(R.data(), A.p, (size_t)n * n * 16, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    LRCC_REQUIRE(inf == 0, LRCC_E_NOCONV, "Hermitian eigensolver did not converge");
    // column k of the column-major result is R[k*n + i]: eigenvector of conj(H)
    V.assign((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k)
      for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = std::conj(R[(size_t)k * n + i]);
  }
};

// X'[Q] = C^H X[Q] C for nq matrices X[Q] (nmo x nmo) with C (nmo x m), all
// row-major on the device.  Y[Q][p][q'] = sum_q X[Q][p][q] C[q][q'] is one
// GEMM over Q*nmo rows; then X'[Q][p'][q'] = sum_p conj(C)[p][p'] Y[Q][p][q'].
void rotate(int64_t nq, int64_t nmo, int64_t m, const void* X, const void* C, void* out, hipStream_t st) {
  DevBuf Y, Yt, Cc, Z;
  Y.ensure((size_t)nq * nmo * m * 16);
  Yt.ensure((size_t)nq * nmo * m * 16);
  Cc.ensure((size_t)nmo * m * 16);
  Z.ensure((size_t)nq * m * m * 16);
  launch_gemm<double>(false, false, nq * nmo, m, nmo, 1.0, 0.0, X, nmo, C, m, 0.0, 0.0, Y.p, m, st);
  // Yt[p][Q][q'] = Y[Q][p][q']
  permute(Y.p, Yt.p, {nmo, nq, m}, {m, nmo * m, 1}, st);
  conj_copy(nmo * m, C, Cc.p, st);
  // Z[p'][Q][q'] = sum_p conj(C)[p][p'] Yt[p][Q][q']
  launch_gemm<double>(true, false, m, nq * m, nmo, 1.0, 0.0, Cc.p, m, Yt.p, nq * m, 0.0, 0.0, Z.p, nq * m, st);
  permute(Z.p, out, {nq, m, m}, {m, nq * m, 1}, st);
  HIP_CHECK(hipStreamSynchronize(st));
}

// Pair densities are formed in chunks of (i, j) pairs of at most this many
// bytes per buffer (LRCC_DENSITY_CHUNK_BYTES overrides it), so that no
// permuted copy of a whole o^2 v^2 tensor is needed.
size_t density_chunk_bytes() {
  static const size_t fixed = size_t(2) << 30;
  const char* e = std::getenv("LRCC_DENSITY_CHUNK_BYTES");
  if (e && *e) {
    const long long b = std::atoll(e);
    if (b > 0) return (size_t)b;
  }
  return fixed;
}

// D[a][b] += alpha sum_{ijc} x_ij^ac conj x_ij^bc for the doubles tensor s
// [i][j][a][c] (x = s, or with Hii/Haa set the first-order amplitudes
// s / (Haa[a] + Haa[c] - Hii[i] - Hii[j] + w)); D row-major v x v.
void pair_density(int64_t o, int64_t v, const void* s, const double* Hii, const double* Haa, double w, double alpha,
                  void* D, DevBuf& X, DevBuf& Xc, hipStream_t st) {
  const int64_t npairs = o * o, per = v * v * 16;
  const int64_t np = std::max<int64_t>(1, std::min<int64_t>(npairs, (int64_t)(density_chunk_bytes() / per)));
  X.ensure(np * per);
  Xc.ensure(np * per);
  for (int64_t p0 = 0; p0 < npairs; p0 += np) {
    const int64_t nc = std::min(np, npairs - p0);
    hipLaunchKernelGGL(pair_chunk_kernel, dim3(grid_of(nc * v * v)), dim3(256), 0, st, o, v, p0, nc,
                       (const double2*)s, Hii, Haa, w, (double2*)X.p, (double2*)Xc.p);
    HIP_CHECK(hipGetLastError());
    launch_gemm<double>(false, true, v, v, nc * v, alpha, 0.0, X.p, nc * v, Xc.p, nc * v, 1.0, 0.0, D, v, st);
  }
}

}  // namespace

// Step 1: MP2 doubles t[i][j][a][b] (Eq. 39) as a full tensor, written into
// the input of the projection program (which reads it in step 3).
static void* mp2_doubles(Context& c) {
  c.ensure_goovv();
  const size_t n2f = (size_t)c.o * c.o * c.v * c.v;
  DevBuf epsd;
  epsd.ensure(c.nmo * 8);
  c.h2d(epsd.p, c.eps.data(), c.nmo * 8);
  void* tm2 = c.x64->ptr(c.P.n_t2);
  hipLaunchKernelGGL(mp2_kernel, dim3(grid_of(n2f)), dim3(256), 0, c.st, c.o, c.v,
                     (const double2*)c.x64->ptr(c.P.m.find("goovv")), epsd.as<double>(), (double2*)tm2);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(c.st));  // before epsd is released
  return tm2;
}

// Steps 1-2: MP2 doubles (full [i][j][a][b] tensor, left in the projection
// program's input) and the Hbar diagonals.
void Context::hbar_diagonals(std::vector<double>& Hii, std::vector<double>& Haa) {
  const int64_t vv = v, oo = o;
  void* tm2 = mp2_doubles(*this);
  // 2. Hbar diagonals: per-i and per-a bilinear sums of t2 with <ij||ab>
  const void* goovv = x64->ptr(P.m.find("goovv"));
  DevBuf dots, wk, part, ev, hd;
  dots.ensure(oo * 16);
  wk.ensure((size_t)oo * 1024 * 16);
  std::vector<cplx> hi(oo);
  // Hii: sum over the row block i of [i][n][e][f]
  launch_batched_dot<double>(oo, oo * vv * vv, tm2, oo * vv * vv, goovv, oo * vv * vv, false, dots.p, wk.p, st);
  HIP_CHECK(hipMemcpyAsync(hi.data(), dots.p, oo * 16, hipMemcpyDeviceToHost, st));
  // Haa: sum over the rows (m, n, f) of column a of [m][n][f][a]
  const int64_t rows = oo * oo * vv, nparts = std::min<int64_t>(rows, 512);
  part.ensure((size_t)nparts * vv * 8);
  ev.ensure(vv * 8);
  hd.ensure(vv * 8);
  h2d(ev.p, eps.data() + o, vv * 8);
  hipLaunchKernelGGL(col_dot_kernel, dim3((unsigned)((vv + 255) / 256), (unsigned)nparts), dim3(256), 0, st, rows, vv,
                     (const double2*)tm2, (const double2*)goovv, part.as<double>());
  HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(col_sum_kernel, dim3((unsigned)((vv + 255) / 256)), dim3(256), 0, st, nparts, vv,
                     part.as<double>(), ev.as<double>(), -0.5, hd.as<double>());
  HIP_CHECK(hipGetLastError());
  Haa.assign(vv, 0.0);
  d2h(Haa.data(), hd.p, vv * 8);
  Hii.assign(oo, 0.0);
  for (int64_t i = 0; i < oo; ++i) Hii[i] = eps[i] + 0.5 * hi[i].real();
}

void Context::fnspp_truncate(const double* om, int nw, double thresh, int keep, int* nvir_out, double* occ_out) {
  require_sizes();
  LRCC_REQUIRE(have_fock, LRCC_E_STATE, "lrcc_load_fock has not been called");
  LRCC_REQUIRE(ncomp > 0, LRCC_E_STATE, "lrcc_load_dipoles has not been called");
  LRCC_REQUIRE(nw >= 1 && om != nullptr, LRCC_E_INVALID, "need at least one frequency");
  LRCC_REQUIRE(keep >= 0 && keep <= v && (keep > 0 || thresh > 0), LRCC_E_INVALID, "bad keep / thresh");
  const int64_t vv = v, oo = o;
  std::vector<double> Hii, Haa;
  hbar_diagonals(Hii, Haa);
  release_goovv_if_alone();  // the projections read the MP2 doubles and A only
  DevBuf Hd;
  Hd.ensure((oo + vv) * 8);
  h2d(Hd.p, Hii.data(), oo * 8);
  h2d((char*)Hd.p + oo * 8, Haa.data(), vv * 8);
  // 3-4. projections per direction, first-order amplitudes per frequency,
  // and the averaged Gram density
  DevBuf Dm, t1A, P1, P1c, X, Xc;
  Dm.ensure(vv * vv * 16);
  launch_fill_zero<double>(Dm.p, vv * vv, st);
  t1A.ensure(oo * vv * 16);
  P1.ensure(oo * vv * 16);
  P1c.ensure(oo * vv * 16);
  const int64_t p0[4] = {0, 0, o, o}, np[4] = {o, o, v, v}, r0[4] = {0, o, 0, o}, nr[4] = {o, v, o, v};
  const double scale = 1.0 / (double)(nw * ncomp);
  for (int c = 0; c < ncomp; ++c) {
    for (int k = 0; k < 4; ++k)
      launch_gather_block(1, nmo, p0[k], np[k], r0[k], nr[k], (const char*)mu.p + c * nmo * nmo * 16,
                          x64->ptr(P.n_A[k]), st);
    x64->run(P.fnspp, 1);
    for (int k = 0; k < nw; ++k) {
      // D[a][b] += s/2 sum_{ijc} t2A[ijac] conj t2A[ijbc], t2A formed chunk by chunk
      pair_density(oo, vv, x64->ptr(P.n_s2), Hd.as<double>(), Hd.as<double>() + oo, om[k], 0.5 * scale, Dm.p, X,
                   Xc, st);
      // D[a][b] += s sum_i t1A[ia] conj t1A[ib]
      hipLaunchKernelGGL(fnspp_singles_kernel, dim3(grid_of(oo * vv)), dim3(256), 0, st, oo, vv, Hd.as<double>(),
                         Hd.as<double>() + oo, om[k], (const double2*)x64->ptr(P.n_s1), (double2*)t1A.p);
      HIP_CHECK(hipGetLastError());
      permute(t1A.p, P1.p, {vv, oo}, {1, vv}, st);  // [a][i]
      conj_copy(oo * vv, P1.p, P1c.p, st);
      launch_gemm<double>(false, true, vv, vv, oo, scale, 0.0, P1.p, oo, P1c.p, oo, 1.0, 0.0, Dm.p, vv, st);
    }
  }
  truncate_by_density(Dm.p, thresh, keep, nvir_out, occ_out);
}

// FNS: steps 5-7 with the ground-state MP2 density D_ab = 1/2 sum_ijc
// t_ij^ac conj t_ij^bc (Eq. 40, read as a Hermitian Gram matrix).
void Context::fns_truncate(double thresh, int keep, int* nvir_out, double* occ_out) {
  require_sizes();
  LRCC_REQUIRE(have_fock, LRCC_E_STATE, "lrcc_load_fock has not been called");
  LRCC_REQUIRE(keep >= 0 && keep <= v && (keep > 0 || thresh > 0), LRCC_E_INVALID, "bad keep / thresh");
  const int64_t vv = v, oo = o;
  DevBuf X, Xc, Dm;
  void* tm2 = mp2_doubles(*this);
  release_goovv_if_alone();
  Dm.ensure(vv * vv * 16);
  launch_fill_zero<double>(Dm.p, vv * vv, st);
  pair_density(oo, vv, tm2, nullptr, nullptr, 0.0, 0.5, Dm.p, X, Xc, st);
  truncate_by_density(Dm.p, thresh, keep, nvir_out, occ_out);
}

// Steps 5-7 from a Hermitian vv density on the device (row-major v x v).
void Context::truncate_by_density(const void* Dmp, double thresh, int keep, int* nvir_out, double* occ_out) {
  const int64_t vv = v;
  // 5. natural spinors, ordered by |n|
  Solver sol(st);
  std::vector<double> nocc;
  std::vector<cplx> Vn;
  sol.eigh((int)vv, Dmp, nocc, Vn, st);
  std::vector<int> order(vv);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::abs(nocc[a]) > std::abs(nocc[b]); });
  int nk = keep;
  if (nk == 0)
    for (int k = 0; k < vv; ++k)
      if (std::abs(nocc[order[k]]) > thresh) ++nk;
  LRCC_REQUIRE(nk >= 2, LRCC_E_INVALID, "fewer than two natural spinors kept");
  if (occ_out)
    for (int k = 0; k < vv; ++k) occ_out[k] = nocc[order[k]];
  std::vector<cplx> Vt((size_t)vv * nk);
  for (int64_t a = 0; a < vv; ++a)
    for (int k = 0; k < nk; ++k) Vt[a * nk + k] = Vn[(size_t)a * vv + order[k]];
  // 6. semicanonical: F~ = V~^H F_vv V~ (F_vv on the device), F~ Z = Z e~, U = V~ Z
  DevBuf Vd, Vc, Fv, Y, Ft, Ud, Zd;
  Vd.ensure(vv * nk * 16);
  Vc.ensure(vv * nk * 16);
  Fv.ensure(vv * vv * 16);
  Y.ensure(vv * nk * 16);
  Ft.ensure((size_t)nk * nk * 16);
  Ud.ensure(vv * nk * 16);
  Zd.ensure((size_t)nk * nk * 16);
  h2d(Vd.p, Vt.data(), vv * nk * 16);
  launch_gather_block(1, nmo, o, v, o, v, fock.p, Fv.p, st);
  launch_gemm<double>(false, false, vv, nk, vv, 1.0, 0.0, Fv.p, vv, Vd.p, nk, 0.0, 0.0, Y.p, nk, st);
  conj_copy(vv * nk, Vd.p, Vc.p, st);
  launch_gemm<double>(true, false, nk, nk, vv, 1.0, 0.0, Vc.p, nk, Y.p, nk, 0.0, 0.0, Ft.p, nk, st);
  std::vector<double> et;
  std::vector<cplx> Z;
  sol.eigh(nk, Ft.p, et, Z, st);
  h2d(Zd.p, Z.data(), (size_t)nk * nk * 16);
  launch_gemm<double>(false, false, vv, nk, nk, 1.0, 0.0, Vd.p, nk, Zd.p, nk, 0.0, 0.0, Ud.p, nk, st);
  // 7. C = diag(1_occ, U) and the rotated inputs
  const int64_t m = o + nk;
  std::vector<cplx> Uh((size_t)vv * nk), C((size_t)nmo * m, 0.0);
  d2h(Uh.data(), Ud.p, vv * nk * 16);
  for (int64_t i = 0; i < o; ++i) C[i * m + i] = 1.0;
  for (int64_t a = 0; a < vv; ++a)
    for (int k = 0; k < nk; ++k) C[(o + a) * m + o + k] = Uh[a * nk + k];
  DevBuf Cd, Bn, Fn, Mn;
  Cd.ensure((size_t)nmo * m * 16);
  h2d(Cd.p, C.data(), (size_t)nmo * m * 16);
  Bn.ensure((size_t)naux * m * m * 16);
  Fn.ensure((size_t)m * m * 16);
  Mn.ensure((size_t)ncomp * m * m * 16);
  rotate(naux, nmo, m, B.p, Cd.p, Bn.p, st);
  rotate(1, nmo, m, fock.p, Cd.p, Fn.p, st);
  rotate(ncomp, nmo, m, mu.p, Cd.p, Mn.p, st);
  const int nc = ncomp;
  const int64_t na = naux;
  load_df((int)o, nk, (int)na, Bn.p, LRCC_DEVICE);
  load_fock(Fn.p, LRCC_DEVICE);
  load_dipoles(nc, Mn.p, LRCC_DEVICE);
  if (nvir_out) *nvir_out = nk;
}

// MP2-level energy and polarizability in the current virtual space, the
// ingredients of the corrections of Eqs. 51-54 (full minus truncated space).
// Reading of the MP2-level response function (built, per the paper, from
// the MP2 amplitudes and the perturbed amplitudes of Eqs. 46-47):
//   t(1) = -Omega(0)/D and lambda(1) = -eta0(0)/D (first Jacobi steps of the
//   T and Lambda equations; Eq. 39 for a diagonal Fock matrix),
//   E_MP2 = E(t(1)),
//   X^B(+-w) = -xi^B(t(1)) / (Dbar -/+ w), Dbar from the Hbar diagonals of
//   Eqs. 49-50 (the Jacobian replaced by that diagonal, as in Eqs. 46-47),
//   alpha from Eq. 36 at (t(1), lambda(1)).
// All in FP64.  The context's T and Lambda are restored afterwards; X, Y and
// the last alpha are not touched.
void Context::mp2_response(int nw, const double* om, cplx& emp2, std::vector<cplx>& al) {
  require_sizes();
  ensure_integrals();
  LRCC_REQUIRE(have_fock, LRCC_E_STATE, "lrcc_load_fock has not been called");
  LRCC_REQUIRE(ncomp > 0, LRCC_E_STATE, "lrcc_load_dipoles has not been called");
  LRCC_REQUIRE(nw >= 1 && om != nullptr, LRCC_E_INVALID, "need at least one frequency");
  const size_t vb = n * 16;
  const int nrhs = nw * ncomp;
  // Dbar (packed like D) from the Hbar diagonals
  std::vector<double> Hii, Haa;
  hbar_diagonals(Hii, Haa);
  std::vector<double> hb(Hii);
  hb.insert(hb.end(), Haa.begin(), Haa.end());
  DevBuf hbd, Dbar;
  hbd.ensure(nmo * 8);
  Dbar.ensure(n * 8);
  h2d(hbd.p, hb.data(), nmo * 8);
  launch_denominators(o, v, hbd.as<double>(), Dbar.as<double>(), st);
  {
    std::vector<double> hD(n);
    HIP_CHECK(hipMemcpyAsync(hD.data(), Dbar.p, n * 8, hipMemcpyDeviceToHost, st));
    sync();
    for (int k = 0; k < nw; ++k)
      for (int64_t i = 0; i < n; ++i)
        LRCC_REQUIRE(std::abs(hD[i] - std::abs(om[k])) >= 1e-8, LRCC_E_SINGULAR,
                     "frequency " + std::to_string(om[k]) + " lies on an Hbar denominator pole");
  }
  // keep the context's amplitudes; primal intermediates are recomputed later
  DevBuf ts, ls;
  const bool had_t = have_t, had_lam = have_lam;
  if (had_t) HIP_CHECK(hipMemcpyAsync(ts.ensure(vb), t.p, vb, hipMemcpyDeviceToDevice, st));
  if (had_lam) HIP_CHECK(hipMemcpyAsync(ls.ensure(vb), lam.p, vb, hipMemcpyDeviceToDevice, st));
  auto invalidate = [&]() {
    primal64 = primal32 = 0;
    ring64 = ring32 = 0;
    gradL_ready = gradL32_ready = 0;
  };
  struct Restore {
    Context& c;
    DevBuf &ts, &ls;
    bool ht, hl;
    size_t vb;
    ~Restore() {
      if (ht) (void)hipMemcpyAsync(c.t.p, ts.p, vb, hipMemcpyDeviceToDevice, c.st);
      if (hl) (void)hipMemcpyAsync(c.lam.p, ls.p, vb, hipMemcpyDeviceToDevice, c.st);
      (void)hipStreamSynchronize(c.st);
      c.have_t = ht;
      c.have_lam = hl;
      c.primal64 = c.primal32 = 0;
      c.ring64 = c.ring32 = 0;
      c.gradL_ready = c.gradL32_ready = 0;
    }
  } restore{*this, ts, ls, had_t, had_lam, vb};
  // Omega(0) and eta0(0)
  DevBuf R, e0;
  R.ensure(vb);
  e0.ensure(vb);
  t.ensure(vb);
  launch_fill_zero<double>(t.p, n, st);
  have_t = true;
  invalidate();
  residual64(t.p, R.p, nullptr);
  x64->run(P.eta0, 1);
  launch_copy_rows<double, double>(1, n1, x64->ptr(P.e_gt1), n1, e0.p, n, st);
  launch_copy_rows<double, double>(1, n2, x64->ptr(P.e_gt2p), n2, (char*)e0.p + n1 * 16, n, st);
  // t(1), lambda(1) and E_MP2 = E(t(1))
  launch_jacobi(1, n, D.as<double>(), nullptr, nullptr, R.p, t.p, nullptr, st);
  lam.ensure(vb);
  launch_jacobi(1, n, D.as<double>(), nullptr, nullptr, e0.p, lam.p, nullptr, st);
  have_lam = true;
  invalidate();
  residual64(t.p, R.p, &emp2);
  // xi^B, eta^B at (t(1), lambda(1)); X^B(+-w) on the Hbar diagonal
  DevBuf xiB, etaB, Xp, Xm, shp, shm;
  xiB.ensure(ncomp * vb);
  etaB.ensure(ncomp * vb);
  xi_vectors(xiB.p);
  std::vector<int> comps(ncomp);
  for (int c = 0; c < ncomp; ++c) comps[c] = c;
  hvp(ncomp, comps.data(), nullptr, etaB.p);
  Xp.ensure(nrhs * vb);
  Xm.ensure(nrhs * vb);
  std::vector<double> sp(nrhs), sm(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    sp[r] = -om[r / ncomp];
    sm[r] = om[r / ncomp];
  }
  shp.ensure(nrhs * 8);
  shm.ensure(nrhs * 8);
  HIP_CHECK(hipMemcpyAsync(shp.p, sp.data(), nrhs * 8, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(shm.p, sm.data(), nrhs * 8, hipMemcpyHostToDevice, st));
  for (int k = 0; k < nw; ++k) {
    launch_jacobi(ncomp, n, Dbar.as<double>(), shp.as<double>() + k * ncomp, nullptr, xiB.p,
                  (char*)Xp.p + (size_t)k * ncomp * vb, nullptr, st);
    launch_jacobi(ncomp, n, Dbar.as<double>(), shm.as<double>() + k * ncomp, nullptr, xiB.p,
                  (char*)Xm.p + (size_t)k * ncomp * vb, nullptr, st);
  }
  alpha_quadratic(nw, rhs_chunk_for(nrhs, 64), Xp.p, Xm.p, etaB.p, 64, al);
}

}  // namespace lrcc
