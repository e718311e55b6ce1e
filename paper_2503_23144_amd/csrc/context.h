// Solver context: device data of one system and the T, Lambda, X, Y solves.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "devmem.h"
#include "common.h"
#include "program.h"
#include "runtime.h"

namespace lrcc {

using cplx = std::complex<double>;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  void* ensure(size_t b) {
    if (b > bytes) {
      release();
      p = dev_alloc(std::max<size_t>(b, 16));
      bytes = std::max<size_t>(b, 16);
    }
    return p;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

struct SolveStats {
  int iterations = 0;
  int converged = 0;
  double residual = 0;
  double seconds = 0;
  int64_t sigma_evals = 0;
};

enum class Side { Right, Left };

// Device bytes the pipeline needs with batches of up to nrhs right-hand sides.
size_t workspace_estimate(const lrcc_config& cfg, int o, int v, int naux, int nrhs);
// Whether an executor of precision prec (64 or 32) takes the factored ring
// terms (lrcc_config.ring_factored; automatic by the size of Z1).
bool ring_factored_for(const lrcc_config& cfg, int o, int v, int prec);

struct Context {
  explicit Context(const lrcc_config& cfg);
  ~Context();

  lrcc_config cfg;
  hipStream_t st = nullptr;
  hipStream_t cst = nullptr;  // private stream that whole solver iterations are captured on
  int64_t iter_captures = 0, iter_replays = 0;  // whole-iteration graphs of the solvers
  std::string err;

  // sizes
  int64_t o = 0, v = 0, naux = 0, nmo = 0, n1 = 0, n2 = 0, n = 0;
  Dims dims;
  CcPrograms P;
  std::unique_ptr<Executor<double>> x64;
  std::unique_ptr<Executor<float>> x32;

  bool lean = false;         // LRCC_MEMORY_LEAN in effect (decided by load_df)
  int mode64 = 0, mode32 = 0;  // storage of W for the FP64 and the FP32 executor (LRCC_LADDER_*)
  DevBuf B, fock, mu, D;     // FP64 inputs; D = real denominators [n]
  DevBuf L64, L32;           // DF-direct ladder: virtual-virtual block of B [naux][v][v] per precision
  DevBuf Tri64, Tri32;       // Hermitian-triangle ladder: row blocks of W's upper triangle per precision
  std::vector<int64_t> tri_bnd, tri_offs;  // block boundaries (over b) and offsets (complex elements)
  template <typename T>
  std::vector<typename Executor<T>::TriBlock> tri_blocks(const void* base) const;
  std::vector<double> eps;   // Fock diagonal (host)
  int ncomp = 0;
  bool have_fock = false;
  DevBuf t, t32, lam, lam32;
  bool have_t = false, have_lam = false;
  int primal64 = 0, primal32 = 0;  // 1 if primal intermediates are at the current t
  int ring64 = 0, ring32 = 0;      // 1 if Z1, Z2 of the factored ring terms are at the current t
  // The factored ring terms in the FP64 (prec 64) or FP32 executor's right
  // and left products (lrcc_config.ring_factored), and the programs to run.
  bool factored(int prec) const;
  const OpList& right_prog(int prec) const { return factored(prec) ? P.right_f : P.right; }
  const OpList& left_prog(int prec) const { return factored(prec) ? P.left_f : P.left; }
  int gradL_ready = 0;
  cplx ecorr = 0;

  // response
  std::vector<double> omegas;
  DevBuf X, Y, xi, eta;      // [nrhs][n], [ncomp][n]
  std::vector<cplx> alpha;   // [nw][ncomp][ncomp]
  bool have_alpha = false;

  KernelTimes kt;
  bool timing = false;

  // scratch
  DevBuf work, dotbuf, sig32, shbuf;

  // ---- setup
  void load_df(int nocc, int nvir, int naux_, const void* Bp, int where);
  void load_fock(const void* F, int where);
  void load_dipoles(int nc, const void* m, int where);
  void fnspp_truncate(const double* om, int nw, double thresh, int keep, int* nvir_out, double* occ_out);
  void fns_truncate(double thresh, int keep, int* nvir_out, double* occ_out);
  void truncate_by_density(const void* Dm, double thresh, int keep, int* nvir_out, double* occ_out);

  // ---- solves
  void solve_ground(double ecorr_out[2], SolveStats& s);
  void solve_lambda(SolveStats& s);
  void solve_response(int nw, const double* om, std::vector<SolveStats>& per, bool quadratic = false);
  void alpha_quadratic(int nw, int chunk, const void* Xp, const void* Xm, const void* etaB, int prec,
                       std::vector<cplx>& out);
  // eta^B + F X^B (etaB: [ncomp][n], used on the mixed path)
  void eta_plus_fx(int nb, const int* comp, const void* Xs, void* out, int prec, const void* etaB);
  // MP2-level energy and alpha in the current virtual space (FNS++ corrections)
  void mp2_response(int nw, const double* om, cplx& emp2, std::vector<cplx>& al);
  void hbar_diagonals(std::vector<double>& Hii, std::vector<double>& Haa);
  int response_route = 0;  // 35: X and Y (Eq. 35); 36: X(w) and X(-w) (Eq. 36, X(-w) in Y)
  // X and Y hold the right-hand sides [resp_first, resp_first + resp_count)
  // of the last response solve (all of them unless cfg.keep_response = 0)
  int resp_first = 0, resp_count = 0;
  void response_alpha(int nw, int chunk, bool quadratic, int prec, std::vector<cplx>& out);

  // ---- Jacobian products on device FP64 vectors [nb][n] (in/out may alias no)
  void residual64(const void* tvec, void* R, cplx* E);
  void ensure_primal(int prec);
  void sigma64(Side side, int nb, const void* in, void* out);
  void sigma32(Side side, int nb, const void* in64, void* out32);  // FP64 in, FP32 out
  void xi_vectors(void* out);                                       // [ncomp][n]
  void hvp(int nb, const int* comp, const void* Xdt, void* out);    // eta^B + F X (Xdt may be null)
  void fx32(int nb, const void* X64, void* out32);                  // F X with FP32 products
  void residual32(const void* tvec, void* R);                       // Omega(t) = D t (FP64) + coupling (FP32)
  int gradL32_ready = 0;

  // generic batched linear solve: for r < nb, (op + s_r) x_r = -b_r
  void solve_linear(Side side, int nb, const double* shifts, const void* b, void* x, int prec, double tol,
                    std::vector<SolveStats>& st_out);

  int rhs_chunk_for(int nrhs, int prec);
  int sigma_chunk(Side side, int nvec, int prec);  // right-hand sides per product that fit free memory
  int64_t sigma_count = 0;
  void sync() { HIP_CHECK(hipStreamSynchronize(st)); }
  // Host <-> device copies ordered on the context's stream; they return once
  // the copy is complete (the host buffer may be reused at once).
  void h2d(void* dst, const void* src, size_t bytes) {
    HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    sync();
  }
  void d2h(void* dst, const void* src, size_t bytes) {
    HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    sync();
  }
  void require_sizes() const;
  void upload_fock_blocks();
  void build_integrals();
  void ensure_integrals();  // every block (on first need)
  void ensure_goovv();      // <oo||vv> alone (what truncation needs)
  void release_goovv_if_alone();
  bool ints_built = false, goovv_built = false;
  void reset_solutions();
  void collect_times();
};

}  // namespace lrcc
