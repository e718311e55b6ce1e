// extern "C" entry points of liblrcc.so (declared in include/lrcc.h).
// Every call catches all C++ exceptions and maps them to LRCC_E_* codes.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>

#include "context.h"
#include "devmem.h"
#include "kernels.h"

using lrcc::Context;
using lrcc::Error;

struct lrcc_ctx {
  std::unique_ptr<lrcc::Arena> arena;  // caller-owned workspace (outlives impl)
  std::unique_ptr<Context> impl;
  std::string err;
};

static thread_local std::string g_create_error;

namespace lrcc {
// Message of the last failing context-free call on this thread (read with
// lrcc_last_error(NULL)).
void set_call_error(const std::string& msg) { g_create_error = msg; }
}  // namespace lrcc

template <typename F>
static int guard(lrcc_ctx* ctx, F&& f) {
  if (!ctx || !ctx->impl) return LRCC_E_INVALID;
  lrcc::ArenaScope scope(ctx->arena.get());  // every allocation of this call comes from the workspace
  try {
    HIP_CHECK(hipSetDevice(ctx->impl->cfg.device));
    f(*ctx->impl);
    ctx->err.clear();
    return LRCC_OK;
  } catch (const Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return LRCC_E_INTERNAL;
  } catch (...) {
    ctx->err = "unknown error";
    return LRCC_E_INTERNAL;
  }
}

static void to_stats(const lrcc::SolveStats& s, lrcc_stats* o) {
  if (!o) return;
  o->iterations = s.iterations;
  o->converged = s.converged;
  o->residual = s.residual;
  o->seconds = s.seconds;
  o->sigma_evals = s.sigma_evals;
}

static void copy_out(void* dst, const void* src, size_t bytes, int where, hipStream_t st) {
  LRCC_REQUIRE(dst != nullptr, LRCC_E_INVALID, "output pointer is null");
  LRCC_REQUIRE(where == LRCC_HOST || where == LRCC_DEVICE, LRCC_E_INVALID, "where must be LRCC_HOST or LRCC_DEVICE");
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, where == LRCC_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
  HIP_CHECK(hipStreamSynchronize(st));
}

extern "C" {

void lrcc_default_config(lrcc_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->device = 0;
  cfg->stream = nullptr;
  cfg->precision = LRCC_FP64;
  cfg->tol_residual = 1e-10;
  cfg->maxit = 100;
  cfg->diis_size = 8;
  cfg->rhs_chunk = 0;
  cfg->autotune = 1;
  cfg->verbose = 0;
  const char* g = std::getenv("LRCC_GRAPHS");  // default override, e.g. for profiling launch by launch
  cfg->graphs = (g && g[0] == '0') ? 0 : 1;
  cfg->ladder_mode = LRCC_LADDER_FULL;
  cfg->ladder_mode_fp64 = -1;
  cfg->memory_mode = LRCC_MEMORY_AUTO;
  cfg->ring_factored = -1;
  cfg->keep_response = 1;
}

int lrcc_create(lrcc_ctx** out, const lrcc_config* cfg) {
  if (!out) return LRCC_E_INVALID;
  *out = nullptr;
  try {
    lrcc_config c;
    lrcc_default_config(&c);
    if (cfg) c = *cfg;
    LRCC_REQUIRE(c.precision == LRCC_FP64 || c.precision == LRCC_MIXED, LRCC_E_INVALID, "bad precision");
    LRCC_REQUIRE(c.ladder_mode >= LRCC_LADDER_FULL && c.ladder_mode <= LRCC_LADDER_TRIANGLE, LRCC_E_INVALID,
                 "bad ladder_mode");
    LRCC_REQUIRE(c.ladder_mode_fp64 >= -1 && c.ladder_mode_fp64 <= LRCC_LADDER_TRIANGLE, LRCC_E_INVALID,
                 "bad ladder_mode_fp64");
    LRCC_REQUIRE(c.memory_mode >= LRCC_MEMORY_AUTO && c.memory_mode <= LRCC_MEMORY_LEAN, LRCC_E_INVALID,
                 "bad memory_mode");
    LRCC_REQUIRE(c.ring_factored >= -1 && c.ring_factored <= 1, LRCC_E_INVALID, "bad ring_factored");
    LRCC_REQUIRE(c.keep_response == 0 || c.keep_response == 1, LRCC_E_INVALID, "bad keep_response");
    LRCC_REQUIRE(c.tol_residual > 0 && c.maxit > 0 && c.diis_size >= 0 && c.diis_size <= 32 && c.rhs_chunk >= 0,
                 LRCC_E_INVALID, "bad tolerance, iteration limit, DIIS size or chunk");
    int ndev = 0;
    HIP_CHECK(hipGetDeviceCount(&ndev));
    LRCC_REQUIRE(c.device >= 0 && c.device < ndev, LRCC_E_INVALID, "no such HIP device");
    std::unique_ptr<lrcc_ctx> ctx(new lrcc_ctx);
    HIP_CHECK(hipSetDevice(c.device));
    lrcc::set_gemm_autotune(c.autotune != 0);
    ctx->impl.reset(new Context(c));
    *out = ctx.release();
    g_create_error.clear();
    return LRCC_OK;
  } catch (const Error& e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return LRCC_E_INTERNAL;
  }
}

void lrcc_destroy(lrcc_ctx* ctx) {
  if (!ctx) return;
  try {
    lrcc::ArenaScope scope(ctx->arena.get());  // workspace blocks go back to the workspace
    if (ctx->impl) {
      (void)hipSetDevice(ctx->impl->cfg.device);
      if (ctx->arena) (void)hipStreamSynchronize(ctx->impl->st);  // the caller may free the buffer next
    }
    ctx->impl.reset();
  } catch (...) {
  }
  delete ctx;
}

const char* lrcc_last_error(const lrcc_ctx* ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

int lrcc_load_df(lrcc_ctx* ctx, int nocc, int nvir, int naux, const void* B, int where) {
  return guard(ctx, [&](Context& c) { c.load_df(nocc, nvir, naux, B, where); });
}

int lrcc_load_fock(lrcc_ctx* ctx, const void* F, int where) {
  return guard(ctx, [&](Context& c) { c.load_fock(F, where); });
}

int lrcc_load_dipoles(lrcc_ctx* ctx, int ncomp, const void* mu, int where) {
  return guard(ctx, [&](Context& c) { c.load_dipoles(ncomp, mu, where); });
}

int lrcc_fnspp_truncate(lrcc_ctx* ctx, const double* omegas, int nw, double thresh, int keep, int* nvir_out,
                        double* occ_out) {
  return guard(ctx, [&](Context& c) { c.fnspp_truncate(omegas, nw, thresh, keep, nvir_out, occ_out); });
}

int lrcc_fns_truncate(lrcc_ctx* ctx, double thresh, int keep, int* nvir_out, double* occ_out) {
  return guard(ctx, [&](Context& c) { c.fns_truncate(thresh, keep, nvir_out, occ_out); });
}

int lrcc_solve_ground(lrcc_ctx* ctx, double ecorr[2], lrcc_stats* stats) {
  return guard(ctx, [&](Context& c) {
    lrcc::SolveStats s;
    c.kt.clear();
    try {
      c.solve_ground(ecorr, s);
    } catch (...) {
      to_stats(s, stats);
      c.collect_times();
      throw;
    }
    to_stats(s, stats);
    c.collect_times();
  });
}

int lrcc_solve_lambda(lrcc_ctx* ctx, lrcc_stats* stats) {
  return guard(ctx, [&](Context& c) {
    lrcc::SolveStats s;
    c.kt.clear();
    try {
      c.solve_lambda(s);
    } catch (...) {
      to_stats(s, stats);
      c.collect_times();
      throw;
    }
    to_stats(s, stats);
    c.collect_times();
  });
}

static int solve_response_route(lrcc_ctx* ctx, int nw, const double* omegas, lrcc_stats* per_rhs, bool quadratic) {
  return guard(ctx, [&](Context& c) {
    std::vector<lrcc::SolveStats> per;
    c.kt.clear();
    auto out = [&]() {
      if (per_rhs)
        for (size_t k = 0; k < per.size(); ++k) to_stats(per[k], per_rhs + k);
      c.collect_times();
    };
    try {
      c.solve_response(nw, omegas, per, quadratic);
    } catch (...) {
      out();
      throw;
    }
    out();
  });
}

int lrcc_solve_response(lrcc_ctx* ctx, int nw, const double* omegas, lrcc_stats* per_rhs) {
  return solve_response_route(ctx, nw, omegas, per_rhs, false);
}

int lrcc_solve_response_quadratic(lrcc_ctx* ctx, int nw, const double* omegas, lrcc_stats* per_rhs) {
  return solve_response_route(ctx, nw, omegas, per_rhs, true);
}

int lrcc_mp2_response(lrcc_ctx* ctx, int nw, const double* omegas, double emp2[2], void* alpha, int where) {
  return guard(ctx, [&](Context& c) {
    LRCC_REQUIRE(emp2 != nullptr && alpha != nullptr, LRCC_E_INVALID, "null output");
    LRCC_REQUIRE(where == LRCC_HOST || where == LRCC_DEVICE, LRCC_E_INVALID, "bad where");
    lrcc::cplx e = 0;
    std::vector<lrcc::cplx> al;
    c.mp2_response(nw, omegas, e, al);
    emp2[0] = e.real();
    emp2[1] = e.imag();
    if (where == LRCC_HOST) {
      std::memcpy(alpha, al.data(), al.size() * 16);
    } else {
      HIP_CHECK(hipMemcpyAsync(alpha, al.data(), al.size() * 16, hipMemcpyHostToDevice, c.st));
      c.sync();
    }
  });
}

int lrcc_get_alpha(lrcc_ctx* ctx, void* alpha, int where) {
  return guard(ctx, [&](Context& c) {
    LRCC_REQUIRE(c.have_alpha, LRCC_E_STATE, "no polarizability (call lrcc_solve_response first)");
    LRCC_REQUIRE(alpha != nullptr, LRCC_E_INVALID, "alpha is null");
    size_t bytes = c.alpha.size() * 16;
    if (where == LRCC_HOST) {
      std::memcpy(alpha, c.alpha.data(), bytes);
    } else {
      LRCC_REQUIRE(where == LRCC_DEVICE, LRCC_E_INVALID, "bad where");
      HIP_CHECK(hipMemcpyAsync(alpha, c.alpha.data(), bytes, hipMemcpyHostToDevice, c.st));
      c.sync();
    }
  });
}

int lrcc_sigma(lrcc_ctx* ctx, int side, int nvec, const double* shifts, const void* in, void* out, int where,
               int precision) {
  return guard(ctx, [&](Context& c) {
    c.require_sizes();
    LRCC_REQUIRE(in && out, LRCC_E_INVALID, "null vector");
    LRCC_REQUIRE(nvec >= 1, LRCC_E_INVALID, "nvec must be >= 1");
    LRCC_REQUIRE(where == LRCC_HOST || where == LRCC_DEVICE, LRCC_E_INVALID, "bad where");
    LRCC_REQUIRE(precision == LRCC_FP64 || precision == LRCC_MIXED, LRCC_E_INVALID, "bad precision");
    LRCC_REQUIRE(c.have_fock, LRCC_E_STATE, "lrcc_load_fock has not been called");
    const size_t vb = c.n * 16;
    // device vectors are used in place (an aliased output goes through a copy)
    lrcc::DevBuf din, dout;
    const void* src = in;
    void* dst = out;
    if (where == LRCC_HOST || in == out) {
      din.ensure(nvec * vb);
      HIP_CHECK(hipMemcpyAsync(din.p, in, nvec * vb,
                               where == LRCC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, c.st));
      src = din.p;
    }
    if (where == LRCC_HOST) dst = dout.ensure(nvec * vb);
    c.kt.clear();
    if (side == LRCC_SIDE_RESIDUAL) {
      LRCC_REQUIRE(nvec == 1, LRCC_E_INVALID, "the residual takes one vector");
      c.residual64(src, dst, nullptr);
    } else {
      LRCC_REQUIRE(side == LRCC_SIDE_RIGHT || side == LRCC_SIDE_LEFT, LRCC_E_INVALID, "bad side");
      lrcc::Side sd = side == LRCC_SIDE_RIGHT ? lrcc::Side::Right : lrcc::Side::Left;
      const int prec = precision == LRCC_FP64 ? 64 : 32;
      const int chunk = c.sigma_chunk(sd, nvec, prec);
      for (int r0 = 0; r0 < nvec; r0 += chunk) {
        const int nb = std::min(chunk, nvec - r0);
        const char* s = (const char*)src + (size_t)r0 * vb;
        char* d = (char*)dst + (size_t)r0 * vb;
        if (prec == 64) {
          c.sigma64(sd, nb, s, d);
        } else {
          // FP32 coupling products plus the FP64 diagonal D X
          void* s32 = c.sig32.ensure(nb * c.n * 8);
          c.sigma32(sd, nb, s, s32);
          lrcc::launch_residual<float>(nb, c.n, s32, nullptr, s, nullptr, 0, d, c.st, c.D.as<double>());
        }
      }
      if (shifts) {
        void* shd = c.shbuf.ensure(nvec * 8);
        HIP_CHECK(hipMemcpyAsync(shd, shifts, nvec * 8, hipMemcpyHostToDevice, c.st));
        lrcc::launch_residual<double>(nvec, c.n, dst, (const double*)shd, src, nullptr, 0, dst, c.st);
      }
    }
    if (where == LRCC_HOST) copy_out(out, dst, nvec * vb, where, c.st);
    c.collect_times();
  });
}

int64_t lrcc_amplitude_length(const lrcc_ctx* ctx) { return (ctx && ctx->impl) ? ctx->impl->n : 0; }

int lrcc_get_amplitudes(lrcc_ctx* ctx, int which, int idx, void* out, int where) {
  return guard(ctx, [&](Context& c) {
    c.require_sizes();
    const size_t vb = c.n * 16;
    const void* src = nullptr;
    if (which == LRCC_AMP_T) {
      LRCC_REQUIRE(c.have_t, LRCC_E_STATE, "no T amplitudes");
      src = c.t.p;
    } else if (which == LRCC_AMP_LAMBDA) {
      LRCC_REQUIRE(c.have_lam, LRCC_E_STATE, "no Lambda amplitudes");
      src = c.lam.p;
    } else {
      LRCC_REQUIRE(which == LRCC_AMP_X || which == LRCC_AMP_Y || which == LRCC_AMP_XMINUS, LRCC_E_INVALID,
                   "bad amplitude kind");
      LRCC_REQUIRE(c.have_alpha, LRCC_E_STATE, "no response amplitudes");
      LRCC_REQUIRE(which != LRCC_AMP_Y || c.response_route == 35, LRCC_E_STATE,
                   "no Y amplitudes (the last response solve took the Eq. 36 route)");
      LRCC_REQUIRE(which != LRCC_AMP_XMINUS || c.response_route == 36, LRCC_E_STATE,
                   "no X(-w) amplitudes (the last response solve took the Eq. 35 route)");
      int nr = (int)c.omegas.size() * c.ncomp;
      LRCC_REQUIRE(idx >= 0 && idx < nr, LRCC_E_INVALID, "bad right-hand-side index");
      LRCC_REQUIRE(idx >= c.resp_first && idx < c.resp_first + c.resp_count, LRCC_E_STATE,
                   "amplitudes of right-hand side " + std::to_string(idx) +
                       " were not kept (lrcc_config.keep_response = 0 keeps the last frequency group only)");
      src = (const char*)(which == LRCC_AMP_X ? c.X.p : c.Y.p) + (size_t)(idx - c.resp_first) * vb;
    }
    copy_out(out, src, vb, where, c.st);
  });
}

int lrcc_set_amplitudes(lrcc_ctx* ctx, int which, int idx, const void* in, int where) {
  return guard(ctx, [&](Context& c) {
    (void)idx;
    c.require_sizes();
    LRCC_REQUIRE(c.have_fock, LRCC_E_STATE, "lrcc_load_fock has not been called");
    LRCC_REQUIRE(in != nullptr, LRCC_E_INVALID, "null input");
    LRCC_REQUIRE(where == LRCC_HOST || where == LRCC_DEVICE, LRCC_E_INVALID, "bad where");
    const size_t vb = c.n * 16;
    auto kind = where == LRCC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (which == LRCC_AMP_T) {
      c.t.ensure(vb);
      HIP_CHECK(hipMemcpyAsync(c.t.p, in, vb, kind, c.st));
      c.sync();
      c.have_t = true;
      c.have_lam = c.have_alpha = false;
      c.primal64 = c.primal32 = c.gradL_ready = 0;
      c.ring64 = c.ring32 = 0;
    } else if (which == LRCC_AMP_LAMBDA) {
      LRCC_REQUIRE(c.have_t, LRCC_E_STATE, "set T before Lambda");
      c.lam.ensure(vb);
      HIP_CHECK(hipMemcpyAsync(c.lam.p, in, vb, kind, c.st));
      c.sync();
      c.have_lam = true;
      c.gradL_ready = 0;
      c.have_alpha = false;
    } else {
      throw Error(LRCC_E_INVALID, "only T and Lambda can be set");
    }
  });
}

int lrcc_gemm(int precision, int transa, int transb, int64_t m, int64_t n, int64_t k, const double alpha[2],
              const void* A, int64_t lda, const void* B, int64_t ldb, const double beta[2], void* C, int64_t ldc,
              void* stream) {
  try {
    LRCC_REQUIRE(alpha && beta && A && B && C, LRCC_E_INVALID, "null argument");
    LRCC_REQUIRE(precision == LRCC_FP64 || precision == LRCC_MIXED, LRCC_E_INVALID, "bad precision");
    LRCC_REQUIRE(m >= 0 && n >= 0 && k >= 0, LRCC_E_INVALID, "negative size");
    LRCC_REQUIRE(lda >= (transa ? m : k) && ldb >= (transb ? k : n) && ldc >= n, LRCC_E_INVALID, "leading dimension");
    // deep products with few output tiles are split over K into a temporary workspace
    const size_t wsb = precision == LRCC_FP64 ? lrcc::gemm_workspace_bytes<double>(m, n, k)
                                              : lrcc::gemm_workspace_bytes<float>(m, n, k);
    lrcc::DevBuf ws;
    if (wsb) ws.ensure(wsb);
    if (precision == LRCC_FP64)
      lrcc::launch_gemm<double>(transa != 0, transb != 0, m, n, k, alpha[0], alpha[1], A, lda, B, ldb, beta[0],
                                beta[1], C, ldc, (hipStream_t)stream, 0, ws.p, wsb);
    else
      lrcc::launch_gemm<float>(transa != 0, transb != 0, m, n, k, alpha[0], alpha[1], A, lda, B, ldb, beta[0],
                               beta[1], C, ldc, (hipStream_t)stream, 0, ws.p, wsb);
    if (wsb) HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));  // before the workspace is freed
    return LRCC_OK;
  } catch (const Error& e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return LRCC_E_INTERNAL;
  }
}

int lrcc_gemm_set_tile(int tile) {
  if (tile < -1 || tile > 4) {
    g_create_error = "tile must be -1..4";
    return LRCC_E_INVALID;
  }
  lrcc::set_gemm_tile(tile);
  return LRCC_OK;
}

int lrcc_gemm_tuned_tile(int precision, int transa, int transb, int64_t m, int64_t n, int64_t k, int ladder) {
  if ((precision != LRCC_FP64 && precision != LRCC_MIXED) || m < 1 || n < 1 || k < 1) return -1;
  return lrcc::gemm_tuned_tile(precision == LRCC_FP64 ? 64 : 32, transa != 0, transb != 0, ladder ? 1 : 0, m, n, k);
}

int64_t lrcc_program_text(int which, char* buf, int64_t cap) {
  try {
    static lrcc::CcPrograms P = [] {
      lrcc::CcPrograms p;
      lrcc::build_programs(p);
      return p;
    }();
    const lrcc::OpList* lists[] = {&P.residual, &P.right, &P.left,       &P.xi,      &P.hvp,   &P.eta0,
                                   &P.gradL,    &P.hvpt, &P.fnspp, &P.ring_setup, &P.right_f, &P.left_f};
    if (which < 0 || which > 11) return -1;
    std::string s = lrcc::serialize(P.m, *lists[which]);
    if (buf && cap > 0) {
      int64_t k = std::min<int64_t>(cap - 1, (int64_t)s.size());
      std::memcpy(buf, s.data(), k);
      buf[k] = 0;
    }
    return (int64_t)s.size();
  } catch (...) {
    return -1;
  }
}

int lrcc_kernel_time(lrcc_ctx* ctx, int cls, double* ms, int64_t* launches, double* flops) {
  return guard(ctx, [&](Context& c) {
    LRCC_REQUIRE(cls >= 0 && cls <= 2, LRCC_E_INVALID, "bad class");
    if (ms) *ms = c.kt.ms[cls];
    if (launches) *launches = c.kt.launches[cls];
    if (flops) *flops = c.kt.flops[cls];
  });
}

int lrcc_set_timing(lrcc_ctx* ctx, int on) {
  return guard(ctx, [&](Context& c) {
    c.timing = on != 0;
    if (c.x64) c.x64->set_timing(c.timing);
    if (c.x32) c.x32->set_timing(c.timing);
  });
}

int lrcc_graph_stats(lrcc_ctx* ctx, int64_t* captures, int64_t* replays) {
  return guard(ctx, [&](Context& c) {
    int64_t cap = 0, rep = 0;
    if (c.x64) cap += c.x64->graph_captures(), rep += c.x64->graph_replays();
    if (c.x32) cap += c.x32->graph_captures(), rep += c.x32->graph_replays();
    cap += c.iter_captures;
    rep += c.iter_replays;
    if (captures) *captures = cap;
    if (replays) *replays = rep;
  });
}

size_t lrcc_workspace_bytes(const lrcc_config* cfg, int nocc, int nvir, int naux, int nrhs) {
  try {
    lrcc_config c;
    lrcc_default_config(&c);
    if (cfg) c = *cfg;
    return lrcc::workspace_estimate(c, nocc, nvir, naux, nrhs);
  } catch (...) {
    return 0;
  }
}

int lrcc_set_workspace(lrcc_ctx* ctx, void* dptr, size_t bytes) {
  if (!ctx || !ctx->impl) return LRCC_E_INVALID;
  if (!dptr || bytes < (size_t(1) << 20)) {
    ctx->err = "workspace must be a device pointer to at least 1 MiB";
    return LRCC_E_INVALID;
  }
  if (ctx->arena || ctx->impl->n != 0) {
    ctx->err = "lrcc_set_workspace must come once, before lrcc_load_df";
    return LRCC_E_STATE;
  }
  ctx->arena.reset(new lrcc::Arena(dptr, bytes));
  ctx->err.clear();
  return LRCC_OK;
}

size_t lrcc_workspace_peak(const lrcc_ctx* ctx) { return (ctx && ctx->arena) ? ctx->arena->peak() : 0; }

int lrcc_trim_memory(void) {
  try {
    lrcc::dev_trim();
    return LRCC_OK;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return LRCC_E_HIP;
  }
}

const char* lrcc_build_info(void) { return "lrcc gfx950 HIP " __DATE__ " " __TIME__; }

}  // extern "C"

namespace lrcc {

void Context::collect_times() {
  if (x64) x64->collect_times(kt);
  if (x32) x32->collect_times(kt);
}

}  // namespace lrcc
