// T, Lambda, X(w), Y(w) solves and the polarizability (Section II.A).
//
// All vectors are FP64 on the device.  Each solve is a batched Jacobi
// iteration x <- x - R / (D + s) with the orbital-energy denominators D and
// per right-hand-side shift s, accelerated by DIIS on the preconditioned
// residuals; the residual R, its norm, the update, the DIIS Gram matrix and
// the extrapolation are FP64.  Only the Jacobian product inside R may run in
// FP32 (mixed mode), in which case an outer FP64 residual drives iterative
// refinement: solve (A + s) delta = -R64 with FP32 products, x += delta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>

#include "context.h"
#include "integrals.h"
#include "kernels.h"

namespace lrcc {

static const char* kBlocks[][2] = {{"goooo", "oooo"}, {"gooov", "ooov"}, {"goovv", "oovv"}, {"govvo", "ovvo"},
                                   {"govvv", "ovvv"}, {"gvvoo", "vvoo"}, {"gvvvo", "vvvo"}, {"govoo", "ovoo"}};

// Integral blocks that LRCC_MEMORY_LEAN does not store: <ov||vv> is kept
// only packed over its last pair (govvp), <vv||vo> = -conj <ov||vv> with
// (a, b, c, i) -> (i, c, a, b), and <vv||oo> = conj <oo||vv> transposed
// (<pq||rs> = conj <rs||pq> for Hermitian factors).
static bool lean_block(const char* name) {
  return !std::strcmp(name, "govvv") || !std::strcmp(name, "gvvvo") || !std::strcmp(name, "gvvoo");
}

template <typename T>
static void set_virtuals(Executor<T>& x, const Module& m) {
  typename Executor<T>::VirtualDef d;
  d.src = m.find("govvp");
  d.vl = "wxyz";
  d.sl = "wxyz";  // govvv[w][x][y][z] = govvp[w][x][P(y, z)]
  d.pair_at = 2;
  d.chunk = 0;
  x.set_virtual(m.find("govvv"), d);
  d.sl = "zywx";  // gvvvo[w][x][y][z] = -conj govvp[z][y][P(w, x)]
  d.sre = -1.0;
  d.conj = true;
  d.chunk = 3;
  x.set_virtual(m.find("gvvvo"), d);
  d.src = m.find("goovv");
  d.sl = "yzwx";  // gvvoo[w][x][y][z] = conj goovv[y][z][w][x]
  d.pair_at = -1;
  d.sre = 1.0;
  d.chunk = 2;
  x.set_virtual(m.find("gvvoo"), d);
  const char* e = std::getenv("LRCC_VIRTUAL_CHUNK_BYTES");  // smaller chunks, for tests of the chunked path
  if (e && std::atoll(e) > 0) x.set_virtual_chunk_bytes((size_t)std::atoll(e));
}

static size_t device_total_bytes() {
  size_t fr = 0, tot = 0;
  int n = 0;
  if (hipGetDeviceCount(&n) == hipSuccess && n > 0 && hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0) return tot;
  return size_t(288) * 1000 * 1000 * 1000;  // MI355X
}

// LRCC_MEMORY_AUTO takes the lean layout when the resident one would need
// more than half the device for a single right-hand side.
static bool lean_layout(const lrcc_config& cfg, int o, int v, int naux) {
  if (cfg.memory_mode == LRCC_MEMORY_LEAN) return true;
  if (cfg.memory_mode == LRCC_MEMORY_RESIDENT) return false;
  lrcc_config r = cfg;
  r.memory_mode = LRCC_MEMORY_RESIDENT;
  return (double)workspace_estimate(r, o, v, naux, 1) > 0.5 * (double)device_total_bytes();
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Context::Context(const lrcc_config& c) : cfg(c) {
  HIP_CHECK(hipSetDevice(cfg.device));
  st = (hipStream_t)cfg.stream;
  build_programs(P);
}

Context::~Context() {
  if (st) (void)hipStreamSynchronize(st);
  x64.reset();
  x32.reset();
  if (cst) (void)hipStreamDestroy(cst);
}

// With lrcc_config.ring_factored = -1, an executor forms Z1 of the factored
// ring terms (o v^3 complex elements at its precision) when it takes at most
// this much.
constexpr double kRingFactorMaxBytes = 24.0 * double(size_t(1) << 30);

bool ring_factored_for(const lrcc_config& cfg, int o, int v, int prec) {
  if (cfg.ring_factored >= 0) return cfg.ring_factored == 1;
  return (double)o * v * v * v * (prec == 64 ? 16.0 : 8.0) <= kRingFactorMaxBytes;
}

bool Context::factored(int prec) const { return ring_factored_for(cfg, (int)o, (int)v, prec); }

void Context::require_sizes() const { LRCC_REQUIRE(n > 0, LRCC_E_STATE, "lrcc_load_df has not been called"); }

void Context::reset_solutions() {
  have_t = have_lam = have_alpha = false;
  primal64 = primal32 = 0;
  ring64 = ring32 = 0;
  gradL_ready = 0;
  omegas.clear();
  alpha.clear();
}

static void copy_in(void* dst, const void* src, size_t bytes, int where, hipStream_t st) {
  LRCC_REQUIRE(where == LRCC_HOST || where == LRCC_DEVICE, LRCC_E_INVALID, "where must be LRCC_HOST or LRCC_DEVICE");
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, where == LRCC_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
  HIP_CHECK(hipStreamSynchronize(st));
}

void Context::load_df(int nocc, int nvir, int na, const void* Bp, int where) {
  LRCC_REQUIRE(Bp != nullptr, LRCC_E_INVALID, "B is null");
  LRCC_REQUIRE(nocc >= 2 && nvir >= 2 && na >= 1, LRCC_E_INVALID, "need nocc >= 2, nvir >= 2, naux >= 1");
  x64.reset();
  x32.reset();
  o = nocc, v = nvir, naux = na, nmo = o + v;
  n1 = o * v;
  dims = Dims{o, v, o * (o - 1) / 2, v * (v - 1) / 2};
  n2 = dims.O * dims.V;
  n = n1 + n2;
  if (B.bytes > 2 * (size_t)(naux * nmo * nmo * 16)) B.release();  // e.g. after a truncation
  B.ensure(naux * nmo * nmo * 16);
  copy_in(B.p, Bp, naux * nmo * nmo * 16, where, st);
  {  // the method (and the ladder's use of W = W^H) needs B^Q Hermitian for every Q
    constexpr int kParts = 1024;
    DevBuf part;
    part.ensure(2 * kParts * 8);
    launch_herm_defect(naux, nmo, B.p, part.p, kParts, st);
    std::vector<double> h(2 * kParts);
    HIP_CHECK(hipMemcpyAsync(h.data(), part.p, h.size() * 8, hipMemcpyDeviceToHost, st));
    sync();
    double dmax = 0, amax = 0;
    for (int b = 0; b < kParts; ++b) dmax = std::max(dmax, h[2 * b]), amax = std::max(amax, h[2 * b + 1]);
    if (!(dmax <= 1e-10 * std::max(amax, 1e-300))) {
      o = v = naux = nmo = n1 = n2 = n = 0;  // nothing loaded
      have_fock = false;
      ncomp = 0;
      reset_solutions();
      throw Error(LRCC_E_INVALID, "density-fitting factors are not Hermitian (B[Q][p][r] != conj B[Q][r][p])");
    }
  }
  const bool mixed = cfg.precision == LRCC_MIXED;
  mode32 = cfg.ladder_mode;
  mode64 = (mixed && cfg.ladder_mode_fp64 >= 0) ? cfg.ladder_mode_fp64 : cfg.ladder_mode;
  lean = lean_layout(cfg, (int)o, (int)v, (int)naux);
  x64.reset(new Executor<double>(P.m, dims, st));
  x64->ladder_const = P.m.find("W");
  x64->set_timing(timing);
  x64->set_graphs(cfg.graphs != 0);
  L64.release();
  L32.release();
  Tri64.release();
  Tri32.release();
  ints_built = goovv_built = false;  // the blocks are formed on first need (ensure_integrals)
  have_fock = false;
  ncomp = 0;
  reset_solutions();
}

// The integral blocks are formed when something first needs them, not by
// load_df: a system loaded only to be truncated (FNS / FNS++) needs <oo||vv>
// alone, while all blocks of its full virtual space may not fit the device.
void Context::ensure_integrals() {
  if (ints_built) return;
  require_sizes();
  if (mode64 != LRCC_LADDER_FULL || (cfg.precision == LRCC_MIXED && mode32 != LRCC_LADDER_FULL)) {
    // the virtual-virtual block of B builds W's rows
    L64.ensure((size_t)naux * v * v * 16);
    launch_gather_block(naux, nmo, o, v, o, v, B.p, L64.p, st);
  }
  if (mode64 == LRCC_LADDER_DIRECT) x64->set_direct_ladder(L64.p, naux, v);
  build_integrals();
  ints_built = true;
}

void Context::ensure_goovv() {
  if (ints_built || goovv_built) return;
  require_sizes();
  build_block(B.p, naux, o, v, "oovv", x64->ptr(P.m.find("goovv")), st);
  goovv_built = true;
}

// <oo||vv> built alone for a truncation is freed once the MP2 doubles and
// Hbar diagonals are formed (the full set is built again on first need).
void Context::release_goovv_if_alone() {
  if (ints_built || !goovv_built) return;
  x64->release(P.m.find("goovv"));
  goovv_built = false;
}

void Context::build_integrals() {
  for (auto& b : kBlocks)
    if (!(lean && lean_block(b[0])) && !(goovv_built && !std::strcmp(b[0], "goovv")))
      build_block(B.p, naux, o, v, b[1], x64->ptr(P.m.find(b[0])), st);
  if (mode64 == LRCC_LADDER_FULL) build_packed_vvvv(B.p, naux, o, v, x64->ptr(P.m.find("W")), st);
  if (mode64 == LRCC_LADDER_TRIANGLE || (cfg.precision == LRCC_MIXED && mode32 == LRCC_LADDER_TRIANGLE)) {
    // row blocks of about equal size (rows grow as b^2): b_j = 1 + (v - 1) sqrt(j / nb)
    const int nb = (int)std::min<int64_t>(8, v - 1);
    tri_bnd.assign(1, 1);
    for (int j = 1; j <= nb; ++j) {
      int64_t b = j == nb ? v : (int64_t)std::llround(1.0 + (double)(v - 1) * std::sqrt((double)j / nb));
      b = std::min<int64_t>(v - (nb - j), std::max<int64_t>(b, tri_bnd.back() + 1));
      tri_bnd.push_back(b);
    }
    const int64_t V = dims.V;
    tri_offs.assign(1, 0);
    for (size_t j = 0; j + 1 < tri_bnd.size(); ++j) {
      const int64_t r0 = tri_bnd[j] * (tri_bnd[j] - 1) / 2, r1 = tri_bnd[j + 1] * (tri_bnd[j + 1] - 1) / 2;
      tri_offs.push_back(tri_offs.back() + (r1 - r0) * (V - r0));
    }
  }
  if (mode64 == LRCC_LADDER_TRIANGLE) {
    Tri64.ensure((size_t)tri_offs.back() * 16);
    build_vvvv_triangle<double>(L64.p, naux, v, tri_bnd, tri_offs, Tri64.p, st);
    x64->set_triangle_ladder(tri_blocks<double>(Tri64.p));
  }
  if (lean) {
    build_block(B.p, naux, o, v, "ovvv", x64->ptr(P.m.find("govvp")), st, true);
    set_virtuals(*x64, P.m);
  } else {
    pack_last_pair(x64->ptr(P.m.find("govvv")), o, v, v, x64->ptr(P.m.find("govvp")), st);
  }
  const double one[2] = {1.0, 0.0};
  HIP_CHECK(hipMemcpyAsync(x64->ptr(P.one), one, 16, hipMemcpyHostToDevice, st));
  sync();
}

template <typename T>
std::vector<typename Executor<T>::TriBlock> Context::tri_blocks(const void* base) const {
  std::vector<typename Executor<T>::TriBlock> out;
  for (size_t j = 0; j + 1 < tri_bnd.size(); ++j)
    out.push_back({tri_bnd[j] * (tri_bnd[j] - 1) / 2, tri_bnd[j + 1] * (tri_bnd[j + 1] - 1) / 2,
                   (const char*)base + tri_offs[j] * 2 * sizeof(T)});
  return out;
}

static void ensure_x32(Context& c) {
  if (c.x32) return;
  c.ensure_integrals();
  const int W = c.P.m.find("W");
  auto stored = [&](int id) {  // constants the FP32 executor holds a copy of (W apart)
    const Role r = c.P.m[id].role;
    if (id == W || (c.lean && lean_block(c.P.m[id].name.c_str()))) return false;
    return r == Role::Const || r == Role::Scalar1 || r == Role::Fock;
  };
  {  // the FP32 copies of the constants; make room from FP64 batch storage if needed
    int64_t need = 0;
    for (size_t id = 0; id < c.P.m.tensors.size(); ++id)
      if (stored((int)id)) need += c.x64->elems((int)id, 1) * 8;
    if (c.mode32 == LRCC_LADDER_FULL) need += c.x64->elems(W, 1) * 8;
    if ((double)dev_available() < 1.1 * (double)need + (1 << 30)) c.x64->release_batched();
  }
  c.x32.reset(new Executor<float>(c.P.m, c.dims, c.st));
  c.x32->ladder_const = W;
  c.x32->set_timing(c.timing);
  c.x32->set_graphs(c.cfg.graphs != 0);
  for (size_t id = 0; id < c.P.m.tensors.size(); ++id) {
    if (!stored((int)id) || (c.P.m[(int)id].role == Role::Fock && !c.have_fock)) continue;
    launch_d2s(c.x64->elems((int)id, 1), c.x64->ptr((int)id), c.x32->ptr((int)id), c.st);
  }
  if (c.mode32 == LRCC_LADDER_FULL) {
    if (c.mode64 == LRCC_LADDER_FULL)
      launch_d2s(c.x64->elems(W, 1), c.x64->ptr(W), c.x32->ptr(W), c.st);
    else  // rows of W formed in FP64 from the factors, rounded once
      build_vvvv_triangle<float>(c.L64.p, c.naux, c.v, {1, c.v}, {0}, c.x32->ptr(W), c.st);
  }
  if (c.mode32 == LRCC_LADDER_DIRECT) {
    c.L32.ensure((size_t)c.naux * c.v * c.v * 8);
    launch_d2s(c.naux * c.v * c.v, c.L64.p, c.L32.p, c.st);
    c.x32->set_direct_ladder(c.L32.p, c.naux, c.v);
  }
  if (c.mode32 == LRCC_LADDER_TRIANGLE) {
    c.Tri32.ensure((size_t)c.tri_offs.back() * 8);
    if (c.mode64 == LRCC_LADDER_TRIANGLE)
      launch_d2s(c.tri_offs.back(), c.Tri64.p, c.Tri32.p, c.st);
    else
      build_vvvv_triangle<float>(c.L64.p, c.naux, c.v, c.tri_bnd, c.tri_offs, c.Tri32.p, c.st);
    c.x32->set_triangle_ladder(c.tri_blocks<float>(c.Tri32.p));
  }
  if (c.lean) set_virtuals(*c.x32, c.P.m);
  if (c.have_fock) {
    launch_zero_diag<float>(c.x32->ptr(c.P.foo), c.o, c.st);
    launch_zero_diag<float>(c.x32->ptr(c.P.fvv), c.v, c.st);
  }
  c.sync();
}

void Context::upload_fock_blocks() {
  const int ids[4] = {P.foo, P.fov, P.fvo, P.fvv};
  const int64_t p0[4] = {0, 0, o, o}, np[4] = {o, o, v, v}, r0[4] = {0, o, 0, o}, nr[4] = {o, v, o, v};
  for (int k = 0; k < 4; ++k) {
    launch_gather_block(1, nmo, p0[k], np[k], r0[k], nr[k], fock.p, x64->ptr(ids[k]), st);
    if (x32) launch_d2s(np[k] * nr[k], x64->ptr(ids[k]), x32->ptr(ids[k]), st);
  }
  if (x32) {  // the FP32 program carries only the off-diagonal part of f
    launch_zero_diag<float>(x32->ptr(P.foo), o, st);
    launch_zero_diag<float>(x32->ptr(P.fvv), v, st);
  }
}

void Context::load_fock(const void* F, int where) {
  require_sizes();
  LRCC_REQUIRE(F != nullptr, LRCC_E_INVALID, "F is null");
  fock.ensure(nmo * nmo * 16);
  copy_in(fock.p, F, nmo * nmo * 16, where, st);
  std::vector<cplx> h(nmo * nmo);
  d2h(h.data(), fock.p, nmo * nmo * 16);
  double herm = 0, scale = 0;
  for (int64_t p = 0; p < nmo; ++p)
    for (int64_t q = 0; q < nmo; ++q) {
      herm = std::max(herm, std::abs(h[p * nmo + q] - std::conj(h[q * nmo + p])));
      scale = std::max(scale, std::abs(h[p * nmo + q]));
    }
  LRCC_REQUIRE(herm <= 1e-10 * std::max(1.0, scale), LRCC_E_INVALID, "Fock matrix is not Hermitian");
  eps.resize(nmo);
  for (int64_t p = 0; p < nmo; ++p) eps[p] = h[p * nmo + p].real();
  double emax_o = *std::max_element(eps.begin(), eps.begin() + o);
  double emin_v = *std::min_element(eps.begin() + o, eps.end());
  LRCC_REQUIRE(emin_v - emax_o > 1e-8, LRCC_E_SINGULAR, "no gap between occupied and virtual Fock diagonals");
  DevBuf e;
  e.ensure(nmo * 8);
  h2d(e.p, eps.data(), nmo * 8);
  D.ensure(n * 8);
  launch_denominators(o, v, e.as<double>(), D.as<double>(), st);
  upload_fock_blocks();
  sync();
  have_fock = true;
  reset_solutions();
}

void Context::load_dipoles(int nc, const void* m, int where) {
  require_sizes();
  LRCC_REQUIRE(m != nullptr && nc >= 1 && nc <= 3, LRCC_E_INVALID, "need 1..3 dipole matrices");
  mu.ensure(nc * nmo * nmo * 16);
  copy_in(mu.p, m, nc * nmo * nmo * 16, where, st);
  std::vector<cplx> h(nc * nmo * nmo);
  d2h(h.data(), mu.p, h.size() * 16);
  for (int c = 0; c < nc; ++c)
    for (int64_t p = 0; p < nmo; ++p)
      for (int64_t q = 0; q <= p; ++q) {
        cplx a = h[(c * nmo + p) * nmo + q], b = h[(c * nmo + q) * nmo + p];
        LRCC_REQUIRE(std::abs(a - std::conj(b)) <= 1e-10 * (1.0 + std::abs(a)), LRCC_E_INVALID,
                     "dipole matrix is not Hermitian");
      }
  ncomp = nc;
  have_alpha = false;
}

// ---------------------------------------------------------------- Jacobian products

// Before a run of `ops` at batch nb on executor `run`: when the device has
// less free memory than the run's transients still need, the other
// executor's batch storage (its pool and scratch, formed again on its next
// run) is released.  The FP32 and FP64 products of a mixed solve alternate,
// so they need not hold their transients at the same time.
template <typename A, typename B>
static void make_room(A* run, const OpList& ops, int nb, const std::vector<int>& keep, B* other,
                      double extra_bytes = 0.0) {
  if (!other || other->batched_bytes() == 0) return;
  const double need = (double)run->transient_bytes(ops, nb, keep) - (double)run->batched_bytes() + extra_bytes;
  if (need > 0.9 * (double)dev_available()) other->release_batched();
}

// Bytes of the tensors the ring setup writes and keeps (Z1, Z2), for make_room.
template <typename X>
static double ring_bytes(X& x, double elem) {
  double b = 0;
  for (const char* nm : {"Z1", "Z2"}) b += elem * (double)x.elems(x.module().find(nm), 1);
  return b;
}

void Context::residual64(const void* tvec, void* R, cplx* E) {
  ensure_integrals();
  make_room(x64.get(), P.residual, 1, {}, x32.get());
  x64->bind(P.t1, const_cast<void*>(tvec));
  x64->bind(P.t2p, (char*)const_cast<void*>(tvec) + n1 * 16);
  x64->bind(P.O1, R);
  x64->bind(P.O2p, (char*)R + n1 * 16);
  x64->run(P.residual, 1);
  x64->unbind(P.O1);
  x64->unbind(P.O2p);
  primal64 = (tvec == t.p) ? 1 : 0;
  ring64 = 0;
  gradL_ready = 0;
  if (E) {
    double e[2];
    HIP_CHECK(hipMemcpyAsync(e, x64->ptr(P.E), 16, hipMemcpyDeviceToHost, st));
    sync();
    *E = cplx(e[0], e[1]);
  }
}

void Context::ensure_primal(int prec) {
  LRCC_REQUIRE(have_t, LRCC_E_STATE, "no ground-state amplitudes (call lrcc_solve_ground first)");
  if (prec == 64) {
    if (!primal64) {
      work.ensure(n * 16);
      residual64(t.p, work.p, nullptr);
    }
    if (factored(64) && !ring64) {
      make_room(x64.get(), P.ring_setup, 1, {}, x32.get(), ring_bytes(*x64, 16.0));
      x64->run(P.ring_setup, 1);
      ring64 = 1;
    }
    return;
  }
  ensure_x32(*this);
  if (!primal32) {
    t32.ensure(n * 8);
    launch_d2s(n, t.p, t32.p, st);
    x32->bind(P.t1, t32.p);
    x32->bind(P.t2p, (char*)t32.p + n1 * 8);
    x32->run(P.residual, 1);
    primal32 = 1;
    ring32 = 0;
    gradL32_ready = 0;
  }
  if (factored(32) && !ring32) {
    make_room(x32.get(), P.ring_setup, 1, {}, x64.get(), ring_bytes(*x32, 8.0));
    x32->run(P.ring_setup, 1);
    ring32 = 1;
  }
}

void Context::sigma64(Side side, int nb, const void* in, void* out) {
  ensure_primal(64);
  x64->set_max_batch(nb);
  const bool r = side == Side::Right;
  make_room(x64.get(), r ? right_prog(64) : left_prog(64), nb, r ? std::vector<int>{P.r_dO1, P.r_dO2p} :
            std::vector<int>{P.l_gt1, P.l_gt2p}, x32.get());
  int a1 = r ? P.r_dt1 : P.l_gO1, a2 = r ? P.r_dt2p : P.l_gO2p;
  int o1 = r ? P.r_dO1 : P.l_gt1, o2 = r ? P.r_dO2p : P.l_gt2p;
  launch_copy_rows<double, double>(nb, n1, in, n, x64->ptr(a1), n1, st);
  launch_copy_rows<double, double>(nb, n2, (const char*)in + n1 * 16, n, x64->ptr(a2), n2, st);
  x64->run(r ? right_prog(64) : left_prog(64), nb, {o1, o2});
  launch_copy_rows<double, double>(nb, n1, x64->ptr(o1), n1, out, n, st);
  launch_copy_rows<double, double>(nb, n2, x64->ptr(o2), n2, (char*)out + n1 * 16, n, st);
  sigma_count += nb;
}

void Context::sigma32(Side side, int nb, const void* in64, void* out32) {
  ensure_primal(32);
  x32->set_max_batch(nb);
  const bool r = side == Side::Right;
  make_room(x32.get(), r ? right_prog(32) : left_prog(32), nb, r ? std::vector<int>{P.r_dO1, P.r_dO2p} :
            std::vector<int>{P.l_gt1, P.l_gt2p}, x64.get());
  int a1 = r ? P.r_dt1 : P.l_gO1, a2 = r ? P.r_dt2p : P.l_gO2p;
  int o1 = r ? P.r_dO1 : P.l_gt1, o2 = r ? P.r_dO2p : P.l_gt2p;
  launch_copy_rows<double, float>(nb, n1, in64, n, x32->ptr(a1), n1, st);
  launch_copy_rows<double, float>(nb, n2, (const char*)in64 + n1 * 16, n, x32->ptr(a2), n2, st);
  x32->run(r ? right_prog(32) : left_prog(32), nb, {o1, o2});
  launch_copy_rows<float, float>(nb, n1, x32->ptr(o1), n1, out32, n, st);
  launch_copy_rows<float, float>(nb, n2, x32->ptr(o2), n2, (char*)out32 + n1 * 8, n, st);
  sigma_count += nb;
}

static void gather_mu_blocks(Context& c, int nb, const int* comp, const int* dst_ids) {
  const int64_t p0[4] = {0, 0, c.o, c.o}, np[4] = {c.o, c.o, c.v, c.v}, r0[4] = {0, c.o, 0, c.o},
                nr[4] = {c.o, c.v, c.o, c.v};
  for (int k = 0; k < 4; ++k) {
    char* dst = (char*)c.x64->ptr(dst_ids[k]);
    for (int r = 0; r < nb; ++r)
      launch_gather_block(1, c.nmo, p0[k], np[k], r0[k], nr[k], (const char*)c.mu.p + comp[r] * c.nmo * c.nmo * 16,
                          dst + r * np[k] * nr[k] * 16, c.st);
  }
}

// One component at a time: these run once per response solve, and a batch
// of one keeps their transients at a single right-hand side's size.
void Context::xi_vectors(void* out) {
  ensure_primal(64);
  for (int c = 0; c < ncomp; ++c) {
    gather_mu_blocks(*this, 1, &c, P.x_df);
    x64->run(P.xi, 1, {P.x_dO1, P.x_dO2p});
    char* o = (char*)out + (size_t)c * n * 16;
    launch_copy_rows<double, double>(1, n1, x64->ptr(P.x_dO1), n1, o, n, st);
    launch_copy_rows<double, double>(1, n2, x64->ptr(P.x_dO2p), n2, o + n1 * 16, n, st);
  }
}

void Context::hvp(int nb, const int* comp, const void* Xdt, void* out) {
  ensure_primal(64);
  LRCC_REQUIRE(have_lam, LRCC_E_STATE, "no Lambda amplitudes (call lrcc_solve_lambda first)");
  if (!gradL_ready) {
    x64->bind(P.g_lam1, lam.p);
    x64->bind(P.g_lam2p, (char*)lam.p + n1 * 16);
    x64->run(P.gradL, 1);
    gradL_ready = 1;
  }
  x64->set_max_batch(nb);
  make_room(x64.get(), P.hvp, nb, {P.h_out1, P.h_out2p}, x32.get());
  if (Xdt) {
    launch_copy_rows<double, double>(nb, n1, Xdt, n, x64->ptr(P.h_dt1), n1, st);
    launch_copy_rows<double, double>(nb, n2, (const char*)Xdt + n1 * 16, n, x64->ptr(P.h_dt2p), n2, st);
  } else {
    launch_fill_zero<double>(x64->ptr(P.h_dt1), nb * n1, st);
    launch_fill_zero<double>(x64->ptr(P.h_dt2p), nb * n2, st);
  }
  gather_mu_blocks(*this, nb, comp, P.h_df);
  x64->run(P.hvp, nb, {P.h_out1, P.h_out2p});
  launch_copy_rows<double, double>(nb, n1, x64->ptr(P.h_out1), n1, out, n, st);
  launch_copy_rows<double, double>(nb, n2, x64->ptr(P.h_out2p), n2, (char*)out + n1 * 16, n, st);
}

static void vec_norms(Context& c, int nb, const void* v, std::vector<double>& out) {
  DevBuf d, w;
  d.ensure(nb * 16);
  w.ensure((size_t)nb * 1024 * 16);
  launch_batched_dot<double>(nb, c.n, v, c.n, v, c.n, true, d.p, w.p, c.st);
  std::vector<cplx> h(nb);
  HIP_CHECK(hipMemcpyAsync(h.data(), d.p, nb * 16, hipMemcpyDeviceToHost, c.st));
  c.sync();
  out.resize(nb);
  for (int r = 0; r < nb; ++r) out[r] = std::sqrt(std::max(0.0, h[r].real()));
}

void Context::residual32(const void* tvec, void* R) {
  ensure_x32(*this);
  make_room(x32.get(), P.residual, 1, {}, x64.get());
  t32.ensure(n * 8);
  work.ensure(n * 16);
  launch_d2s(n, tvec, t32.p, st);
  x32->bind(P.t1, t32.p);
  x32->bind(P.t2p, (char*)t32.p + n1 * 8);
  x32->bind(P.O1, work.p);
  x32->bind(P.O2p, (char*)work.p + n1 * 8);
  x32->run(P.residual, 1);
  x32->unbind(P.O1);
  x32->unbind(P.O2p);
  primal32 = 0;
  ring32 = 0;
  gradL32_ready = 0;
  launch_residual<float>(1, n, work.p, nullptr, tvec, nullptr, 0, R, st, D.as<double>());
}

void Context::fx32(int nb, const void* X64, void* out32) {
  ensure_primal(32);
  LRCC_REQUIRE(have_lam, LRCC_E_STATE, "no Lambda amplitudes (call lrcc_solve_lambda first)");
  if (!gradL32_ready) {
    lam32.ensure(n * 8);
    launch_d2s(n, lam.p, lam32.p, st);
    x32->bind(P.g_lam1, lam32.p);
    x32->bind(P.g_lam2p, (char*)lam32.p + n1 * 8);
    x32->run(P.gradL, 1);
    gradL32_ready = 1;
  }
  x32->set_max_batch(nb);
  make_room(x32.get(), P.hvpt, nb, {P.f_out1, P.f_out2p}, x64.get());
  launch_copy_rows<double, float>(nb, n1, X64, n, x32->ptr(P.f_dt1), n1, st);
  launch_copy_rows<double, float>(nb, n2, (const char*)X64 + n1 * 16, n, x32->ptr(P.f_dt2p), n2, st);
  x32->run(P.hvpt, nb, {P.f_out1, P.f_out2p});
  launch_copy_rows<float, float>(nb, n1, x32->ptr(P.f_out1), n1, out32, n, st);
  launch_copy_rows<float, float>(nb, n2, x32->ptr(P.f_out2p), n2, (char*)out32 + n1 * 8, n, st);
}

// ---------------------------------------------------------------- DIIS

// Batched DIIS-accelerated Jacobi solver over `nb` slots, resident on the
// device.  One iteration is: the residual resid(na, shift, X, B, R) of the
// active slots (a Jacobian product and the residual kernel), the residual
// norms, the convergence test (launch_diis_check), the Jacobi step written
// into each slot's history ring, the new Gram row, the DIIS coefficients
// (launch_diis_coef: the small linear solve per slot) and the extrapolation
// -- every step a kernel on the context's stream.  The host reads the slots'
// state back once per iteration (one synchronization) to retire converged
// slots: a retired slot's iterate is copied out and the last active slot
// moves into its place, so uneven convergence costs no wasted products.
// With graphs on (and no kernel timing), the whole iteration at a given
// batch is captured into one HIP graph on its second occurrence and
// replayed from the third.  b (slot order, may be null) sets the reference
// norms; without it the first residual norm is the reference (or `ref`).
using ResidFn = std::function<void(int, const double*, const void*, const void*, void*)>;

namespace {

// Whole-iteration graphs of one diis_solve call, keyed by the batch.
struct IterGraphs {
  struct Entry {
    int seen = 0;
    hipGraphExec_t exec = nullptr;
    int64_t e64 = -1, e32 = -1;
  };
  std::map<int, Entry> by_na;
  bool broken = false;  // a capture failed: eager from here on
  ~IterGraphs() {
    for (auto& kv : by_na)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  }
};

}  // namespace

static void diis_solve(Context& c, int nb, const double* shifts_host, const void* b, void* x, double tol, int maxit,
                       const ResidFn& resid, std::vector<SolveStats>& stats, int sig_per_eval,
                       int stall = 0, double ref = -1.0) {
  const int64_t n = c.n;
  const int m = std::max(0, c.cfg.diis_size);
  const size_t vb = n * 16;
  double t0 = now_s();
  DevBuf Xw, Bw, Rw, En, Hx, He, shift, coef, gram, dots, work, G, state, flags;
  Xw.ensure(nb * vb);
  Rw.ensure(nb * vb);
  if (m > 0) En.ensure(nb * vb);
  if (b) {
    Bw.ensure(nb * vb);
    HIP_CHECK(hipMemcpyAsync(Bw.p, b, nb * vb, hipMemcpyDeviceToDevice, c.st));
  }
  if (m > 0) {
    Hx.ensure((size_t)nb * m * vb);
    He.ensure((size_t)nb * m * vb);
    launch_fill_zero<double>(He.p, (int64_t)nb * m * n, c.st);
    launch_fill_zero<double>(Hx.p, (int64_t)nb * m * n, c.st);
    coef.ensure(nb * m * 16);
    gram.ensure(nb * m * 16);
    G.ensure((size_t)nb * m * m * 16);
    launch_fill_zero<double>(G.p, (int64_t)nb * m * m, c.st);
  }
  shift.ensure(nb * 8);
  dots.ensure(nb * 16);
  work.ensure((size_t)nb * std::max(m, 1) * 1024 * 16);
  state.ensure(nb * sizeof(DiisSlot));
  flags.ensure(2 * nb * sizeof(int));  // active[nb], hrow[nb]
  int* active = flags.as<int>();
  int* hrow = active + nb;
  HIP_CHECK(hipMemcpyAsync(Xw.p, x, nb * vb, hipMemcpyDeviceToDevice, c.st));
  std::vector<double> sh(nb, 0.0);
  if (shifts_host) sh.assign(shifts_host, shifts_host + nb);
  std::vector<DiisSlot> q(nb);
  std::vector<int> rhs(nb), act(2 * nb, 1);
  {
    std::vector<cplx> hd(nb);
    if (b) {
      launch_batched_dot<double>(nb, n, Bw.p, n, Bw.p, n, true, dots.p, work.p, c.st);
      c.d2h(hd.data(), dots.p, nb * 16);
    }
    for (int s = 0; s < nb; ++s) {
      rhs[s] = s;
      q[s] = DiisSlot{0.0, b ? std::sqrt(std::max(0.0, hd[s].real())) : ref, 1e300, 0, 0, 0, 0, 0, 0, 0};
      if (b && q[s].bnorm == 0) q[s].bnorm = 1e-300;
      act[nb + s] = s * std::max(m, 1);
    }
  }
  stats.assign(nb, SolveStats());
  auto slot_ptr = [&](DevBuf& buf, int s) { return (char*)buf.p + (size_t)s * vb; };
  auto hist_ptr = [&](DevBuf& buf, int s, int k) { return (char*)buf.p + ((size_t)s * m + k) * vb; };
  auto finalize = [&](int s, bool at_limit) {
    const DiisSlot& t = q[s];
    HIP_CHECK(hipMemcpyAsync((char*)x + (size_t)rhs[s] * vb, slot_ptr(Xw, s), vb, hipMemcpyDeviceToDevice, c.st));
    SolveStats& so = stats[rhs[s]];
    so.iterations = t.iters - (at_limit ? 1 : 0);  // at the limit the last test was not followed by an update
    so.converged = at_limit ? 0 : t.conv;
    so.residual = t.bnorm > 0 ? t.rn / t.bnorm : t.rn;
    so.sigma_evals = (int64_t)t.itc * sig_per_eval;
    so.seconds = now_s() - t0;
  };
  auto move_slot = [&](int from, int to) {
    if (from == to) return;
    HIP_CHECK(hipMemcpyAsync(slot_ptr(Xw, to), slot_ptr(Xw, from), vb, hipMemcpyDeviceToDevice, c.st));
    if (b) HIP_CHECK(hipMemcpyAsync(slot_ptr(Bw, to), slot_ptr(Bw, from), vb, hipMemcpyDeviceToDevice, c.st));
    if (m > 0) {
      HIP_CHECK(hipMemcpyAsync(hist_ptr(Hx, to, 0), hist_ptr(Hx, from, 0), m * vb, hipMemcpyDeviceToDevice, c.st));
      HIP_CHECK(hipMemcpyAsync(hist_ptr(He, to, 0), hist_ptr(He, from, 0), m * vb, hipMemcpyDeviceToDevice, c.st));
      HIP_CHECK(hipMemcpyAsync((char*)G.p + (size_t)to * m * m * 16, (char*)G.p + (size_t)from * m * m * 16,
                               (size_t)m * m * 16, hipMemcpyDeviceToDevice, c.st));
    }
    q[to] = q[from];
    rhs[to] = rhs[from];
    sh[to] = sh[from];
  };
  auto upload = [&](int na) {  // slot state, flags and shifts of the active slots
    for (int s = 0; s < na; ++s) {
      act[s] = 1;
      act[nb + s] = s * std::max(m, 1) + (m > 0 ? q[s].next : 0);
    }
    HIP_CHECK(hipMemcpyAsync(state.p, q.data(), na * sizeof(DiisSlot), hipMemcpyHostToDevice, c.st));
    HIP_CHECK(hipMemcpyAsync(active, act.data(), na * sizeof(int), hipMemcpyHostToDevice, c.st));
    HIP_CHECK(hipMemcpyAsync(hrow, act.data() + nb, na * sizeof(int), hipMemcpyHostToDevice, c.st));
    HIP_CHECK(hipMemcpyAsync(shift.p, sh.data(), na * 8, hipMemcpyHostToDevice, c.st));
  };
  // one iteration on the device; `update` false: residual and test only
  auto body = [&](int na, bool update) {
    resid(na, shift.as<double>(), Xw.p, b ? Bw.p : nullptr, Rw.p);
    launch_batched_dot<double>(na, n, Rw.p, n, Rw.p, n, true, dots.p, work.p, c.st);
    launch_diis_check(na, dots.p, tol, stall, m, (DiisSlot*)state.p, active, hrow, c.st);
    if (!update) return;
    if (m == 0) {  // plain Jacobi, in place
      launch_jacobi(na, n, c.D.as<double>(), shift.as<double>(), Xw.p, Rw.p, Xw.p, nullptr, c.st, nullptr, nullptr,
                    active);
      return;
    }
    launch_jacobi(na, n, c.D.as<double>(), shift.as<double>(), Xw.p, Rw.p, Hx.p, He.p, c.st, hrow, En.p, active);
    launch_gram(na, m, n, He.p, m, En.p, gram.p, work.p, c.st);
    launch_diis_coef(na, m, gram.p, (DiisSlot*)state.p, active, G.p, coef.p, c.st);
    launch_combine(na, m, n, coef.p, Hx.p, m, Xw.p, c.st, active);
  };
  IterGraphs graphs;
  const bool use_graphs = c.cfg.graphs != 0 && !c.timing;
  auto epoch = [&](bool is64) -> int64_t {
    if (is64) return c.x64 ? c.x64->epoch() : -1;
    return c.x32 ? c.x32->epoch() : -1;
  };
  // one iteration through a whole-iteration graph: eager the first time at
  // this batch, captured the second time, replayed afterwards
  auto run_iteration = [&](int na) {
    if (!use_graphs || graphs.broken) return body(na, true);
    IterGraphs::Entry& e = graphs.by_na[na];
    if (e.exec && (e.e64 != epoch(true) || e.e32 != epoch(false))) {  // buffers moved: capture again
      (void)hipGraphExecDestroy(e.exec);
      e.exec = nullptr;
      e.seen = 1;
    }
    if (e.exec) {
      HIP_CHECK(hipGraphLaunch(e.exec, c.st));
      ++c.iter_replays;
      return;
    }
    if (e.seen++ == 0) return body(na, true);
    if (!c.cst) HIP_CHECK(hipStreamCreateWithFlags(&c.cst, hipStreamNonBlocking));
    // the capture stream starts after everything queued on the context's stream
    hipEvent_t ev;
    HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(ev, c.st));
    HIP_CHECK(hipStreamWaitEvent(c.cst, ev, 0));
    (void)hipEventDestroy(ev);
    const hipStream_t home = c.st;
    hipGraph_t g = nullptr;
    bool ok = true;
    HIP_CHECK(hipStreamBeginCapture(c.cst, hipStreamCaptureModeThreadLocal));
    c.st = c.cst;
    if (c.x64) c.x64->begin_outer(c.cst);
    if (c.x32) c.x32->begin_outer(c.cst);
    try {
      body(na, true);
    } catch (const Error&) {
      ok = false;  // e.g. an allocation the capture cannot hold: this solve stays eager
    }
    if (c.x64) c.x64->end_outer();
    if (c.x32) c.x32->end_outer();
    c.st = home;
    const hipError_t ec = hipStreamEndCapture(c.cst, &g);
    hipGraphExec_t ex = nullptr;
    if (ok && ec == hipSuccess && g) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
    else ok = false;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
      if (ex) (void)hipGraphExecDestroy(ex);
      (void)hipGetLastError();
      graphs.broken = true;
      return body(na, true);
    }
    e.exec = ex;
    e.e64 = epoch(true);
    e.e32 = epoch(false);
    ++c.iter_captures;
    HIP_CHECK(hipGraphLaunch(ex, c.st));
  };
  int na = nb;
  upload(na);
  for (int it = 0;; ++it) {
    const bool last = it == maxit;
    if (last)
      body(na, false);
    else
      run_iteration(na);
    c.d2h(q.data(), state.p, na * sizeof(DiisSlot));
    c.d2h(act.data(), active, na * sizeof(int));
    for (int s = 0; s < na; ++s)
      LRCC_REQUIRE(!q[s].bad, LRCC_E_NOCONV, "residual is not finite");
    if (c.cfg.verbose >= 2) {
      fprintf(stderr, "[lrcc] it %d active %d", it, na);
      for (int s = 0; s < std::min(na, 4); ++s) fprintf(stderr, " %.3e", q[s].rn / q[s].bnorm);
      fprintf(stderr, "\n");
    }
    const int na0 = na;
    for (int s = 0; s < na;) {
      if (!act[s]) {
        finalize(s, false);
        move_slot(na - 1, s);
        act[s] = act[na - 1];
        --na;
      } else {
        ++s;
      }
    }
    if (na == 0) break;
    if (last) {
      for (int s = 0; s < na; ++s) finalize(s, true);
      break;
    }
    if (na != na0) upload(na);
  }
  c.sync();
}

// ---------------------------------------------------------------- solves

void Context::solve_ground(double ecorr_out[2], SolveStats& so) {
  require_sizes();
  LRCC_REQUIRE(have_fock, LRCC_E_STATE, "lrcc_load_fock has not been called");
  t.ensure(n * 16);
  launch_fill_zero<double>(t.p, n, st);
  have_t = have_lam = have_alpha = false;
  primal64 = primal32 = gradL_ready = 0;
  ring64 = ring32 = 0;
  std::vector<SolveStats> ss;
  if (cfg.precision == LRCC_MIXED) {
    // FP32 coupling terms with the FP64 diagonal until the iteration stalls
    // or converges, then FP64 residuals finish (and certify) the solve.  The
    // reference norm is that of the driving terms, ||Omega(0)||.
    std::vector<double> r0;
    work.ensure(n * 16);
    DevBuf R0;
    R0.ensure(n * 16);
    residual64(t.p, R0.p, nullptr);
    vec_norms(*this, 1, R0.p, r0);
    double ref = std::max(r0[0], 1e-300);
    std::vector<SolveStats> s32;
    diis_solve(*this, 1, nullptr, nullptr, t.p, cfg.tol_residual, cfg.maxit,
               [&](int, const double*, const void* X, const void*, void* R) { residual32(X, R); }, s32, 0, 4, ref);
    diis_solve(*this, 1, nullptr, nullptr, t.p, cfg.tol_residual, cfg.maxit,
               [&](int, const double*, const void* X, const void*, void* R) { residual64(X, R, nullptr); }, ss, 0,
               0, ref);
    ss[0].iterations += s32[0].iterations;
  } else {
    diis_solve(*this, 1, nullptr, nullptr, t.p, cfg.tol_residual, cfg.maxit,
               [&](int, const double*, const void* X, const void*, void* R) { residual64(X, R, nullptr); }, ss, 0);
  }
  so = ss[0];
  primal32 = 0;
  ring32 = 0;
  gradL32_ready = 0;
  // evaluate once more at the solution: every stored intermediate then belongs to it
  have_t = true;
  work.ensure(n * 16);
  cplx E;
  residual64(t.p, work.p, &E);
  ecorr = E;
  if (ecorr_out) {
    ecorr_out[0] = E.real();
    ecorr_out[1] = E.imag();
  }
  LRCC_REQUIRE(so.converged, LRCC_E_NOCONV, "ground-state amplitudes did not converge");
}

// Batched linear solve (op + s_r) x_r = -b_r (op = A for Right, A^T for Left).
// x holds the initial guesses on entry.  prec 64: FP64 products; prec 32:
// iterative refinement with FP64 outer residuals and FP32 inner products.
void Context::solve_linear(Side side, int nb, const double* shifts, const void* b, void* x, int prec, double tol,
                           std::vector<SolveStats>& out) {
  const size_t vb = n * 16;
  DevBuf sig;
  if (prec == 64) {
    sig.ensure(nb * vb);
    diis_solve(*this, nb, shifts, b, x, tol, cfg.maxit,
               [&](int na, const double* sh, const void* X, const void* Bw, void* R) {
                 sigma64(side, na, X, sig.p);
                 launch_residual<double>(na, n, sig.p, sh, X, Bw, n, R, st);
               },
               out, 1);
    return;
  }
  // Mixed precision.  The FP32 program carries f without its diagonal, so
  // it computes the coupling part (A - D) X; the residual kernel adds
  // (D + s) X and b in FP64.  FP32 rounding therefore perturbs only the small
  // coupling term and the FP32 iteration converges well below the FP32
  // epsilon.  An FP64 product then certifies every right-hand side (defect
  // correction); any that fall short continue with FP64 products.
  sig.ensure(nb * n * 8);
  std::vector<SolveStats> s32;
  diis_solve(*this, nb, shifts, b, x, tol, cfg.maxit,
             [&](int na, const double* sh, const void* X, const void* Bw, void* R) {
               sigma32(side, na, X, sig.p);
               launch_residual<float>(na, n, sig.p, sh, X, Bw, n, R, st, D.as<double>());
             },
             s32, 1, 4);
  out = s32;
  DevBuf s64, R64, shd;
  s64.ensure(nb * vb);
  R64.ensure(nb * vb);
  shd.ensure(nb * 8);
  std::vector<double> sh(nb, 0.0);
  if (shifts) sh.assign(shifts, shifts + nb);
  HIP_CHECK(hipMemcpyAsync(shd.p, sh.data(), nb * 8, hipMemcpyHostToDevice, st));
  sigma64(side, nb, x, s64.p);
  launch_residual<double>(nb, n, s64.p, shd.as<double>(), x, b, n, R64.p, st);
  std::vector<double> rn, bn;
  vec_norms(*this, nb, R64.p, rn);
  vec_norms(*this, nb, b, bn);
  std::vector<int> redo;
  for (int r = 0; r < nb; ++r) {
    out[r].sigma_evals += 1;
    out[r].residual = rn[r] / std::max(bn[r], 1e-300);
    out[r].converged = out[r].residual <= tol ? 1 : 0;
    if (!out[r].converged) redo.push_back(r);
  }
  if (redo.empty()) return;
  // finish the remaining right-hand sides with FP64 products
  const int nr = (int)redo.size();
  DevBuf Xr, Br;
  Xr.ensure(nr * vb);
  Br.ensure(nr * vb);
  std::vector<double> shr(nr);
  for (int q = 0; q < nr; ++q) {
    HIP_CHECK(hipMemcpyAsync((char*)Xr.p + q * vb, (char*)x + redo[q] * vb, vb, hipMemcpyDeviceToDevice, st));
    HIP_CHECK(hipMemcpyAsync((char*)Br.p + q * vb, (const char*)b + redo[q] * vb, vb, hipMemcpyDeviceToDevice, st));
    shr[q] = sh[redo[q]];
  }
  std::vector<SolveStats> s2;
  DevBuf sg;
  sg.ensure(nr * vb);
  diis_solve(*this, nr, shr.data(), Br.p, Xr.p, tol, cfg.maxit,
             [&](int na, const double* shv, const void* X, const void* Bw, void* R) {
               sigma64(side, na, X, sg.p);
               launch_residual<double>(na, n, sg.p, shv, X, Bw, n, R, st);
             },
             s2, 1);
  for (int q = 0; q < nr; ++q) {
    HIP_CHECK(hipMemcpyAsync((char*)x + redo[q] * vb, (char*)Xr.p + q * vb, vb, hipMemcpyDeviceToDevice, st));
    SolveStats& o = out[redo[q]];
    o.iterations += s2[q].iterations;
    o.sigma_evals += s2[q].sigma_evals;
    o.converged = s2[q].converged;
    o.residual = s2[q].residual;
    o.seconds += s2[q].seconds;
  }
  sync();
}

void Context::solve_lambda(SolveStats& so) {
  require_sizes();
  LRCC_REQUIRE(have_t, LRCC_E_STATE, "no ground-state amplitudes (call lrcc_solve_ground first)");
  ensure_primal(64);
  const size_t vb = n * 16;
  DevBuf e0;
  e0.ensure(vb);
  x64->run(P.eta0, 1);
  launch_copy_rows<double, double>(1, n1, x64->ptr(P.e_gt1), n1, e0.p, n, st);
  launch_copy_rows<double, double>(1, n2, x64->ptr(P.e_gt2p), n2, (char*)e0.p + n1 * 16, n, st);
  lam.ensure(vb);
  launch_jacobi(1, n, D.as<double>(), nullptr, nullptr, e0.p, lam.p, nullptr, st);
  std::vector<SolveStats> ss;
  solve_linear(Side::Left, 1, nullptr, e0.p, lam.p, cfg.precision == LRCC_MIXED ? 32 : 64, cfg.tol_residual, ss);
  so = ss[0];
  have_lam = true;
  gradL_ready = 0;
  gradL32_ready = 0;
  have_alpha = false;
  LRCC_REQUIRE(so.converged, LRCC_E_NOCONV, "Lambda amplitudes did not converge");
}

// Right-hand sides per batched solve: the configured chunk, or as many as
// fit in 70% of the free device memory (transient tensors of the Jacobian
// programs at the working precision(s) plus the DIIS history per RHS).
// Right-hand sides per batched product that fit the device.  `per` is the
// device bytes one right-hand side needs; the batch storage already held by
// the executors that will run (use64 / use32) counts as available.  If that
// is not enough for all right-hand sides, the batch storage of the executor
// that will not run is released first.
static int fit_chunk(int nrhs, int64_t per, Executor<double>* x64, Executor<float>* x32, bool use64, bool use32) {
  auto count = [&]() {
    double avail = (double)dev_available();  // free + cached device memory, or the workspace's free bytes
    if (use64 && x64) avail += (double)x64->batched_bytes();
    if (use32 && x32) avail += (double)x32->batched_bytes();
    return (int64_t)(0.85 * avail) / std::max<int64_t>(per, 1);
  };
  int64_t k = count();
  if (k < nrhs && (!use64 || !use32)) {
    if (!use64 && x64) x64->release_batched();
    if (!use32 && x32) x32->release_batched();
    k = count();
  }
  return (int)std::max<int64_t>(1, std::min<int64_t>(nrhs, k));
}

// Device bytes for the whole pipeline (load, T, Lambda, X/Y in batches of
// up to nrhs right-hand sides, alpha) at the configured precision: the sum
// of every buffer the context, its executors and the solves allocate, with
// the batched parts sized by the same liveness plans the executors use.
size_t workspace_estimate(const lrcc_config& cfg, int o, int v, int naux, int nrhs) {
  if (o < 2 || v < 2 || naux < 1 || nrhs < 1) return 0;
  static CcPrograms P = [] {
    CcPrograms p;
    build_programs(p);
    return p;
  }();
  const Module& m = P.m;
  const Dims d{o, v, (int64_t)o * (o - 1) / 2, (int64_t)v * (v - 1) / 2};
  const int64_t nmo = o + v, n = (int64_t)o * v + d.O * d.V;
  const bool mixed = cfg.precision == LRCC_MIXED;
  const int nb = nrhs;
  const int mode32 = cfg.ladder_mode;
  const int mode64 = (mixed && cfg.ladder_mode_fp64 >= 0) ? cfg.ladder_mode_fp64 : cfg.ladder_mode;
  const bool lean = lean_layout(cfg, o, v, naux);
  // context buffers: B, F, mu, D, t, lambda, work, xi, eta, X, Y (+ FP32 copies)
  double bytes = 16.0 * ((double)naux * nmo * nmo + 4.0 * nmo * nmo) + 8.0 * n + 16.0 * n * (3 + 6) +
                 2 * 16.0 * (double)nrhs * n + (mixed ? 8.0 * n * (2 + nb) : 0.0);
  if (mode64 != LRCC_LADDER_FULL || (mixed && mode32 != LRCC_LADDER_FULL))
    bytes += 16.0 * naux * (double)v * v;  // the virtual-virtual block of B
  // one executor: its unbatched tensors (constants, Fock blocks, primal
  // intermediates), the pool, the batched tensors outside the pool, scratch
  // returns the executor's fixed bytes; its batch storage goes to *batch
  // unbatched tensors the FP64 gradient of L writes: in mixed precision they
  // exist only while eta is formed (F X runs in FP32 afterwards)
  std::vector<char> grad_result(m.tensors.size(), 0);
  for (const Op& op : P.gradL) grad_result[op.out] = !m.tensors[op.out].batched;
  double grad64 = 0;
  auto executor = [&](double elem, int mode, const std::vector<std::pair<const OpList*, int>>& runs,
                      double* batch) {
    double b = 0;
    std::vector<char> in_pool(m.tensors.size(), 0), touched(m.tensors.size(), 0);
    for (auto& r : runs) {  // unbatched intermediates of a single run live in the pool
      for (auto& ts : plan_pool(m, d, *r.first, r.second, {}, nullptr).slot) in_pool[ts.first] = 1;
      for (const Op& op : *r.first)
        for (int u : {op.out, op.a, op.b})
          if (u >= 0) touched[u] = 1;
    }
    static const bool trace = std::getenv("LRCC_TRACE_ESTIMATE") != nullptr;
    for (size_t id = 0; id < m.tensors.size(); ++id) {
      if (m.tensors[id].batched || in_pool[id] || !touched[id]) continue;
      if ((int)id == m.find("W") && mode != LRCC_LADDER_FULL) continue;
      if (lean && lean_block(m.tensors[id].name.c_str())) continue;
      if (mixed && elem == 16.0 && grad_result[id]) {
        grad64 += elem * (double)tensor_elems(m, d, (int)id, 1);
        continue;
      }
      b += elem * (double)tensor_elems(m, d, (int)id, 1);
      if (trace && elem * (double)tensor_elems(m, d, (int)id, 1) > 1e8)
        fprintf(stderr, "[estimate] %s unbatched %s %.2f GB\n", elem == 16 ? "fp64" : "fp32",
                m.tensors[id].name.c_str(), elem * (double)tensor_elems(m, d, (int)id, 1) / 1e9);
    }
    if (mode == LRCC_LADDER_TRIANGLE)  // row blocks of the upper triangle: about (V^2 + V^2 / nb) / 2
      b += elem * 0.5625 * (double)d.V * (double)d.V;
    if (mode == LRCC_LADDER_DIRECT && elem == 8.0) b += 8.0 * naux * (double)v * v;  // its FP32 copy
    if (lean) b += 1.25 * (double)(size_t(1) << 30);  // chunks of the blocks formed on use
    std::vector<int64_t> pool;
    std::vector<char> pooled(m.tensors.size(), 0), used(m.tensors.size(), 0);
    int64_t big = 0;
    for (auto& r : runs) {
      PoolPlan pl = plan_pool(m, d, *r.first, r.second, {}, nullptr);
      if (trace) {
        double tot = 0;
        for (int64_t e : pl.slot_elems) tot += elem * (double)e;
        fprintf(stderr, "[estimate] %s run of %zu ops at batch %d: pool %zu slots %.2f GB\n",
                elem == 16 ? "fp64" : "fp32", r.first->size(), r.second, pl.slot_elems.size(), tot / 1e9);
      }
      if (pool.size() < pl.slot_elems.size()) pool.resize(pl.slot_elems.size(), 0);
      for (size_t k = 0; k < pl.slot_elems.size(); ++k) pool[k] = std::max(pool[k], pl.slot_elems[k]);
      for (auto& ts : pl.slot) pooled[ts.first] = 1;
      for (const Op& op : *r.first)
        for (int u : {op.out, op.a, op.b})
          if (u >= 0 && m.tensors[u].batched) {
            used[u] = 1;
            big = std::max(big, tensor_elems(m, d, u, r.second));
          }
    }
    double fixed = b;
    b = 0;
    for (int64_t e : pool) b += elem * (double)e;
    if (trace) {
      double pb = 0;
      for (int64_t e : pool) pb += elem * (double)e;
      fprintf(stderr, "[estimate] %s pool %zu slots %.2f GB, 4 x big %.2f GB\n", elem == 16 ? "fp64" : "fp32",
              pool.size(), pb / 1e9, elem * 4.0 * (double)big / 1e9);
    }
    for (size_t id = 0; id < m.tensors.size(); ++id)
      if (used[id] && !pooled[id]) {
        b += elem * (double)tensor_elems(m, d, (int)id, nb);
        if (trace)
          fprintf(stderr, "[estimate] %s batched kept %s %.2f GB\n", elem == 16 ? "fp64" : "fp32",
                  m.tensors[id].name.c_str(), elem * (double)tensor_elems(m, d, (int)id, nb) / 1e9);
      }
    b += elem * 4.0 * (double)big;  // three permutation slots and one tile-timing output
    *batch = b;
    if (mode == LRCC_LADDER_DIRECT) fixed += 2.0 * (double)Executor<double>::kDirectChunkBytes;
    return fixed + 320.0 * (1 << 20);  // split-K partials (at most 256 MB) and small buffers
  };
  // the two executors' batch storage is not held at once when memory is
  // short (the products alternate; see make_room)
  double batch64 = 0, batch32 = 0;
  const bool f64 = ring_factored_for(cfg, o, v, 64), f32 = ring_factored_for(cfg, o, v, 32);
  std::vector<std::pair<const OpList*, int>> runs64{{&P.residual, 1}, {f64 ? &P.right_f : &P.right, nb},
                                                    {f64 ? &P.left_f : &P.left, nb}, {&P.xi, 1}, {&P.eta0, 1},
                                                    {&P.gradL, 1}, {&P.hvp, nb}};
  if (f64) runs64.push_back({&P.ring_setup, 1});
  bytes += executor(16.0, mode64, runs64, &batch64);
  if (mixed) {
    std::vector<std::pair<const OpList*, int>> runs32{{&P.residual, 1}, {f32 ? &P.right_f : &P.right, nb},
                                                      {f32 ? &P.left_f : &P.left, nb}, {&P.gradL, 1}, {&P.hvpt, nb}};
    if (f32) runs32.push_back({&P.ring_setup, 1});
    bytes += executor(8.0, mode32, runs32, &batch32);
  }
  // solver buffers per right-hand side (iterates, residuals, driving terms,
  // DIIS history, products, certification)
  const double solver = (double)nb * (2.0 * std::max(cfg.diis_size, 0) + 12.0) * 16.0 * n;
  // phases: eta (the FP64 Hessian products with the FP64 gradient of L), then
  // the solves (the executors' transients alternate); the integral build
  // temporaries are freed before either
  const double build = 4.0 * 16.0 * naux * (double)v * v + (double)(size_t(1) << 30);
  bytes += std::max({batch64 + grad64, std::max(batch64, batch32) + solver, build});
  return (size_t)(1.1 * bytes) + (size_t(64) << 20);
}

int Context::rhs_chunk_for(int nrhs, int prec) {
  if (cfg.rhs_chunk > 0) return std::min(cfg.rhs_chunk, nrhs);
  if (prec == 32) ensure_x32(*this);
  int64_t per = 0;
  per += std::max(x64->transient_bytes(right_prog(64), 1, {P.r_dO1, P.r_dO2p}),
                  x64->transient_bytes(left_prog(64), 1, {P.l_gt1, P.l_gt2p}));
  per = std::max(per, x64->transient_bytes(P.hvp, 1, {P.h_out1, P.h_out2p}));
  if (prec == 32)
    per += std::max(x32->transient_bytes(right_prog(32), 1, {P.r_dO1, P.r_dO2p}),
                    x32->transient_bytes(left_prog(32), 1, {P.l_gt1, P.l_gt2p}));
  per += (int64_t)(2 * std::max(cfg.diis_size, 0) + 12) * n * 16;
  // both executors run within one solve: their batch storage all counts
  return fit_chunk(nrhs, per, x64.get(), x32.get(), true, prec == 32);
}

int Context::sigma_chunk(Side side, int nvec, int prec) {
  if (cfg.rhs_chunk > 0) return std::min(cfg.rhs_chunk, nvec);
  const bool r = side == Side::Right;
  const std::vector<int> keep = r ? std::vector<int>{P.r_dO1, P.r_dO2p} : std::vector<int>{P.l_gt1, P.l_gt2p};
  if (prec == 64) {
    int64_t per = x64->transient_bytes(r ? right_prog(64) : left_prog(64), 1, keep);
    return fit_chunk(nvec, per, x64.get(), x32.get(), true, false);
  }
  ensure_x32(*this);
  int64_t per = x32->transient_bytes(r ? right_prog(32) : left_prog(32), 1, keep) + n * 8;
  return fit_chunk(nvec, per, x64.get(), x32.get(), false, true);
}

// Eq. 35 route (quadratic = false): X(w) from (A - w) X = -xi, then Y(w)
// from Y (A + w) = -(eta + F X(w)); f_AB = Y^B.xi^A + eta^A.X^B.
// Eq. 36 route (quadratic = true): X(w) and X(-w), no left solves;
// f_AB(w) = eta^A.X^B(w) + eta^B.X^A(-w) + X^A(-w).F.X^B(w).  Both give
// alpha_AB = -1/2 [f_AB(w) + conj f_AB(-w)] (f_AB(-w) = f_BA(w) on the
// Eq. 35 route).  X(-w) is kept in the Y slot.
void Context::solve_response(int nw, const double* om, std::vector<SolveStats>& per, bool quadratic) {
  require_sizes();
  LRCC_REQUIRE(have_lam, LRCC_E_STATE, "no Lambda amplitudes (call lrcc_solve_lambda first)");
  LRCC_REQUIRE(ncomp > 0, LRCC_E_STATE, "lrcc_load_dipoles has not been called");
  LRCC_REQUIRE(nw >= 1 && om != nullptr, LRCC_E_INVALID, "need at least one frequency");
  // a frequency on a denominator makes (A -/+ w) singular in the Jacobi metric
  {
    std::vector<double> hD(n);
    d2h(hD.data(), D.p, n * 8);
    for (int k = 0; k < nw; ++k)
      for (int64_t i = 0; i < n; ++i)
        LRCC_REQUIRE(std::abs(hD[i] - std::abs(om[k])) >= 1e-8, LRCC_E_SINGULAR,
                     "frequency " + std::to_string(om[k]) + " lies on a denominator pole");
  }
  const int prec = cfg.precision == LRCC_MIXED ? 32 : 64;
  const size_t vb = n * 16;
  const int nrhs = nw * ncomp;
  omegas.assign(om, om + nw);
  xi.ensure(ncomp * vb);
  eta.ensure(ncomp * vb);
  xi_vectors(xi.p);
  for (int c = 0; c < ncomp; ++c) hvp(1, &c, nullptr, (char*)eta.p + (size_t)c * vb);
  if (prec == 32) {
    // F X runs with FP32 products from here on: the FP64 gradient of L that
    // only the FP64 Hessian products read is dropped (rebuilt on demand)
    x64->release_results(P.gradL);
    gradL_ready = 0;
  }
  have_alpha = false;
  response_route = quadratic ? 36 : 35;
  per.assign(2 * nrhs, SolveStats());
  const int chunk = rhs_chunk_for(nrhs, prec);
  // Frequency groups: all frequencies at once, or (lrcc_config.keep_response
  // = 0) as many as one batched product holds, each group's alpha formed
  // before the next group's amplitudes overwrite X and Y
  const int gw = cfg.keep_response ? nw : std::max(1, chunk / ncomp);
  const int gmax = std::min(gw, nw) * ncomp;
  X.ensure(gmax * vb);
  Y.ensure(gmax * vb);
  if (cfg.verbose >= 1)
    fprintf(stderr, "[lrcc] response: %d right-hand sides in chunks of %d, frequencies in groups of %d\n", nrhs, chunk,
            std::min(gw, nw));
  DevBuf bc, shd;
  shd.ensure(chunk * 8);
  alpha.assign(nw * ncomp * ncomp, 0.0);
  for (int k0 = 0; k0 < nw; k0 += gw) {
    const int k1 = std::min(nw, k0 + gw), ng = (k1 - k0) * ncomp, r0 = k0 * ncomp;
    bc.ensure(std::min(chunk, gmax) * vb);
    for (int side = 0; side < 2; ++side) {
      for (int c0 = 0; c0 < ng; c0 += chunk) {
        int nc = std::min(chunk, ng - c0);
        std::vector<double> sh(nc);
        std::vector<int> cp(nc);
        for (int q = 0; q < nc; ++q) {
          int r = r0 + c0 + q;
          cp[q] = r % ncomp;
          sh[q] = side == 0 ? -omegas[r / ncomp] : omegas[r / ncomp];
        }
        void* xc = (char*)(side == 0 ? X.p : Y.p) + c0 * vb;
        if (side == 0 || quadratic) {
          for (int q = 0; q < nc; ++q)
            HIP_CHECK(
                hipMemcpyAsync((char*)bc.p + q * vb, (char*)xi.p + cp[q] * vb, vb, hipMemcpyDeviceToDevice, st));
        } else {
          eta_plus_fx(nc, cp.data(), (char*)X.p + c0 * vb, bc.p, prec, eta.p);
        }
        HIP_CHECK(hipMemcpyAsync(shd.p, sh.data(), nc * 8, hipMemcpyHostToDevice, st));
        launch_jacobi(nc, n, D.as<double>(), shd.as<double>(), nullptr, bc.p, xc, nullptr, st);
        std::vector<SolveStats> ss;
        const Side sd = (side == 0 || quadratic) ? Side::Right : Side::Left;
        solve_linear(sd, nc, sh.data(), bc.p, xc, prec, cfg.tol_residual, ss);
        for (int q = 0; q < nc; ++q) per[side * nrhs + r0 + c0 + q] = ss[q];
        if (cfg.verbose >= 1) {
          int itmax = 0;
          for (auto& t : ss) itmax = std::max(itmax, t.iterations);
          fprintf(stderr, "[lrcc] %s right-hand sides %d..%d of %d: up to %d iterations\n", side == 0 ? "X" : "Y",
                  r0 + c0, r0 + c0 + nc - 1, nrhs, itmax);
        }
      }
    }
    std::vector<cplx> ag;
    if (quadratic) bc.release();  // room for the F X^B(w) of Eq. 36
    response_alpha(k1 - k0, chunk, quadratic, prec, ag);
    std::copy(ag.begin(), ag.end(), alpha.begin() + (size_t)k0 * ncomp * ncomp);
    resp_first = r0;
    resp_count = ng;
  }
  have_alpha = true;
  bool all = true;
  for (auto& s : per) all = all && s.converged;
  LRCC_REQUIRE(all, LRCC_E_NOCONV, "some response equations did not converge");
}

// eta^B + F X^B for nb right-hand sides with components comp.  On the mixed
// path F X takes FP32 products (F does not involve the Fock diagonal) and
// eta^B is added in FP64.
void Context::eta_plus_fx(int nb, const int* comp, const void* Xs, void* out, int prec, const void* etaB) {
  if (prec == 64) return hvp(nb, comp, Xs, out);
  const size_t vb = n * 16;
  DevBuf f32;
  f32.ensure(nb * n * 8);
  fx32(nb, Xs, f32.p);
  for (int q = 0; q < nb; ++q)
    launch_residual<float>(1, n, (char*)f32.p + (size_t)q * n * 8, nullptr, nullptr,
                           (const char*)etaB + comp[q] * vb, 0, (char*)out + q * vb, st);
}

// alpha on the Eq. 36 route from X(w) (Xp) and X(-w) (Xm), [nw][ncomp][n]
// each, and eta^B (etaB, [ncomp][n]).  With
// H^B = eta^B + F X^B(w) and the symmetry of F (a Hessian: u.F v = v.F u),
//   f_AB(w)  = eta^A.X^B(w) + eta^B.X^A(-w) + X^A(-w).F X^B(w)
//            = eta^A.X^B(w) + X^A(-w).H^B,
//   f_AB(-w) = eta^B.X^A(w) + X^B(-w).H^A.
// H is built in chunks of right-hand sides; the bilinear dots run on the
// device.
// alpha of the nw frequencies whose amplitudes X and Y hold (from their
// start): Eq. 35, alpha_AB(w) = -1/2 [f_AB + conj f_BA] with f_AB = Y^B . xi^A
// + eta^A . X^B, or Eq. 36 (quadratic: Y holds X(-w)).
void Context::response_alpha(int nw, int chunk, bool quadratic, int prec, std::vector<cplx>& out) {
  if (quadratic) {
    alpha_quadratic(nw, chunk, X.p, Y.p, eta.p, prec, out);
    return;
  }
  const size_t vb = n * 16;
  const int nrhs = nw * ncomp;
  DevBuf d1, d2, w;
  d1.ensure(nrhs * 16);
  d2.ensure(nrhs * 16);
  w.ensure((size_t)nrhs * 1024 * 16);
  std::vector<cplx> fy(nrhs * ncomp), fx(nrhs * ncomp);
  for (int a = 0; a < ncomp; ++a) {
    launch_batched_dot<double>(nrhs, n, Y.p, n, (char*)xi.p + a * vb, 0, false, d1.p, w.p, st);
    std::vector<cplx> h(nrhs);
    HIP_CHECK(hipMemcpyAsync(h.data(), d1.p, nrhs * 16, hipMemcpyDeviceToHost, st));
    sync();
    for (int r = 0; r < nrhs; ++r) fy[r * ncomp + a] = h[r];
    launch_batched_dot<double>(nrhs, n, X.p, n, (char*)eta.p + a * vb, 0, false, d2.p, w.p, st);
    HIP_CHECK(hipMemcpyAsync(h.data(), d2.p, nrhs * 16, hipMemcpyDeviceToHost, st));
    sync();
    for (int r = 0; r < nrhs; ++r) fx[r * ncomp + a] = h[r];
  }
  out.assign(nw * ncomp * ncomp, 0.0);
  for (int k = 0; k < nw; ++k) {
    std::vector<cplx> f(ncomp * ncomp);
    for (int a = 0; a < ncomp; ++a)
      for (int bb = 0; bb < ncomp; ++bb) {
        int r = k * ncomp + bb;
        f[a * ncomp + bb] = fy[r * ncomp + a] + fx[r * ncomp + a];
      }
    for (int a = 0; a < ncomp; ++a)
      for (int bb = 0; bb < ncomp; ++bb)
        out[(k * ncomp + a) * ncomp + bb] = -0.5 * (f[a * ncomp + bb] + std::conj(f[bb * ncomp + a]));
  }
}

void Context::alpha_quadratic(int nw, int chunk, const void* Xp, const void* Xm, const void* etaB, int prec,
                              std::vector<cplx>& out) {
  const size_t vb = n * 16;
  const int nrhs = nw * ncomp;
  DevBuf dots, work;
  dots.ensure((size_t)nrhs * ncomp * 16);
  work.ensure((size_t)nrhs * 1024 * 16);
  auto fetch = [&](size_t cnt) {
    std::vector<cplx> h(cnt);
    HIP_CHECK(hipMemcpyAsync(h.data(), dots.p, cnt * 16, hipMemcpyDeviceToHost, st));
    sync();
    return h;
  };
  // ep[r][a] = eta^a . X_r(w) for every right-hand side r
  std::vector<cplx> ep(nrhs * ncomp);
  for (int a = 0; a < ncomp; ++a) {
    launch_batched_dot<double>(nrhs, n, Xp, n, (const char*)etaB + a * vb, 0, false, dots.p, work.p, st);
    auto h = fetch(nrhs);
    for (int r = 0; r < nrhs; ++r) ep[r * ncomp + a] = h[r];
  }
  // q[r][a] = X^a(-w_k) . H_r for r = k * ncomp + b
  DevBuf H;
  H.ensure((size_t)std::min(chunk, nrhs) * vb);
  for (int c0 = 0; c0 < nrhs; c0 += chunk) {
    const int nc = std::min(chunk, nrhs - c0);
    std::vector<int> cp(nc);
    for (int q = 0; q < nc; ++q) cp[q] = (c0 + q) % ncomp;
    eta_plus_fx(nc, cp.data(), (const char*)Xp + c0 * vb, H.p, prec, etaB);
    for (int q = 0; q < nc; ++q) {
      const int r = c0 + q, k = r / ncomp;
      for (int a = 0; a < ncomp; ++a)
        launch_batched_dot<double>(1, n, (const char*)Xm + ((size_t)k * ncomp + a) * vb, n, (char*)H.p + q * vb, n,
                                   false, (char*)dots.p + ((size_t)r * ncomp + a) * 16, work.p, st);
    }
  }
  const auto qv = fetch((size_t)nrhs * ncomp);
  out.assign(nw * ncomp * ncomp, 0.0);
  for (int k = 0; k < nw; ++k)
    for (int a = 0; a < ncomp; ++a)
      for (int b = 0; b < ncomp; ++b) {
        const int ra = k * ncomp + a, rb = k * ncomp + b;
        const cplx fp = ep[rb * ncomp + a] + qv[rb * ncomp + a];  // eta^a.X^b(w) + X^a(-w).H^b
        const cplx fm = ep[ra * ncomp + b] + qv[ra * ncomp + b];  // eta^b.X^a(w) + X^b(-w).H^a
        out[(k * ncomp + a) * ncomp + b] = -0.5 * (fp + std::conj(fm));
      }
}

}  // namespace lrcc
