// Host-only checks of the library's bookkeeping, built with AddressSanitizer
// and UndefinedBehaviorSanitizer (tests/test_sanitizers.py): the workspace
// arena's first-fit allocator, and the program parser and transforms,
// including their error paths.  No device is touched.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "common.h"
#include "devmem.h"
#include "program.h"
#include "runtime.h"

using namespace lrcc;

static int failures = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                 \
    }                                                             \
  } while (0)

static void arena_checks() {
  // a fake, unaligned base: the arena only does bookkeeping on it
  char* base = reinterpret_cast<char*>(uintptr_t(1) << 32) + 7;
  const size_t size = size_t(64) << 20;
  Arena a(base, size);
  const size_t free0 = a.free_bytes(), largest0 = a.largest_free();
  CHECK(largest0 == free0 && free0 <= size);
  std::mt19937_64 rng(5);
  std::vector<void*> live;
  for (int round = 0; round < 2000; ++round) {
    if (live.empty() || (rng() % 3 != 0 && live.size() < 200)) {
      const size_t b = 1 + rng() % (size / 64);
      try {
        void* p = a.alloc(b);
        CHECK(a.owns(p) && (reinterpret_cast<uintptr_t>(p) & 255) == 0);
        live.push_back(p);
      } catch (const Error& e) {
        CHECK(e.code == LRCC_E_NOMEM);
      }
    } else {
      const size_t k = rng() % live.size();
      a.free(live[k]);
      live.erase(live.begin() + (long)k);
    }
  }
  for (void* p : live) a.free(p);
  CHECK(a.free_bytes() == free0 && a.largest_free() == largest0);  // every range coalesced back
  CHECK(a.peak() <= size);
  bool threw = false;
  try {
    a.alloc(size + 1);
  } catch (const Error& e) {
    threw = e.code == LRCC_E_NOMEM;
  }
  CHECK(threw);
  CHECK(!a.owns(base + size + 512));
}

static void program_checks() {
  CcPrograms P;
  build_programs(P);
  const OpList* lists[] = {&P.residual, &P.right, &P.left, &P.eta0,       &P.xi,      &P.gradL,
                           &P.hvp,      &P.hvpt,  &P.fnspp, &P.ring_setup, &P.right_f, &P.left_f};
  CHECK(P.m.forward.empty());
  CHECK(P.right_f.size() < P.right.size() && P.left_f.size() < P.left.size());
  for (const OpList* l : lists) {
    CHECK(!l->empty());
    CHECK(!serialize(P.m, *l).empty() && !dump(P.m, *l).empty());
    // the planner over every list at a few batch sizes
    const Dims d{5, 9, 10, 36};
    for (int nb : {1, 3, 8}) {
      PoolPlan pl = plan_pool(P.m, d, *l, nb, {}, nullptr);
      for (size_t k = 1; k < pl.slot_elems.size(); ++k) CHECK(pl.slot_elems[k - 1] >= pl.slot_elems[k]);
      for (auto& ts : pl.slot) CHECK(ts.second >= 0 && ts.second < (int)pl.slot_elems.size());
    }
  }
  // transforms of a small program: tangent, adjoint, pruning
  Module m;
  OpList prog = parse_program(m, "input x[ia]\nconst g[iajb]\ny[jb] = x[ia] * g[iajb]\nz[ia] = 2 * y[ia]\n");
  CHECK(prog.size() == 2);
  std::map<int, int> tan;
  tan[m.find("x")] = m.add("dx", "ov", Role::Tangent, true);
  OpList jp = jvp(m, prog, tan, {m.find("z")});
  CHECK(jp.size() == 2);
  std::map<int, int> adj;
  adj[m.find("z")] = m.add("gz", "ov", Role::Adjoint, true);
  OpList vp = vjp(m, prog, adj, {m.find("x")}, true);
  CHECK(vp.size() == 2);
  CHECK(prune(m, vp, {adj.at(m.find("x"))}).size() == 2);
  // via terms: y = a . w(u) with w = u . g; the first derivatives through w
  // take du . Z (Z formed by a later program) instead of forming dw
  {
    Module mv;
    OpList pv = parse_program(mv, "input a[ik] u[kl]\nconst g[lj]\nw[kj] = u[kl] * g[lj]\n"
                                  "y[ij] = a[ik] * w[kj] | u[kl] * Z[iklj]\n");
    CHECK(mv.forward.size() == 1);
    OpList setup = parse_program(mv, "Z[iklj] = a[ik] * g[lj]\n");
    CHECK(setup.size() == 1 && mv.forward.empty());
    const int u = mv.find("u"), y = mv.find("y"), z = mv.find("Z");
    for (bool via : {false, true}) {
      std::map<int, int> tn{{u, mv.add(via ? "du1" : "du0", "oo", Role::Tangent, true)}};
      OpList d = prune(mv, jvp(mv, pv, tn, {y}, via ? "T1" : "T0", via), {tn.at(y)});
      CHECK(d.size() == (via ? 1u : 2u));
      if (via) CHECK(d[0].b == z && d[0].a == tn.at(u) && d[0].via.empty());
      std::map<int, int> an{{y, mv.add(via ? "gy1" : "gy0", "oo", Role::Adjoint, true)}};
      OpList g = prune(mv, vjp(mv, pv, an, {u}, true, via ? "A1" : "A0", via), {an.at(u)});
      CHECK(g.size() == (via ? 1u : 2u));
      if (via) CHECK(g[0].a == z && g[0].b == an.at(y));
    }
    const char* badv[] = {"input x[ia]\ny[ia] = 2 * x[ia] | x[ia] * Z[ia]\n",
                          "input a[ik] u[kl]\nconst g[kj]\ny[ij] = a[ik] * g[kj] | u[kl] * Z[kl]\n"};
    for (const char* t : badv) {
      Module mb;
      bool threw = false;
      try {
        parse_program(mb, t);
      } catch (const Error&) {
        threw = true;
      }
      CHECK(threw);
    }
    Module mf;
    parse_program(mf, "input a[ik] u[kl]\nconst g[kj]\ny[ij] = a[ik] * g[kj] | u[kl] * Z[iklj]\n");
    bool threw = false;
    try {
      parse_program(mf, "Z[iklj] += a[ik] * u[kl]\n");  // a forward-declared tensor's first write is '='
    } catch (const Error&) {
      threw = true;
    }
    CHECK(threw);
  }
  // malformed programs fail with an error, not a crash
  const char* bad[] = {"y[ia] = q[ia]\n", "input x[ia]\ny[ia] += x[ia]\n", "input x[ia]\ny[ab] = x[ia]\n",
                       "input x[ia]\ny[ia] = x[ia] *\n", "input x[ia]\ny[ia] = unpack(x[ia], 7)\n",
                       "input x[iz]\n", "input x[ia]\nx[ia] = 2 * x[ia]\n"};
  for (const char* t : bad) {
    Module mb;
    bool threw = false;
    try {
      parse_program(mb, t);
    } catch (const Error&) {
      threw = true;
    }
    CHECK(threw);
  }
}

int main() {
  arena_checks();
  program_checks();
  if (failures) {
    std::fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
