// Contraction-program IR for the CC residual and its derivatives.
//
// The CCSD residual Omega(t) = <mu| exp(-T) H exp(T) |0> (Section II.A,
// Eqs. 9-10) is held once, as a list of tensor operations over named
// tensors with occupied/virtual index classes.  The Jacobian products the
// response theory needs are derived from it mechanically:
//   * right sigma  A X         (Eqs. 29-30)  = forward-mode tangent of Omega
//   * left sigma   lambda A    (Eqs. 22, 32) = reverse-mode adjoint of Omega
//   * xi^B                     (Eq. 31)      = tangent of Omega along f -> mu_B
//   * eta^B + F X^B            (Eqs. 33-34)  = tangent of grad_t L, L = E + lambda.Omega
// Every derived operation is again one of the four kinds below, so one
// executor (HIP kernels) runs them all.
//
// Index letters: i..n occupied, a..h virtual, I..N packed occupied pairs
// (i<j), A..H packed virtual pairs (a<b); '#' is the batch (right-hand
// side) index of batched tensors and is added by the planner.
#pragma once
#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace lrcc {

enum class Role { Input, Fock, Const, Temp, Tangent, Adjoint, Scalar1 };

struct TensorDecl {
  std::string name;
  std::string cls;   // one char per dim: 'o','v' (orbital), 'O','V' (packed pair)
  Role role;
  bool batched = false;
};

enum class OpKind { Add, Contract, Pack, Unpack, Zero };

// out[oi] (+)= alpha * a[ai] (* b[bi])
// Pack:   out (packed) <- a (full);   Unpack: out (full) <- a (packed).
// Pair modes per packed letter, in order: 0 = take upper triangle / scatter to
// upper triangle; 1 = antisymmetric gather x[pq]-x[qp] / antisymmetric expand.
struct Op {
  OpKind kind = OpKind::Add;
  bool acc = false;
  double are = 1.0, aim = 0.0;
  int out = -1;
  std::string oi;
  int a = -1;
  std::string ai;
  int b = -1;
  std::string bi;
  int mode[2] = {0, 0};
  // Derivative annotations (the op itself runs as written):
  //  nodiff    an Add whose contribution the derivative programs leave out;
  //  partner   a Contract whose derivative with respect to its first
  //            operand a takes the tensor `partner` (same indices as b) in
  //            place of b.
  // Together they express a term a . W(a) in which W = W1 + Y(a), with Y
  // linear in a, and the output is read only through an antisymmetrizer
  // under which a . Y(c) = c . Y(a): its derivative along da is then
  // da . (W1 + 2 Y) + a . dW1, one contraction with da fewer.
  bool nodiff = false;
  int partner = -1;
  //  via       a Contract whose first-order derivative through its second
  //            operand b is given directly as sum_k du_k[vi] * Z_k[zi], with u_k
  //            the variables b depends on and Z_k primal tensors a setup
  //            program forms (a re-association: the derivative programs
  //            that use it contract the small tangent du_k with a
  //            precomputed Z_k instead of forming db and contracting it with
  //            the first operand).  Valid for first derivatives only: a
  //            program differentiated again must not use it, since Z_k's own
  //            dependence on the variables is not part of the program.
  struct Via {
    int var = -1;
    std::string vi;
    int z = -1;
    std::string zi;
  };
  std::vector<Via> via;
};

using OpList = std::vector<Op>;

struct Module {
  std::vector<TensorDecl> tensors;
  std::map<std::string, int> by_name;
  // persistent[id] = 1: an unbatched temporary that some program reads
  // before writing it (a primal intermediate or a gradient that another
  // program consumes).  The executor keeps such tensors between runs; other
  // unbatched temporaries that a program both writes and reads live only
  // for that run.
  std::vector<char> persistent;
  // Tensors named by a `via` hint before any program writes them; the
  // program that forms them may then write them with '=' once.
  std::set<int> forward;
  int add(const std::string& name, const std::string& cls, Role role, bool batched = false);
  int find(const std::string& name) const;  // -1 if absent
  const TensorDecl& operator[](int i) const { return tensors.at(i); }
};

char letter_class(char c);

// Parse the statement language (one statement per line, '#' comments):
//   input  t1[ia] t2p[IA]         declares tensors with a role
//   fock   foo[ij] ...
//   const  goovv[ijab] ...
//   X[idx]  = [c *] A[idx]                      Add (permuted copy)
//   X[idx] += [c *] A[idx] * B[idx]             Contract
//   X[idx] += [c *] pack(A[idx], m1[, m2])      Pack / unpack(...) Unpack
//   X[idx] += nodiff(A[idx])                    Add left out of derivatives
//   X[idx] = A[idx] * B[idx] ~ C[idx]           Contract; d/dA takes C for B
//   X[idx] = A[idx] * B[idx] ... | u[i1] * Z[i2] + v[i3] * Y[i4]
//                                               the same, with `via` terms for d/dB
OpList parse_program(Module& m, const std::string& text);

// Forward-mode tangent program.  `tan` maps seed tensors to their (batched)
// tangent tensors on entry and is extended with every tangent created.
// `want` lists primal tensors whose tangents must be produced (zero-filled
// if they receive no contribution).
// With use_via, a Contract carrying `via` terms takes its derivative
// through b from them.
OpList jvp(Module& m, const OpList& prog, std::map<int, int>& tan, const std::vector<int>& want,
           const std::string& tag = "d", bool use_via = false);

// Reverse-mode adjoint program.  `adj` maps output tensors to their
// cotangent tensors on entry; `wrt` lists inputs whose adjoints are wanted.
// Adjoints are created batched if `batched`.
OpList vjp(Module& m, const OpList& prog, std::map<int, int>& adj, const std::vector<int>& wrt,
           bool batched, const std::string& tag = "g", bool use_via = false);

// Remove ops that do not contribute to `keep`.
OpList prune(const Module& m, const OpList& prog, const std::vector<int>& keep);

std::string dump(const Module& m, const OpList& prog);
// Machine-readable form: the tensor table, then one line per op.
//   T <id> <name> <cls|-> <role> <batched>
//   O <kind> <acc> <are> <aim> <out> <oi|-> <a> <ai|-> <b> <bi|-> <m0> <m1>
std::string serialize(const Module& m, const OpList& prog);

// The CCSD residual and energy as a program over the module's tensors.
extern const char* kCcsdProgram;

// Singles and doubles projections of the perturbation operator over the MP2
// doubles (the numerators of the FNS++ first-order amplitudes).
extern const char* kFnsppProgram;

// Primal setup of the tensors the ring contraction's via terms read.
extern const char* kRingSetup;

// All programs the solvers run, derived from kCcsdProgram.
struct CcPrograms {
  Module m;
  OpList residual;  // O1, O2p, E from t1, t2p, f, <||>          (primal, all temps kept)
  OpList right;     // dO = A dt                                 (tangent, batched)
  OpList left;      // g_t = gO A                                (adjoint, batched)
  OpList eta0;      // dE/dt                                     (adjoint of E, unbatched)
  OpList xi;        // dO along f -> mu                          (tangent in f, batched)
  OpList gradL;     // d/dt (E + lambda.Omega)                   (adjoint, unbatched)
  OpList hvp;       // tangent of gradL along (dt, df)           (batched)
  OpList hvpt;      // tangent of gradL along dt only: F dt      (batched)
  OpList ring_setup;  // Z1, Z2 of the ring's via terms            (primal, once per t)
  OpList right_f;     // right with the ring's via terms (reads Z1, Z2; same tensors as right)
  OpList left_f;      // left with the ring's via terms (same tensors as left)
  // tensor ids
  int t1, t2p, foo, fov, fvo, fvv, O1, O2p, E, one;
  int r_dt1, r_dt2p, r_dO1, r_dO2p;           // right
  int l_gO1, l_gO2p, l_gt1, l_gt2p;           // left
  int e_gt1, e_gt2p;                          // eta0
  int x_df[4], x_dO1, x_dO2p;                 // xi (df in foo, fov, fvo, fvv order)
  int g_lam1, g_lam2p, g_gt1, g_gt2p;         // gradL
  int h_dt1, h_dt2p, h_df[4], h_out1, h_out2p;  // hvp
  int f_dt1, f_dt2p, f_out1, f_out2p;           // hvpt
  OpList fnspp;                                 // Abar_i^a, Abar_ij^ac from (t2 MP2, A)
  int n_t2, n_A[4], n_s1, n_s2;
};
void build_programs(CcPrograms& P);
// Marks in m.persistent the unbatched temporaries read by some program of
// `progs` before that program writes them.
void mark_persistent(Module& m, const std::vector<const OpList*>& progs);

}  // namespace lrcc
