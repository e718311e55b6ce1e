// Contraction-program IR: parser, forward/reverse transforms, pruning.
#include "program.h"

#include <algorithm>
#include <cctype>
#include <regex>
#include <sstream>

#include "common.h"

namespace lrcc {

char letter_class(char c) {
  if (c >= 'i' && c <= 'n') return 'o';
  if (c >= 'a' && c <= 'h') return 'v';
  if (c >= 'I' && c <= 'N') return 'O';
  if (c >= 'A' && c <= 'H') return 'V';
  throw Error(LRCC_E_INTERNAL, std::string("bad index letter '") + c + "'");
}

static std::string classes_of(const std::string& idx) {
  std::string s;
  for (char c : idx) s += letter_class(c);
  return s;
}

int Module::add(const std::string& name, const std::string& cls, Role role, bool batched) {
  if (by_name.count(name)) throw Error(LRCC_E_INTERNAL, "duplicate tensor " + name);
  tensors.push_back(TensorDecl{name, cls, role, batched});
  by_name[name] = (int)tensors.size() - 1;
  return (int)tensors.size() - 1;
}

int Module::find(const std::string& name) const {
  auto it = by_name.find(name);
  return it == by_name.end() ? -1 : it->second;
}

static std::string trim(const std::string& s) {
  size_t b = s.find_first_not_of(" \t\r");
  if (b == std::string::npos) return "";
  size_t e = s.find_last_not_of(" \t\r");
  return s.substr(b, e - b + 1);
}

OpList parse_program(Module& m, const std::string& text) {
  static const std::regex re_decl(R"(^(input|fock|const|scalar1)\s+(.*)$)");
  static const std::regex re_ref(R"((\w+)\[(\w*)\])");
  static const std::regex re_stmt(R"(^(\w+)\[(\w*)\]\s*(\+?=)\s*(.*)$)");
  static const std::regex re_coef(R"(^([-+]?[0-9]*\.?[0-9]+(?:[eE][-+]?[0-9]+)?)\s*\*\s*(.*)$)");
  static const std::regex re_pack(R"(^(pack|unpack)\(\s*(\w+)\[(\w*)\]\s*,\s*([01])(?:\s*,\s*([01]))?\s*\)$)");
  static const std::regex re_prod(R"(^(\w+)\[(\w*)\]\s*\*\s*(\w+)\[(\w*)\]$)");
  static const std::regex re_one(R"(^(\w+)\[(\w*)\]$)");
  static const std::regex re_nodiff(R"(^nodiff\(\s*(\w+)\[(\w*)\]\s*\)$)");
  static const std::regex re_partner(R"(^(\w+)\[(\w*)\]\s*\*\s*(\w+)\[(\w*)\]\s*~\s*(\w+)\[(\w*)\]$)");
  static const std::regex re_viaterm(R"(^(\w+)\[(\w*)\]\s*\*\s*(\w+)\[(\w*)\]$)");

  OpList ops;
  std::set<int> read;      // tensors already read (no further writes allowed)
  std::set<int> written;
  std::istringstream in(text);
  std::string line;
  int lineno = 0;
  auto fail = [&](const std::string& msg) {
    throw Error(LRCC_E_INTERNAL, "program line " + std::to_string(lineno) + ": " + msg + " [" + line + "]");
  };
  auto use = [&](const std::string& name, const std::string& idx) {
    int id = m.find(name);
    if (id < 0) fail("unknown tensor " + name);
    if (m[id].cls != classes_of(idx)) fail("index classes of " + name + "[" + idx + "] do not match " + m[id].cls);
    read.insert(id);
    return id;
  };
  while (std::getline(in, line)) {
    ++lineno;
    std::string s = line.substr(0, line.find('#'));
    s = trim(s);
    if (s.empty()) continue;
    std::smatch mt;
    if (std::regex_match(s, mt, re_decl)) {
      Role role = mt[1] == "input" ? Role::Input : mt[1] == "fock" ? Role::Fock
                : mt[1] == "const" ? Role::Const : Role::Scalar1;
      std::string rest = mt[2];
      for (auto it = std::sregex_iterator(rest.begin(), rest.end(), re_ref); it != std::sregex_iterator(); ++it)
        m.add((*it)[1], classes_of((*it)[2]), role);
      continue;
    }
    if (!std::regex_match(s, mt, re_stmt)) fail("cannot parse");
    Op op;
    std::string oname = mt[1], oidx = mt[2], rhs = trim(mt[4]);
    op.acc = (mt[3] == "+=");
    int out = m.find(oname);
    if (out < 0) {
      if (op.acc) fail("first write of " + oname + " must be '='");
      out = m.add(oname, classes_of(oidx), Role::Temp);
    } else {
      if (m[out].role != Role::Temp) fail("cannot write " + oname);
      if (read.count(out)) fail(oname + " written after being read");
      if (!op.acc && !m.forward.count(out)) fail(oname + " overwritten");
      if (op.acc && m.forward.count(out)) fail("first write of " + oname + " must be '='");
      if (m[out].cls != classes_of(oidx)) fail("index classes of " + oname);
      m.forward.erase(out);
    }
    written.insert(out);
    op.out = out;
    op.oi = oidx;
    std::string via_text;
    const size_t bar = rhs.find('|');
    if (bar != std::string::npos) {
      via_text = trim(rhs.substr(bar + 1));
      rhs = trim(rhs.substr(0, bar));
    }
    std::smatch mc;
    if (std::regex_match(rhs, mc, re_coef)) {
      op.are = std::stod(mc[1]);
      rhs = trim(mc[2]);
    }
    std::smatch mx;
    if (std::regex_match(rhs, mx, re_pack)) {
      op.kind = mx[1] == "pack" ? OpKind::Pack : OpKind::Unpack;
      op.a = use(mx[2], mx[3]);
      op.ai = mx[3];
      op.mode[0] = std::stoi(mx[4]);
      op.mode[1] = mx[5].matched ? std::stoi(mx[5]) : 0;
    } else if (std::regex_match(rhs, mx, re_prod)) {
      op.kind = OpKind::Contract;
      op.a = use(mx[1], mx[2]);
      op.ai = mx[2];
      op.b = use(mx[3], mx[4]);
      op.bi = mx[4];
    } else if (std::regex_match(rhs, mx, re_partner)) {
      op.kind = OpKind::Contract;
      op.a = use(mx[1], mx[2]);
      op.ai = mx[2];
      op.b = use(mx[3], mx[4]);
      op.bi = mx[4];
      if (mx[6] != mx[4]) fail("the partner must carry the indices of the second operand");
      op.partner = use(mx[5], mx[6]);
      if (m[op.partner].cls != m[op.b].cls) fail("partner and second operand differ in class");
    } else if (std::regex_match(rhs, mx, re_nodiff)) {
      op.kind = OpKind::Add;
      op.nodiff = true;
      op.a = use(mx[1], mx[2]);
      op.ai = mx[2];
      if (!op.acc) fail("nodiff must accumulate into a tensor written before");
      std::string x = op.ai, y = op.oi;
      std::sort(x.begin(), x.end());
      std::sort(y.begin(), y.end());
      if (x != y) fail("copy must permute indices");
    } else if (std::regex_match(rhs, mx, re_one)) {
      op.kind = OpKind::Add;
      op.a = use(mx[1], mx[2]);
      op.ai = mx[2];
      std::string x = op.ai, y = op.oi;
      std::sort(x.begin(), x.end());
      std::sort(y.begin(), y.end());
      if (x != y) fail("copy must permute indices");
    } else {
      fail("bad right-hand side");
    }
    if (!via_text.empty()) {
      if (op.kind != OpKind::Contract) fail("via terms need a contraction");
      std::istringstream terms(via_text);
      std::string term;
      while (std::getline(terms, term, '+')) {
        term = trim(term);
        std::smatch mv;
        if (!std::regex_match(term, mv, re_viaterm)) fail("bad via term '" + term + "'");
        Op::Via vt;
        vt.var = use(mv[1], mv[2]);
        vt.vi = mv[2];
        vt.z = m.find(mv[3]);
        if (vt.z < 0) {  // formed later by a setup program
          vt.z = m.add(mv[3], classes_of(mv[4]), Role::Temp);
          m.forward.insert(vt.z);
        }
        vt.z = use(mv[3], mv[4]);
        vt.zi = mv[4];
        // the term must produce the op's output indices
        std::string have = vt.vi + vt.zi, want = op.oi;
        for (char c : want)
          if (have.find(c) == std::string::npos) fail("via term does not carry index " + std::string(1, c));
        op.via.push_back(vt);
      }
      if (op.via.empty()) fail("empty via list");
    }
    if (op.a == op.out || op.b == op.out || op.partner == op.out) fail("in-place update");
    ops.push_back(op);
  }
  return ops;
}

// A derived tensor by name: a second derivation with the same tag (a variant
// of a program) reuses the tensors of the first.
static int derived_tensor(Module& m, const std::string& name, const std::string& cls, Role role, bool batched) {
  const int id = m.find(name);
  if (id < 0) return m.add(name, cls, role, batched);
  if (m[id].cls != cls || m[id].role != role || m[id].batched != batched)
    throw Error(LRCC_E_INTERNAL, "derived tensor " + name + " redeclared differently");
  return id;
}

static int tangent_of(Module& m, std::map<int, int>& tan, int t, const std::string& tag) {
  auto it = tan.find(t);
  if (it != tan.end()) return it->second;
  const int id = derived_tensor(m, tag + "(" + m[t].name + ")", m[t].cls, Role::Tangent, true);
  tan[t] = id;
  return id;
}

OpList jvp(Module& m, const OpList& prog, std::map<int, int>& tan, const std::vector<int>& want,
           const std::string& tag, bool use_via) {
  std::set<int> live;
  for (auto& kv : tan) live.insert(kv.first);
  OpList out;
  for (const Op& op : prog) {
    std::vector<Op> contrib;
    auto lv = [&](int t) { return t >= 0 && live.count(t) > 0; };
    if (op.kind == OpKind::Zero) {
      live.erase(op.out);
      continue;
    }
    if (op.nodiff) continue;  // left out of derivatives (an accumulation: liveness unchanged)
    if (op.kind == OpKind::Contract) {
      if (lv(op.a)) {
        Op c = op;
        c.a = tangent_of(m, tan, op.a, tag);
        if (op.partner >= 0) c.b = op.partner;
        c.partner = -1;
        c.via.clear();
        contrib.push_back(c);
      }
      if (lv(op.b) && use_via && !op.via.empty()) {
        for (const Op::Via& vt : op.via) {
          if (!lv(vt.var)) continue;  // a variable with no tangent contributes nothing
          Op c = op;
          c.a = tangent_of(m, tan, vt.var, tag);
          c.ai = vt.vi;
          c.b = vt.z;
          c.bi = vt.zi;
          c.partner = -1;
          c.via.clear();
          contrib.push_back(c);
        }
      } else if (lv(op.b)) {
        Op c = op;
        c.b = tangent_of(m, tan, op.b, tag);
        c.partner = -1;
        c.via.clear();
        contrib.push_back(c);
      }
    } else if (lv(op.a)) {
      Op c = op;
      c.a = tangent_of(m, tan, op.a, tag);
      contrib.push_back(c);
    }
    if (!op.acc) live.erase(op.out);
    bool first = !live.count(op.out);
    for (Op& c : contrib) {
      c.out = tangent_of(m, tan, op.out, tag);
      c.acc = !first;
      first = false;
      out.push_back(c);
    }
    if (!contrib.empty()) live.insert(op.out);
  }
  for (int w : want) {
    if (!live.count(w)) {
      Op z;
      z.kind = OpKind::Zero;
      z.out = tangent_of(m, tan, w, tag);
      out.push_back(z);
    }
  }
  return out;
}

OpList vjp(Module& m, const OpList& prog, std::map<int, int>& adj, const std::vector<int>& wrt,
           bool batched, const std::string& tag, bool use_via) {
  std::set<int> act(wrt.begin(), wrt.end());
  for (const Op& op : prog)
    if (!op.nodiff && (act.count(op.a) || (op.b >= 0 && act.count(op.b)))) act.insert(op.out);
  std::set<int> live;
  for (auto& kv : adj) live.insert(kv.first);
  auto adjoint = [&](int t) {
    auto it = adj.find(t);
    if (it != adj.end()) return it->second;
    const int id = derived_tensor(m, tag + "(" + m[t].name + ")", m[t].cls, Role::Adjoint, batched);
    adj[t] = id;
    return id;
  };
  OpList out;
  auto emit = [&](Op c, int target) {
    c.out = adjoint(target);
    c.acc = live.count(target) > 0;
    live.insert(target);
    out.push_back(c);
  };
  for (auto it = prog.rbegin(); it != prog.rend(); ++it) {
    const Op& op = *it;
    if (op.kind == OpKind::Zero || op.nodiff || !live.count(op.out)) {
      if (!op.acc) live.erase(op.out);
      continue;
    }
    int g = adj.at(op.out);
    Op c;
    c.are = op.are;
    c.aim = op.aim;
    switch (op.kind) {
      case OpKind::Add:
        if (act.count(op.a)) {
          c.kind = OpKind::Add;
          c.oi = op.ai;
          c.a = g;
          c.ai = op.oi;
          emit(c, op.a);
        }
        break;
      case OpKind::Contract:
        if (act.count(op.a)) {
          Op d = c;
          d.kind = OpKind::Contract;
          d.oi = op.ai;
          d.a = g;
          d.ai = op.oi;
          d.b = op.partner >= 0 ? op.partner : op.b;
          d.bi = op.bi;
          emit(d, op.a);
        }
        if (act.count(op.b) && use_via && !op.via.empty()) {
          for (const Op::Via& vt : op.via) {
            if (!act.count(vt.var)) continue;
            Op d = c;
            d.kind = OpKind::Contract;
            d.oi = vt.vi;
            d.a = vt.z;
            d.ai = vt.zi;
            d.b = g;
            d.bi = op.oi;
            emit(d, vt.var);
          }
        } else if (act.count(op.b)) {
          Op d = c;
          d.kind = OpKind::Contract;
          d.oi = op.bi;
          d.a = op.a;
          d.ai = op.ai;
          d.b = g;
          d.bi = op.oi;
          emit(d, op.b);
        }
        break;
      case OpKind::Pack:
      case OpKind::Unpack:
        if (act.count(op.a)) {
          c.kind = op.kind == OpKind::Pack ? OpKind::Unpack : OpKind::Pack;
          c.oi = op.ai;
          c.a = g;
          c.ai = op.oi;
          c.mode[0] = op.mode[0];
          c.mode[1] = op.mode[1];
          emit(c, op.a);
        }
        break;
      default:
        break;
    }
    if (!op.acc) live.erase(op.out);
  }
  for (int w : wrt) {
    if (!live.count(w)) {
      Op z;
      z.kind = OpKind::Zero;
      z.out = adjoint(w);
      out.push_back(z);
      live.insert(w);
    }
  }
  return out;
}

OpList prune(const Module& m, const OpList& prog, const std::vector<int>& keep) {
  (void)m;
  std::set<int> need(keep.begin(), keep.end());
  std::vector<char> use(prog.size(), 0);
  for (int k = (int)prog.size() - 1; k >= 0; --k) {
    const Op& op = prog[k];
    if (!need.count(op.out)) continue;
    use[k] = 1;
    if (op.a >= 0) need.insert(op.a);
    if (op.b >= 0) need.insert(op.b);
    if (op.partner >= 0) need.insert(op.partner);
  }
  OpList out;
  for (size_t k = 0; k < prog.size(); ++k)
    if (use[k]) out.push_back(prog[k]);
  return out;
}

std::string dump(const Module& m, const OpList& prog) {
  std::ostringstream os;
  for (const Op& op : prog) {
    const auto& o = m[op.out];
    os << o.name << (o.batched ? "#" : "") << "[" << op.oi << "] ";
    if (op.kind == OpKind::Zero) {
      os << "= 0\n";
      continue;
    }
    os << (op.acc ? "+= " : "= ");
    os << op.are;
    if (op.aim != 0) os << (op.aim > 0 ? "+" : "") << op.aim << "i";
    os << " * ";
    auto ref = [&](int t, const std::string& idx) {
      return m[t].name + (m[t].batched ? "#" : "") + "[" + idx + "]";
    };
    switch (op.kind) {
      case OpKind::Add: os << (op.nodiff ? "nodiff(" : "") << ref(op.a, op.ai) << (op.nodiff ? ")" : ""); break;
      case OpKind::Contract:
        os << ref(op.a, op.ai) << " * " << ref(op.b, op.bi);
        if (op.partner >= 0) os << " ~ " << ref(op.partner, op.bi);
        for (size_t k = 0; k < op.via.size(); ++k)
          os << (k ? " + " : " | ") << ref(op.via[k].var, op.via[k].vi) << " * " << ref(op.via[k].z, op.via[k].zi);
        break;
      case OpKind::Pack:
      case OpKind::Unpack:
        os << (op.kind == OpKind::Pack ? "pack(" : "unpack(") << ref(op.a, op.ai) << ", " << op.mode[0]
           << ", " << op.mode[1] << ")";
        break;
      default: break;
    }
    os << "\n";
  }
  return os.str();
}

std::string serialize(const Module& m, const OpList& prog) {
  std::ostringstream os;
  os.precision(17);
  for (size_t k = 0; k < m.tensors.size(); ++k) {
    const auto& t = m.tensors[k];
    os << "T " << k << " " << t.name << " " << (t.cls.empty() ? "-" : t.cls) << " " << (int)t.role << " "
       << (int)t.batched << "\n";
  }
  auto s = [](const std::string& x) { return x.empty() ? std::string("-") : x; };
  for (const Op& op : prog)
    os << "O " << (int)op.kind << " " << (int)op.acc << " " << op.are << " " << op.aim << " " << op.out << " "
       << s(op.oi) << " " << op.a << " " << s(op.ai) << " " << op.b << " " << s(op.bi) << " " << op.mode[0] << " "
       << op.mode[1] << " " << (int)op.nodiff << " " << op.partner << "\n";
  return os.str();
}

// CCSD residual Omega(t) and energy E(t) for complex spinors (standard
// spin-orbital CCSD; singles driver f_ai, doubles driver <ab||ij>; the full
// Fock matrix appears in F_ae and F_mi, so Omega includes its diagonal part).
// The vvvv term is written on packed pairs (the ladder) and the vovv/tau
// contraction Z is factored out of W_abef; the quarter of tau<mn||ef>tau
// that belongs to W_abef is folded into W_mnij (coefficient 1/2).  W_mbej is
// stored in ring order [j b m e] and its doubles term written with (e,f)
// swapped in both factors, so both ring contractions of a Jacobian product
// read the doubles in the same permuted order [i a m e].  The part of
// W_mbej quadratic in t2, Y = -1/2 t2 <mn||fe>, enters the ring term
// t2 . (W1 + Y(t2)), which is read only through the antisymmetrizer of O2p;
// there t2 . Y(c) = c . Y(t2) (swap (i,a) <-> (j,b), m <-> n, e <-> f), so
// its derivative along dt is dt . (W1 + 2 Y) + t2 . dW1: the derivative
// programs run one (ov)^3 ring contraction fewer (nodiff / partner below).
// The remaining t2 . dW1 is linear in dt1 alone (W1 depends on t1 and the
// integrals only): t2[imae] dW1[jbme] = dt1[jf] Z1[iabf] + dt1[nb] Z2[ianj]
// with Z1, Z2 formed once per t by kRingSetup, so first-derivative programs
// built with via terms replace that o^3 v^3 contraction per right-hand side
// by two of o^2 v^3 and o^3 v^2 (the via list below).
const char* kCcsdProgram = R"(
input  t1[ia] t2p[IA]
fock   foo[ij] fov[ia] fvo[ai] fvv[ab]
const  goooo[ijkl] gooov[ijka] goovv[ijab] govvo[iabj] govvv[iabc] gvvoo[abij] gvvvo[abci] govoo[iajk]
const  govvp[iaE] W[AE]

t2[ijab]    = unpack(t2p[IA], 1, 1)
tt[ijab]    = t1[ia] * t1[jb]
tau[ijab]   = t2[ijab]
tau[ijab]  += tt[ijab]
tau[ijab]  += -1 * tt[ijba]
taut[ijab]  = t2[ijab]
taut[ijab] += 0.5 * tt[ijab]
taut[ijab] += -0.5 * tt[ijba]

Fae[ae]  = fvv[ae]
Fae[ae] += -0.5 * fov[me] * t1[ma]
Fae[ae] += t1[mf] * govvv[mafe]
Fae[ae] += -0.5 * taut[mnaf] * goovv[mnef]
Fmi[mi]  = foo[mi]
Fmi[mi] += 0.5 * t1[ie] * fov[me]
Fmi[mi] += t1[ne] * gooov[mnie]
Fmi[mi] += 0.5 * taut[inef] * goovv[mnef]
Fme[me]  = fov[me]
Fme[me] += t1[nf] * goovv[mnef]

Xmnij[mnij]  = t1[je] * gooov[mnie]
Wmnij[mnij]  = goooo[mnij]
Wmnij[mnij] += Xmnij[mnij]
Wmnij[mnij] += -1 * Xmnij[mnji]
Wmnij[mnij] += 0.5 * tau[ijef] * goovv[mnef]

Xmnej[mnej]  = t1[jf] * goovv[mnef]
W1[jbme]     = govvo[mbej]
W1[jbme]    += t1[jf] * govvv[mbef]
W1[jbme]    += t1[nb] * gooov[mnje]
W1[jbme]    += -1 * t1[nb] * Xmnej[mnej]
Yq[jbme]     = -0.5 * t2[jnbf] * goovv[mnfe]
Wmbej[jbme]  = W1[jbme]
Wmbej[jbme] += nodiff(Yq[jbme])
W2[jbme]     = W1[jbme]
W2[jbme]    += 2 * Yq[jbme]

O1[ia]  = fvo[ai]
O1[ia] += t1[ie] * Fae[ae]
O1[ia] += -1 * t1[ma] * Fmi[mi]
O1[ia] += t2[imae] * Fme[me]
O1[ia] += t1[nf] * govvo[nafi]
O1[ia] += -0.5 * t2[imef] * govvv[maef]
O1[ia] += 0.5 * t2[mnae] * gooov[nmie]

Ft[be]   = Fae[be]
Ft[be]  += -0.5 * t1[mb] * Fme[me]
Fmt[mj]  = Fmi[mj]
Fmt[mj] += 0.5 * t1[je] * Fme[me]
Xmbij[mbij] = t1[ie] * govvo[mbej]

Pab[ijab]    = t2[ijae] * Ft[be]
Pab[ijab]   += -1 * t1[ma] * govoo[mbij]
Pij[ijab]    = -1 * t2[imab] * Fmt[mj]
Pij[ijab]   += t1[ie] * gvvvo[abej]
Pijab[ijab]  = t2[imae] * Wmbej[jbme] ~ W2[jbme] | t1[jf] * Z1[iabf] + t1[nb] * Z2[ianj]
Pijab[ijab] += -1 * t1[ma] * Xmbij[mbij]
S0[ijab]     = gvvoo[abij]
S0[ijab]    += 0.5 * tau[mnab] * Wmnij[mnij]

taup[IA] = pack(tau[ijab], 0, 0)
Zp[Ima]  = taup[IE] * govvp[maE]
Zb[Iab]  = Zp[Ima] * t1[mb]

O2p[IA]  = taup[IE] * W[AE]
O2p[IA] += pack(Zb[Iab], 1)
O2p[IA] += pack(S0[ijab], 0, 0)
O2p[IA] += pack(Pab[ijab], 0, 1)
O2p[IA] += pack(Pij[ijab], 1, 0)
O2p[IA] += pack(Pijab[ijab], 1, 1)

Xjb[jb] = goovv[ijab] * t1[ia]
E[]  = fov[ia] * t1[ia]
E[] += 0.25 * goovv[ijab] * t2[ijab]
E[] += 0.5 * Xjb[jb] * t1[jb]
)";

// The tensors of the via terms of the ring contraction, from the primal
// intermediates t2, t1 and X_mnej of kCcsdProgram:
//   Z1[iabf] = sum_me t2[imae] (<mb||ef> - sum_n t1[nb] <mn||ef>)
//   Z2[ianj] = sum_me t2[imae] (<mn||je> - X[mnej])
// (the dt1 coefficients of dW1: <mb||ef>, the -t1 X(dt1) term through
// X_mnej = t1 . <mn||ef>, and <mn||je> - X_mnej).  Forming Z1 costs o^2 v^4
// once per t.
const char* kRingSetup = R"(
Zq[ianf]  = t2[imae] * goovv[mnef]
Z1[iabf]  = t2[imae] * govvv[mbef]
Z1[iabf] += -1 * t1[nb] * Zq[ianf]
Z2[ianj]  = t2[imae] * gooov[mnje]
Z2[ianj] += -1 * t2[imae] * Xmnej[mnej]
)";

// Abar_i^a = A_ai + sum_me A_me t_im^ae;
// Abar_ij^ac = P(a,c) sum_e t_ij^ec A_ae - P(i,j) sum_m t_mj^ac A_mi.
const char* kFnsppProgram = R"(
input  tm2[ijab] Aoo[ij] Aov[ia] Avo[ai] Avv[ab]
s1[ia]    = Avo[ai]
s1[ia]   += tm2[imae] * Aov[me]
Tca[ijca] = tm2[ijec] * Avv[ae]
s2[ijac]  = Tca[ijca]
s2[ijac] += -1 * Tca[ijac]
Tmi[ijac] = Aoo[mi] * tm2[mjac]
s2[ijac] += -1 * Tmi[ijac]
s2[ijac] += Tmi[jiac]
)";

void mark_persistent(Module& m, const std::vector<const OpList*>& progs) {
  m.persistent.assign(m.tensors.size(), 0);
  for (const OpList* prog : progs) {
    std::set<int> written;
    for (const Op& op : *prog) {
      for (int u : {op.a, op.b}) {
        if (u < 0 || written.count(u)) continue;
        const TensorDecl& t = m[u];
        if (!t.batched && (t.role == Role::Temp || t.role == Role::Adjoint || t.role == Role::Tangent))
          m.persistent[u] = 1;
      }
      written.insert(op.out);
    }
  }
}

void build_programs(CcPrograms& P) {
  Module& m = P.m;
  P.residual = parse_program(m, kCcsdProgram);
  P.ring_setup = parse_program(m, kRingSetup);
  if (!m.forward.empty()) throw Error(LRCC_E_INTERNAL, "a via tensor is never formed");
  P.fnspp = parse_program(m, kFnsppProgram);
  P.n_t2 = m.find("tm2");
  P.n_A[0] = m.find("Aoo");
  P.n_A[1] = m.find("Aov");
  P.n_A[2] = m.find("Avo");
  P.n_A[3] = m.find("Avv");
  P.n_s1 = m.find("s1");
  P.n_s2 = m.find("s2");
  P.t1 = m.find("t1");
  P.t2p = m.find("t2p");
  P.foo = m.find("foo");
  P.fov = m.find("fov");
  P.fvo = m.find("fvo");
  P.fvv = m.find("fvv");
  P.O1 = m.find("O1");
  P.O2p = m.find("O2p");
  P.E = m.find("E");
  P.one = m.add("one", "", Role::Scalar1, false);
  const int fb[4] = {P.foo, P.fov, P.fvo, P.fvv};

  {  // right sigma: tangent of Omega along dt
    std::map<int, int> tan;
    P.r_dt1 = m.add("R(t1)", "ov", Role::Tangent, true);
    P.r_dt2p = m.add("R(t2p)", "OV", Role::Tangent, true);
    tan[P.t1] = P.r_dt1;
    tan[P.t2p] = P.r_dt2p;
    OpList ops = jvp(m, P.residual, tan, {P.O1, P.O2p}, "R");
    P.r_dO1 = tan.at(P.O1);
    P.r_dO2p = tan.at(P.O2p);
    P.right = prune(m, ops, {P.r_dO1, P.r_dO2p});
    // the same tangent tensors, with the ring's via terms
    std::map<int, int> tf{{P.t1, P.r_dt1}, {P.t2p, P.r_dt2p}};
    OpList fops = jvp(m, P.residual, tf, {P.O1, P.O2p}, "R", true);
    if (tf.at(P.O1) != P.r_dO1 || tf.at(P.O2p) != P.r_dO2p) throw Error(LRCC_E_INTERNAL, "right variant outputs");
    P.right_f = prune(m, fops, {P.r_dO1, P.r_dO2p});
  }
  {  // left sigma: adjoint of Omega with batched cotangents
    std::map<int, int> adj;
    P.l_gO1 = m.add("L(O1)", "ov", Role::Adjoint, true);
    P.l_gO2p = m.add("L(O2p)", "OV", Role::Adjoint, true);
    adj[P.O1] = P.l_gO1;
    adj[P.O2p] = P.l_gO2p;
    OpList ops = vjp(m, P.residual, adj, {P.t1, P.t2p}, true, "L");
    P.l_gt1 = adj.at(P.t1);
    P.l_gt2p = adj.at(P.t2p);
    P.left = prune(m, ops, {P.l_gt1, P.l_gt2p});
    // the same adjoint tensors, with the ring's via terms
    std::map<int, int> af{{P.O1, P.l_gO1}, {P.O2p, P.l_gO2p}};
    OpList fops = vjp(m, P.residual, af, {P.t1, P.t2p}, true, "L", true);
    if (af.at(P.t1) != P.l_gt1 || af.at(P.t2p) != P.l_gt2p) throw Error(LRCC_E_INTERNAL, "left variant outputs");
    P.left_f = prune(m, fops, {P.l_gt1, P.l_gt2p});
  }
  {  // eta0 = dE/dt
    std::map<int, int> adj;
    adj[P.E] = P.one;
    OpList ops = vjp(m, P.residual, adj, {P.t1, P.t2p}, false, "E");
    P.e_gt1 = adj.at(P.t1);
    P.e_gt2p = adj.at(P.t2p);
    P.eta0 = prune(m, ops, {P.e_gt1, P.e_gt2p});
  }
  {  // xi: tangent of Omega along the one-electron operator
    std::map<int, int> tan;
    const char* nm[4] = {"X(foo)", "X(fov)", "X(fvo)", "X(fvv)"};
    for (int k = 0; k < 4; ++k) {
      P.x_df[k] = m.add(nm[k], m[fb[k]].cls, Role::Tangent, true);
      tan[fb[k]] = P.x_df[k];
    }
    OpList ops = jvp(m, P.residual, tan, {P.O1, P.O2p}, "X");
    P.x_dO1 = tan.at(P.O1);
    P.x_dO2p = tan.at(P.O2p);
    P.xi = prune(m, ops, {P.x_dO1, P.x_dO2p});
  }
  {  // gradient of L = E + lambda.Omega (unbatched), then its tangent
    std::map<int, int> adj;
    P.g_lam1 = m.add("lam1", "ov", Role::Input, false);
    P.g_lam2p = m.add("lam2p", "OV", Role::Input, false);
    adj[P.E] = P.one;
    adj[P.O1] = P.g_lam1;
    adj[P.O2p] = P.g_lam2p;
    OpList ops = vjp(m, P.residual, adj, {P.t1, P.t2p}, false, "G");
    P.g_gt1 = adj.at(P.t1);
    P.g_gt2p = adj.at(P.t2p);
    P.gradL = prune(m, ops, {P.g_gt1, P.g_gt2p});

    OpList comb = P.residual;
    comb.insert(comb.end(), P.gradL.begin(), P.gradL.end());
    std::map<int, int> tan;
    P.h_dt1 = m.add("H(t1)", "ov", Role::Tangent, true);
    P.h_dt2p = m.add("H(t2p)", "OV", Role::Tangent, true);
    tan[P.t1] = P.h_dt1;
    tan[P.t2p] = P.h_dt2p;
    const char* nm[4] = {"H(foo)", "H(fov)", "H(fvo)", "H(fvv)"};
    for (int k = 0; k < 4; ++k) {
      P.h_df[k] = m.add(nm[k], m[fb[k]].cls, Role::Tangent, true);
      tan[fb[k]] = P.h_df[k];
    }
    OpList hops = jvp(m, comb, tan, {P.g_gt1, P.g_gt2p}, "H");
    P.h_out1 = tan.at(P.g_gt1);
    P.h_out2p = tan.at(P.g_gt2p);
    P.hvp = prune(m, hops, {P.h_out1, P.h_out2p});

    std::map<int, int> tt;
    P.f_dt1 = m.add("F(t1)", "ov", Role::Tangent, true);
    P.f_dt2p = m.add("F(t2p)", "OV", Role::Tangent, true);
    tt[P.t1] = P.f_dt1;
    tt[P.t2p] = P.f_dt2p;
    OpList fops = jvp(m, comb, tt, {P.g_gt1, P.g_gt2p}, "F");
    P.f_out1 = tt.at(P.g_gt1);
    P.f_out2p = tt.at(P.g_gt2p);
    P.hvpt = prune(m, fops, {P.f_out1, P.f_out2p});
  }
  mark_persistent(m, {&P.residual, &P.ring_setup, &P.right, &P.right_f, &P.left, &P.left_f, &P.eta0, &P.xi, &P.gradL,
                      &P.hvp, &P.hvpt, &P.fnspp});
}

}  // namespace lrcc
