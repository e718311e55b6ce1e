// Executor of contraction programs (see runtime.h).
#include "runtime.h"

#include <algorithm>
#include <cstring>
#include <tuple>

#include "devmem.h"
#include "kernels.h"

namespace lrcc {

template <typename T>
struct vec2_of;
template <>
struct vec2_of<double> {
  using type = double2;
};
template <>
struct vec2_of<float> {
  using type = float2;
};

// c = alpha * d (+ c if acc); d is an FP64 complex scalar in device memory.
template <typename T>
__global__ void scalar_set_kernel(const double2* d, typename vec2_of<T>::type* c, double are, double aim, int acc) {
  double re = are * d->x - aim * d->y, im = are * d->y + aim * d->x;
  if (acc) {
    re += (double)c->x;
    im += (double)c->y;
  }
  *c = {(T)re, (T)im};
}

template <typename T>
Executor<T>::Executor(const Module& m, Dims d, hipStream_t st) : m_(m), d_(d), st_(st) {
  size_t n = m.tensors.size();
  buf_.assign(n, nullptr);
  cap_.assign(n, 0);
  bound_.assign(n, 0);
  pooled_.assign(n, 0);
  // 0-2 permutations, 3 virtual constants, 4 split-K partials, 5-6 cached permutations,
  // 7-8 DF-direct ladder: (ae|bf) block and rebuilt rows of W
  scr_.assign(9, nullptr);
  scr_cap_.assign(9, 0);
  dot_out_ = dev_alloc(64);
  dot_work_ = dev_alloc(1024 * 16);
}

template <typename T>
Executor<T>::~Executor() {
  try {
    clear_graphs();
  } catch (...) {
  }
  for (size_t k = 0; k < buf_.size(); ++k)
    if (buf_[k] && !bound_[k] && !pooled_[k]) dev_free(buf_[k]);
  for (void* p : scr_)
    if (p) dev_free(p);
  for (void* p : pool_)
    if (p) dev_free(p);
  dev_free(dot_out_);
  dev_free(dot_work_);
  if (gst_) (void)hipStreamDestroy(gst_);
  if (fork_) (void)hipEventDestroy(fork_);
  if (join_) (void)hipEventDestroy(join_);
  for (auto& p : pending_) {
    event_pool_.push_back(p.a);
    event_pool_.push_back(p.b);
  }
  for (auto e : event_pool_) (void)hipEventDestroy(e);
}

template <typename T>
int64_t Executor<T>::elems(int id, int nb) const {
  const TensorDecl& t = m_[id];
  int64_t n = t.batched ? nb : 1;
  for (char c : t.cls) n *= d_.of(c);
  return n;
}

template <typename T>
void* Executor<T>::ptr(int id) {
  if (bound_[id] || pooled_[id]) return buf_[id];
  LRCC_REQUIRE(!is_virtual(id), LRCC_E_INTERNAL, "constant " + m_[id].name + " has no storage of its own");
  int64_t need = elems(id, max_nb_);
  if (cap_[id] < need) {
    on_realloc();
    if (buf_[id]) {
      HIP_CHECK(hipStreamSynchronize(st_));
      dev_free(buf_[id]);
      buf_[id] = nullptr;
    }
    buf_[id] = dev_alloc(std::max<int64_t>(need, 1) * sizeof(T) * 2);
    cap_[id] = need;
  }
  return buf_[id];
}

template <typename T>
void Executor<T>::bind(int id, void* p) {
  LRCC_REQUIRE(!pooled_[id], LRCC_E_INTERNAL, "cannot bind a pooled transient");
  if (buf_[id] && !bound_[id]) {
    on_realloc();
    HIP_CHECK(hipStreamSynchronize(st_));
    dev_free(buf_[id]);
  }
  buf_[id] = p;
  cap_[id] = 0;
  bound_[id] = 1;
}

template <typename T>
void Executor<T>::unbind(int id) {
  if (bound_[id]) {
    buf_[id] = nullptr;
    bound_[id] = 0;
    cap_[id] = 0;
  }
}

template <typename T>
void Executor<T>::set_max_batch(int nb) {
  if (nb <= max_nb_) return;
  max_nb_ = nb;  // batched buffers grow on next use
}

template <typename T>
void Executor<T>::release_batched() {
  on_realloc();
  HIP_CHECK(hipStreamSynchronize(st_));
  for (size_t k = 0; k < buf_.size(); ++k)
    if (m_[k].batched && buf_[k] && !bound_[k] && !pooled_[k]) {
      dev_free(buf_[k]);
      buf_[k] = nullptr;
      cap_[k] = 0;
    }
  for (size_t s = 0; s < pool_.size(); ++s)
    if (pool_[s]) {
      dev_free(pool_[s]);
      pool_[s] = nullptr;
      pool_cap_[s] = 0;
    }
  for (size_t k = 0; k < buf_.size(); ++k)
    if (pooled_[k]) {
      buf_[k] = nullptr;
      cap_[k] = 0;
      pooled_[k] = 0;
    }
  for (size_t s = 0; s < scr_.size(); ++s)
    if (scr_[s]) {
      dev_free(scr_[s]);
      scr_[s] = nullptr;
      scr_cap_[s] = 0;
    }
  plans_.clear();
}

template <typename T>
void Executor<T>::release_results(const OpList& ops) {
  bool any = false;
  for (const Op& op : ops) {
    const int t = op.out;
    if (m_[t].batched || bound_[t] || pooled_[t] || !buf_[t]) continue;
    if (!any) {
      on_realloc();
      HIP_CHECK(hipStreamSynchronize(st_));
      any = true;
    }
    dev_free(buf_[t]);
    buf_[t] = nullptr;
    cap_[t] = 0;
  }
}

template <typename T>
void Executor<T>::release(int id) {
  if (id < 0 || m_[id].batched || bound_[id] || pooled_[id] || !buf_[id]) return;
  on_realloc();
  HIP_CHECK(hipStreamSynchronize(st_));
  dev_free(buf_[id]);
  buf_[id] = nullptr;
  cap_[id] = 0;
}

template <typename T>
size_t Executor<T>::bytes_allocated() const {
  size_t s = 0;
  for (size_t k = 0; k < buf_.size(); ++k)
    if (!bound_[k] && !pooled_[k]) s += cap_[k] * sizeof(T) * 2;
  for (size_t c : scr_cap_) s += c;
  for (int64_t c : pool_cap_) s += c * sizeof(T) * 2;
  return s;
}

template <typename T>
void* Executor<T>::scratch(int slot, size_t bytes) {
  if (scr_cap_[slot] < bytes) {
    on_realloc();
    if (scr_[slot]) {
      HIP_CHECK(hipStreamSynchronize(st_));
      dev_free(scr_[slot]);
    }
    size_t b = std::max(bytes, scr_cap_[slot] + scr_cap_[slot] / 4);
    scr_[slot] = dev_alloc(b);
    scr_cap_[slot] = b;
  }
  return scr_[slot];
}

// current batch of the op being executed (dims of '#')
static thread_local int64_t g_nb = 1;

template <typename T>
int64_t Executor<T>::capacity(int id) {
  if (bound_[id]) return elems(id, (int)g_nb);
  ptr(id);
  return cap_[id];
}

template <typename T>
int64_t Executor<T>::dim(char l) const {
  if (l == '#') return max_nb_;  // replaced by the actual batch in run()
  return d_.of(letter_class(l));
}

template <typename T>
std::string Executor<T>::letters(int id, const std::string& idx) const {
  return (m_[id].batched ? std::string("#") : std::string()) + idx;
}

template <typename T>
hipEvent_t Executor<T>::get_event() {
  if (event_pool_.empty()) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    return e;
  }
  hipEvent_t e = event_pool_.back();
  event_pool_.pop_back();
  return e;
}

template <typename T>
void Executor<T>::collect_times(KernelTimes& kt) {
  if (pending_.empty()) return;
  HIP_CHECK(hipStreamSynchronize(st_));
  for (auto& p : pending_) {
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, p.a, p.b));
    for (int c : {p.cls, 2}) {
      if (c < 0) continue;
      kt.ms[c] += ms;
      kt.launches[c] += 1;
      kt.flops[c] += p.flops;
    }
    event_pool_.push_back(p.a);
    event_pool_.push_back(p.b);
  }
  pending_.clear();
}

template <typename T>
void Executor<T>::permute_into(const void* src, int64_t src_cap, const std::string& sl, void* dst, int64_t dst_cap,
                               const std::string& dl, double are, double aim, double bre, double bim) {
  LRCC_REQUIRE((int)dl.size() <= kMaxRank, LRCC_E_INTERNAL, "rank too large");
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  // source strides (row-major)
  std::vector<int64_t> sstr(sl.size());
  int64_t s = 1;
  for (int k = (int)sl.size() - 1; k >= 0; --k) {
    sstr[k] = s;
    s *= dimof(sl[k]);
  }
  // merge runs of output letters that are also consecutive in the source
  PermDesc d{};
  d.rank = 0;
  for (size_t k = 0; k < dl.size(); ++k) {
    size_t p = sl.find(dl[k]);
    LRCC_REQUIRE(p != std::string::npos, LRCC_E_INTERNAL, "permute letter missing");
    int64_t n = dimof(dl[k]);
    if (d.rank > 0 && k > 0) {
      size_t pp = sl.find(dl[k - 1]);
      if (pp + 1 == p) {  // previous output letter directly precedes in source
        d.dims[d.rank - 1] *= n;
        d.istride[d.rank - 1] = sstr[p];
        continue;
      }
    }
    d.dims[d.rank] = n;
    d.istride[d.rank] = sstr[p];
    ++d.rank;
  }
  if (d.rank == 0) {
    d.rank = 1;
    d.dims[0] = 1;
    d.istride[0] = 1;
  }
  int64_t total = 1, maxin = 0;
  for (int k = 0; k < d.rank; ++k) {
    total *= d.dims[k];
    maxin += (d.dims[k] - 1) * d.istride[k];
  }
  LRCC_REQUIRE(total <= dst_cap && maxin < src_cap, LRCC_E_INTERNAL,
               "permute " + sl + "->" + dl + " exceeds its buffers");
  launch_permute<T>(src, dst, d, are, aim, bre, bim, st_);
}

template <typename T>
void Executor<T>::gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double are, double aim, const void* A,
                       int64_t lda, int64_t capA, const void* B, int64_t ldb, int64_t capB, double bre, void* C,
                       int64_t ldc, int64_t capC, bool ladder, const OutMap* om, bool conjb) {
  if (M > 0 && N > 0 && K > 0) {
    int64_t spanA = ta ? (K - 1) * lda + M : (M - 1) * lda + K;
    int64_t spanB = tb ? (N - 1) * ldb + K : (K - 1) * ldb + N;
    // the last element the output map reaches (maps are monotone in each digit)
    int64_t lastC = om ? om->row(M - 1) + om->col(N - 1) : (M - 1) * ldc + N - 1;
    LRCC_REQUIRE(spanA <= capA && spanB <= capB && lastC < capC && lda >= (ta ? M : K) && ldb >= (tb ? K : N) &&
                     (om || ldc >= N),
                 LRCC_E_INTERNAL, "gemm operands exceed their buffers");
  }
  const size_t wsb = gemm_workspace_bytes<T>(M, N, K);
  void* ws = wsb ? scratch(4, wsb) : nullptr;
  GemmArgs g{ta, tb, M, N, K, are, aim, A, lda, B, ldb, bre, C, ldc, ladder, ws, wsb, OutMap(), om != nullptr, conjb};
  if (om) g.om = *om;
  if (capturing_) {
    if (timing_ && ladder) {  // leave the graph: the ladder is timed between segments
      end_segment();
      rec_->timed.push_back(g);
      launch_timed(g);
      HIP_CHECK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    } else {
      launch_gemm<T>(ta, tb, M, N, K, are, aim, A, lda, B, ldb, bre, 0.0, C, ldc, st_, ladder ? 1 : 0, ws, wsb, om,
                     conjb);
    }
    return;
  }
  launch_timed(g);
}

template <typename T>
void Executor<T>::launch_timed(const GemmArgs& g) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timing_) {
    e0 = get_event();
    HIP_CHECK(hipEventRecord(e0, st_));
  }
  launch_gemm<T>(g.ta, g.tb, g.M, g.N, g.K, g.are, g.aim, g.A, g.lda, g.B, g.ldb, g.bre, 0.0, g.C, g.ldc, st_,
                 g.ladder ? 1 : 0, g.ws, g.wsb, g.mapped ? &g.om : nullptr, g.conjb);
  if (timing_) {
    e1 = get_event();
    HIP_CHECK(hipEventRecord(e1, st_));
    double fl = (sizeof(T) == 8 ? 8.0 : 6.0) * (double)g.M * (double)g.N * (double)g.K;
    pending_.push_back({e0, e1, g.ladder ? (sizeof(T) == 4 ? 0 : 1) : -1, fl});
  }
}

// Digits of the product's M and N index strings in the layout of the output
// string cl (row-major): each letter's stride in cl, letters that are also
// adjacent in cl merged.  False if either side needs more than kMapRank.
template <typename T>
bool Executor<T>::output_map(const std::string& Mc, const std::string& Nc, const std::string& cl, OutMap& om) const {
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  std::vector<int64_t> str(cl.size());
  int64_t s = 1;
  for (int k = (int)cl.size() - 1; k >= 0; --k) {
    str[k] = s;
    s *= dimof(cl[k]);
  }
  auto side = [&](const std::string& letters, int& nd, int64_t* dims, int64_t* strides) {
    nd = 0;
    for (char l : letters) {
      const int64_t d = dimof(l), st = str[cl.find(l)];
      if (nd > 0 && strides[nd - 1] == st * d) {  // continues the previous digit in cl
        dims[nd - 1] *= d;
        strides[nd - 1] = st;
        continue;
      }
      if (nd == kMapRank) return false;
      dims[nd] = d;
      strides[nd] = st;
      ++nd;
    }
    if (nd == 0) {
      dims[0] = 1;
      strides[0] = 0;
      nd = 1;
    }
    return true;
  };
  return side(Mc, om.nm, om.mdim, om.mstr) && side(Nc, om.nn, om.ndim, om.nstr);
}

// Permuted copies of batched operands live in two scratch slots for the
// rest of a run, keyed by (tensor, permutation of its index positions).  A
// tensor is final once it is first read in a program, so a copy made from it
// stays valid until the run ends; graph replays repeat the permutation that
// was recorded for the first use.
template <typename T>
int Executor<T>::cached_permute(int id, const std::string& src, const std::string& dst, const void* p, int64_t cap) {
  std::vector<int> perm;
  for (char ch : dst) perm.push_back((int)src.find(ch));
  for (int s = 0; s < 2; ++s)
    if (pcache_[s].tensor == id && pcache_[s].perm == perm && pcache_[s].nb == g_nb) return kPermSlot + s;
  const int s = pnext_;
  pnext_ ^= 1;
  int64_t n = 1;
  for (char ch : src) n *= ch == '#' ? g_nb : dim(ch);
  void* t = scratch(kPermSlot + s, (size_t)n * sizeof(T) * 2);
  permute_into(p, cap, src, t, scratch_elems(kPermSlot + s), dst, 1, 0, 0, 0);
  pcache_[s] = PermEntry{id, perm, g_nb};
  return kPermSlot + s;
}

template <typename T>
void Executor<T>::contract(const Op& op, int nb) {
  (void)nb;
  if (dl_L_ && (op.a == ladder_const || op.b == ladder_const)) return ladder_direct(op);
  if (!tri_.empty() && (op.a == ladder_const || op.b == ladder_const)) return ladder_triangle(op);
  if (is_virtual(op.a) || is_virtual(op.b)) return contract_virtual(op);
  std::string a = letters(op.a, op.ai), b = letters(op.b, op.bi), c = letters(op.out, op.oi);
  const void* pa = ptr(op.a);
  const void* pb = ptr(op.b);
  void* pc = ptr(op.out);
  int64_t ca = capacity(op.a), cb = capacity(op.b), cc = capacity(op.out);
  auto size_of = [&](const std::string& sx) {
    int64_t p = 1;
    for (char ch : sx) p *= (ch == '#' ? g_nb : dim(ch));
    return p;
  };
  bool ladder = (op.a == ladder_const || op.b == ladder_const);
  int ida = op.a, idb = op.b;
  if (m_[op.b].batched && !m_[op.a].batched) {
    std::swap(ida, idb);
    std::swap(a, b);
    std::swap(pa, pb);
    std::swap(ca, cb);
  }
  LRCC_REQUIRE(size_of(a) <= ca && size_of(b) <= cb && size_of(c) <= cc, LRCC_E_INTERNAL,
               "contraction operand larger than its buffer");
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  auto size = [&](const std::string& s) {
    int64_t p = 1;
    for (char ch : s) p *= dimof(ch);
    return p;
  };
  std::string K, Mc, Nc;
  for (char ch : a)
    if (b.find(ch) != std::string::npos) {
      LRCC_REQUIRE(c.find(ch) == std::string::npos, LRCC_E_INTERNAL, "index in all three operands");
      K += ch;
    }
  for (char ch : c) {
    if (a.find(ch) != std::string::npos)
      Mc += ch;
    else if (b.find(ch) != std::string::npos)
      Nc += ch;
    else
      throw Error(LRCC_E_INTERNAL, "output index not in operands");
  }
  LRCC_REQUIRE(Mc.size() + K.size() == a.size() && Nc.size() + K.size() == b.size(), LRCC_E_INTERNAL,
               "contraction letters inconsistent");
  const bool acc = op.acc;

  if (Mc.empty() && Nc.empty()) {  // full contraction to a scalar
    LRCC_REQUIRE(!m_[op.out].batched, LRCC_E_INTERNAL, "batched scalar output");
    const void* pb2 = pb;
    if (b != a) {
      void* t = scratch(1, size(b) * sizeof(T) * 2);
      permute_into(pb, cb, b, t, scratch_elems(1), a, 1, 0, 0, 0);
      pb2 = t;
    }
    launch_batched_dot<T>(1, size(a), pa, 0, pb2, 0, false, dot_out_, dot_work_, st_);
    hipLaunchKernelGGL(scalar_set_kernel<T>, dim3(1), dim3(1), 0, st_, (const double2*)dot_out_,
                       (typename vec2_of<T>::type*)pc, op.are, op.aim, acc ? 1 : 0);
    HIP_CHECK(hipGetLastError());
    return;
  }

  bool direct = (c == Mc + Nc);
  if (!direct && c == Nc + Mc && a.find('#') == std::string::npos) {
    std::swap(ida, idb);
    std::swap(a, b);
    std::swap(pa, pb);
    std::swap(ca, cb);
    std::swap(Mc, Nc);
    direct = true;
  }
  const int64_t Ms = size(Mc), Ns = size(Nc), Ks = size(K);
  // choose the K order needing the fewest operand permutations
  std::string Ka, Kb;
  for (char ch : a)
    if (K.find(ch) != std::string::npos) Ka += ch;
  for (char ch : b)
    if (K.find(ch) != std::string::npos) Kb += ch;
  auto a_ok = [&](const std::string& Kx) { return a == Mc + Kx || a == Kx + Mc; };
  auto b_ok = [&](const std::string& Kx) { return b == Kx + Nc || b == Nc + Kx; };
  auto cost = [&](const std::string& Kx) {
    return (a_ok(Kx) ? 0 : size(a)) + (b_ok(Kx) ? 0 : size(b));
  };
  std::string Kx = cost(Ka) <= cost(Kb) ? Ka : Kb;

  bool ta, tb;
  int64_t lda, ldb;
  const void* A = pa;
  const void* B = pb;
  int64_t capA = ca, capB = cb;
  if (a == Mc + Kx) {
    ta = false;
    lda = Ks;
  } else if (a == Kx + Mc) {
    ta = true;
    lda = Ms;
  } else {
    const std::string tgt = Mc + Kx;
    if (m_[ida].batched) {  // batched operands: reuse a copy already permuted this run
      const int slot = cached_permute(ida, a, tgt, pa, ca);
      A = scr_[slot];
      capA = scratch_elems(slot);
    } else {
      void* t = scratch(0, size(a) * sizeof(T) * 2);
      permute_into(pa, ca, a, t, scratch_elems(0), tgt, 1, 0, 0, 0);
      A = t;
      capA = scratch_elems(0);
    }
    ta = false;
    lda = Ks;
  }
  // FP32 GEMMs run 3-7 % faster with B stored [N][K] (measured on the ring
  // and ladder shapes), so an unbatched B in [K][N] order is transposed
  // once when the product is large enough to repay the copy.  The vvvv
  // matrix needs no copy: it is Hermitian (W[x][y] = conj W[y][x], the DF
  // factors being Hermitian), so its [K][N] use is conj of its [N][K] use.
  const bool w_conj = sizeof(T) == 4 && idb == ladder_const && b == Kx + Nc && Ns == Ks;
  const bool b_to_nt = sizeof(T) == 4 && b == Kx + Nc && b.find('#') == std::string::npos && !ladder &&
                       Ms >= 16384 && Ns >= 64 && Ks >= 64;
  bool conjb = false;
  if (w_conj) {
    tb = true;
    ldb = Ks;
    conjb = true;
  } else if (b == Kx + Nc && !b_to_nt) {
    tb = false;
    ldb = Ns;
  } else if (b_to_nt) {
    void* t = scratch(1, size(b) * sizeof(T) * 2);
    permute_into(pb, cb, b, t, scratch_elems(1), Nc + Kx, 1, 0, 0, 0);
    B = t;
    capB = scratch_elems(1);
    tb = true;
    ldb = Ks;
  } else if (b == Nc + Kx) {
    tb = true;
    ldb = Ks;
  } else if (sizeof(T) == 4) {  // a permuted copy is made anyway: make it [N][K]
    void* t = scratch(1, size(b) * sizeof(T) * 2);
    permute_into(pb, cb, b, t, scratch_elems(1), Nc + Kx, 1, 0, 0, 0);
    B = t;
    capB = scratch_elems(1);
    tb = true;
    ldb = Ks;
  } else {
    void* t = scratch(1, size(b) * sizeof(T) * 2);
    permute_into(pb, cb, b, t, scratch_elems(1), Kx + Nc, 1, 0, 0, 0);
    B = t;
    capB = scratch_elems(1);
    tb = false;
    ldb = Ns;
  }
  OutMap om;
  if (direct) {
    gemm(ta, tb, Ms, Ns, Ks, op.are, op.aim, A, lda, capA, B, ldb, capB, acc ? 1.0 : 0.0, pc, Ns, cc, ladder,
         nullptr, conjb);
  } else if (output_map(Mc, Nc, c, om)) {  // the epilogue writes straight into c's index order
    gemm(ta, tb, Ms, Ns, Ks, op.are, op.aim, A, lda, capA, B, ldb, capB, acc ? 1.0 : 0.0, pc, Ns, cc, ladder, &om,
         conjb);
  } else {
    void* t = scratch(2, (size_t)Ms * Ns * sizeof(T) * 2);
    gemm(ta, tb, Ms, Ns, Ks, op.are, op.aim, A, lda, capA, B, ldb, capB, 0.0, t, Ns, scratch_elems(2), ladder,
         nullptr, conjb);
    permute_into(t, scratch_elems(2), Mc + Nc, pc, cc, c, 1, 0, acc ? 1 : 0, 0);
  }
}

// Operands of a ladder contraction: the other operand X (contracted index
// last) and the output, both [M][V] row-major, and which index of W is
// contracted.
template <typename T>
typename Executor<T>::LadderOperands Executor<T>::ladder_operands(const Op& op) {
  const bool w_is_a = op.a == ladder_const;
  const int idx = w_is_a ? op.b : op.a;
  const std::string w = letters(ladder_const, w_is_a ? op.ai : op.bi), x = letters(idx, w_is_a ? op.bi : op.ai),
                    c = letters(op.out, op.oi);
  LRCC_REQUIRE(w.size() == 2 && x.size() >= 2, LRCC_E_INTERNAL, "ladder: unexpected operands");
  const char kl = x.back();
  LRCC_REQUIRE(w.find(kl) != std::string::npos && c.find(kl) == std::string::npos, LRCC_E_INTERNAL,
               "ladder: operand X must end with the contracted index");
  LadderOperands L;
  L.over_col = w[1] == kl;
  const std::string Mc = x.substr(0, x.size() - 1);
  LRCC_REQUIRE(c == Mc + (L.over_col ? w[0] : w[1]), LRCC_E_INTERNAL, "ladder: unsupported output order");
  L.M = 1;
  for (char ch : Mc) L.M *= ch == '#' ? g_nb : dim(ch);
  L.V = dim(kl);
  LRCC_REQUIRE(dim(L.over_col ? w[0] : w[1]) == L.V, LRCC_E_INTERNAL, "ladder: sizes");
  L.X = ptr(idx);
  L.C = ptr(op.out);
  L.capX = capacity(idx);
  L.capC = capacity(op.out);
  LRCC_REQUIRE(L.M * L.V <= L.capX && L.M * L.V <= L.capC, LRCC_E_INTERNAL, "ladder: operand larger than its buffer");
  return L;
}

// Ladder contraction without a resident W (DF-direct).  W's rows P(a,b)
// (b-major, so the rows of b in [b0, b1) are contiguous) are rebuilt in
// chunks: one GEMM over the auxiliary index gives (ae|bf) for b in the
// chunk and every a < b1, a pack kernel antisymmetrizes it into
// W[P(a,b)][P(e,f)] = (ae|bf) - (af|be), and the ladder GEMM consumes the
// rows: X[M][K=ef] W^T (contraction over W's column index: the chunk fills
// columns R0..R1 of the output) or X[M][K=ab] W (over W's row index: the
// chunk adds its K-range).  Extra work per ladder: naux v^4 / 2 complex MACs.
template <typename T>
void Executor<T>::ladder_direct(const Op& op) {
  const LadderOperands L = ladder_operands(op);
  const bool over_col = L.over_col;
  const int64_t M = L.M, v = dl_v_, nq = dl_naux_, V = v * (v - 1) / 2;
  LRCC_REQUIRE(L.V == V, LRCC_E_INTERNAL, "DF-direct ladder: sizes");
  const void* X = L.X;
  void* C = L.C;
  const int64_t capX = L.capX, capC = L.capC, capL = nq * v * v;
  const size_t es = 2 * sizeof(T);
  const size_t budget = kDirectChunkBytes;
  bool first = true;
  for (int64_t b0 = 1; b0 < v;) {
    auto fits = [&](int64_t bb) {
      return (size_t)((bb - b0) * v) * (size_t)(bb * v) * es <= budget &&
             (size_t)(bb * (bb - 1) / 2 - b0 * (b0 - 1) / 2) * (size_t)V * es <= budget;
    };
    int64_t b1 = b0 + 1;
    while (b1 < v && fits(b1 + 1)) ++b1;
    const int64_t R0 = b0 * (b0 - 1) / 2, nr = b1 * (b1 - 1) / 2 - R0;
    LRCC_REQUIRE(nr <= 65535, LRCC_E_INTERNAL, "DF-direct ladder: chunk too tall");
    void* Cb = scratch(7, (size_t)((b1 - b0) * v) * (size_t)(b1 * v) * es);
    void* Wc = scratch(8, (size_t)nr * (size_t)V * es);
    // (ae|bf): rows (b, f) for b in [b0, b1), columns (a, e) for a < b1
    gemm(true, false, (b1 - b0) * v, b1 * v, nq, 1.0, 0.0, (const char*)dl_L_ + b0 * v * es, v * v, capL - b0 * v,
         dl_L_, v * v, capL, 0.0, Cb, b1 * v, scratch_elems(7), false);
    launch_pack_wrows<T>(v, b0, b1, Cb, Wc, st_);
    if (over_col)
      gemm(false, true, M, nr, V, op.are, op.aim, X, V, capX, Wc, V, scratch_elems(8), op.acc ? 1.0 : 0.0,
           (char*)C + R0 * es, V, capC - R0, true);
    else
      gemm(false, false, M, V, nr, op.are, op.aim, (const char*)X + R0 * es, V, capX - R0, Wc, V, scratch_elems(8),
           (first && !op.acc) ? 0.0 : 1.0, C, V, capC, true);
    first = false;
    b0 = b1;
  }
}

// Ladder contraction with W held as its upper triangle in row blocks
// (block l: rows [r0, r1), columns [r0, V), S_l[i][c] = W[r0 + i][r0 + c]).
// W = W^H gives the entries left of each block: W[n][k] = conj(W[k][n]).
//   C = X W^T:  C[:, r0:r1]  = X[:, r0:] S_l^T              (every block first)
//               C[:, r1:]   += X[:, r0:r1] conj(S_l[:, r1-r0:])
//   C = X W:    C[:, r0:]   += X[:, r0:r1] S_l              (block 0 sets C)
//               C[:, r0:r1] += X[:, r1:] conj(S_l[:, r1-r0:])^T
template <typename T>
void Executor<T>::ladder_triangle(const Op& op) {
  const LadderOperands L = ladder_operands(op);
  const int64_t M = L.M, V = L.V;
  const size_t es = 2 * sizeof(T);
  const double beta0 = op.acc ? 1.0 : 0.0;
  LRCC_REQUIRE(!tri_.empty() && tri_.front().r0 == 0 && tri_.back().r1 == V, LRCC_E_INTERNAL,
               "triangle ladder: blocks do not cover W");
  if (L.over_col) {
    for (const TriBlock& b : tri_) {
      const int64_t ld = V - b.r0, nr = b.r1 - b.r0;
      gemm(false, true, M, nr, V - b.r0, op.are, op.aim, (const char*)L.X + b.r0 * es, V, L.capX - b.r0, b.p, ld,
           nr * ld, beta0, (char*)L.C + b.r0 * es, V, L.capC - b.r0, true);
    }
    for (const TriBlock& b : tri_) {
      const int64_t ld = V - b.r0, nr = b.r1 - b.r0;
      if (b.r1 == V) continue;
      gemm(false, false, M, V - b.r1, nr, op.are, op.aim, (const char*)L.X + b.r0 * es, V, L.capX - b.r0,
           (const char*)b.p + nr * es, ld, nr * ld - nr, 1.0, (char*)L.C + b.r1 * es, V, L.capC - b.r1, true,
           nullptr, true);
    }
    return;
  }
  bool first = true;
  for (const TriBlock& b : tri_) {
    const int64_t ld = V - b.r0, nr = b.r1 - b.r0;
    gemm(false, false, M, V - b.r0, nr, op.are, op.aim, (const char*)L.X + b.r0 * es, V, L.capX - b.r0, b.p, ld,
         nr * ld, first ? beta0 : 1.0, (char*)L.C + b.r0 * es, V, L.capC - b.r0, true);
    first = false;
    if (b.r1 == V) continue;
    gemm(false, true, M, nr, V - b.r1, op.are, op.aim, (const char*)L.X + b.r1 * es, V, L.capX - b.r1,
         (const char*)b.p + nr * es, ld, nr * ld - nr, 1.0, (char*)L.C + b.r0 * es, V, L.capC - b.r0, true, nullptr,
         true);
  }
}

template <typename T>
void Executor<T>::set_virtual(int id, const VirtualDef& d) {
  if (vdef_.size() < buf_.size()) vdef_.resize(buf_.size());
  LRCC_REQUIRE(id >= 0 && id < (int)buf_.size() && m_[id].role == Role::Const && !m_[id].batched, LRCC_E_INTERNAL,
               "only unbatched constants can be virtual");
  LRCC_REQUIRE(d.src >= 0 && d.src != id && !is_virtual(d.src) && d.vl.size() == m_[id].cls.size() &&
                   d.sl.size() == d.vl.size() && (d.chunk < (int)d.vl.size()),
               LRCC_E_INTERNAL, "bad virtual constant " + m_[id].name);
  if (buf_[id] && !bound_[id]) {
    on_realloc();
    HIP_CHECK(hipStreamSynchronize(st_));
    dev_free(buf_[id]);
  }
  buf_[id] = nullptr;
  cap_[id] = 0;
  bound_[id] = 0;
  vdef_[id] = d;
  on_realloc();
}

template <typename T>
void Executor<T>::materialize(int id, const std::string& vlet, const std::string& tgt, char g, int64_t g0,
                              int64_t gl, void* dst, int64_t dst_cap, double are, double aim, bool acc) {
  const VirtualDef& vd = vdef_[id];
  LRCC_REQUIRE(vlet.size() == vd.vl.size() && tgt.size() == vlet.size(), LRCC_E_INTERNAL, "materialize: letters");
  std::string sl;  // the source's indices in op letters
  for (char ch : vd.sl) {
    const size_t p = vd.vl.find(ch);
    LRCC_REQUIRE(p != std::string::npos, LRCC_E_INTERNAL, "materialize: source letter");
    sl += vlet[p];
  }
  // stored dims of the source: one per plain index, one for the packed pair
  const std::string& scls = m_[vd.src].cls;
  const int ns = (int)scls.size();
  std::vector<int64_t> sdim(ns), sstr(ns);
  for (int k = 0; k < ns; ++k) sdim[k] = d_.of(scls[k]);
  int64_t s = 1;
  for (int k = ns - 1; k >= 0; --k) sstr[k] = s, s *= sdim[k];
  std::vector<int> stored_of(sl.size(), -1);
  int k = 0;
  for (int j = 0; j < (int)sl.size(); ++k) {
    LRCC_REQUIRE(k < ns, LRCC_E_INTERNAL, "materialize: source rank");
    if (j == vd.pair_at) {
      const int64_t n = dim(sl[j]);
      LRCC_REQUIRE(j + 1 < (int)sl.size() && dim(sl[j + 1]) == n && sdim[k] == n * (n - 1) / 2, LRCC_E_INTERNAL,
                   "materialize: packed pair");
      stored_of[j] = stored_of[j + 1] = k;
      j += 2;
    } else {
      LRCC_REQUIRE(sdim[k] == dim(sl[j]), LRCC_E_INTERNAL, "materialize: source dims");
      stored_of[j] = k;
      j += 1;
    }
  }
  LRCC_REQUIRE(k == ns, LRCC_E_INTERNAL, "materialize: source rank");
  MatDesc md{};
  md.rank = (int)tgt.size();
  LRCC_REQUIRE(md.rank <= kMaxRank, LRCC_E_INTERNAL, "materialize: rank");
  int64_t total = 1;
  for (int q = 0; q < md.rank; ++q) {
    const char ch = tgt[q];
    const size_t j = sl.find(ch);
    LRCC_REQUIRE(j != std::string::npos, LRCC_E_INTERNAL, "materialize: target letter");
    const bool restricted = g != 0 && ch == g;
    LRCC_REQUIRE(!restricted || (g0 >= 0 && gl >= 1 && g0 + gl <= dim(ch)), LRCC_E_INTERNAL, "materialize: range");
    md.dims[q] = restricted ? gl : dim(ch);
    md.shift[q] = restricted ? g0 : 0;
    md.pairpos[q] = (int)j == vd.pair_at ? 0 : ((int)j == vd.pair_at + 1 && vd.pair_at >= 0 ? 1 : -1);
    md.str[q] = md.pairpos[q] < 0 ? sstr[stored_of[j]] : 0;
    total *= md.dims[q];
  }
  md.pstride = vd.pair_at >= 0 ? sstr[stored_of[vd.pair_at]] : 0;
  md.conj = vd.conj ? 1 : 0;
  LRCC_REQUIRE(total <= dst_cap && s <= capacity(vd.src), LRCC_E_INTERNAL, "materialize exceeds its buffers");
  const double re = are * vd.sre - aim * vd.sim, im = are * vd.sim + aim * vd.sre;
  launch_materialize<T>(ptr(vd.src), dst, md, re, im, acc, st_);
}

// A contraction with a virtual constant G (made the B operand): G is
// materialized in [N][K] order into scratch slot 3, in chunks over its
// chunk index g when g is contracted (the chunks split K; the other
// operand's K order puts g first, so each chunk is a contiguous range of
// its columns, and the partial products accumulate) or an output index (the
// chunks write disjoint parts of the output through a mapped epilogue).
template <typename T>
void Executor<T>::contract_virtual(const Op& op) {
  LRCC_REQUIRE(!(is_virtual(op.a) && is_virtual(op.b)), LRCC_E_INTERNAL, "two virtual operands");
  const bool va = is_virtual(op.a);
  const int idg = va ? op.a : op.b, idx = va ? op.b : op.a;
  const std::string b = letters(idg, va ? op.ai : op.bi), a = letters(idx, va ? op.bi : op.ai),
                    c = letters(op.out, op.oi);
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  auto size = [&](const std::string& x) {
    int64_t p = 1;
    for (char ch : x) p *= dimof(ch);
    return p;
  };
  std::string K, Mc, Nc;
  for (char ch : a)
    if (b.find(ch) != std::string::npos) K += ch;
  for (char ch : c) {
    if (a.find(ch) != std::string::npos)
      Mc += ch;
    else if (b.find(ch) != std::string::npos)
      Nc += ch;
    else
      throw Error(LRCC_E_INTERNAL, "output index not in operands");
  }
  LRCC_REQUIRE(Mc.size() + K.size() == a.size() && Nc.size() + K.size() == b.size() && !K.empty() &&
                   !(Mc.empty() && Nc.empty()),
               LRCC_E_INTERNAL, "virtual contraction: unsupported letters");
  const VirtualDef& vd = vdef_[idg];
  const char g = vd.chunk >= 0 ? b[vd.chunk] : 0;
  const bool gK = g && K.find(g) != std::string::npos, gN = g && Nc.find(g) != std::string::npos;
  std::string Kx = K;  // in a's order, g first when contracted
  if (gK && Kx[0] != g) Kx = std::string(1, g) + Kx.erase(Kx.find(g), 1);
  const int64_t Ms = size(Mc), Ns = size(Nc), Ks = size(Kx);
  const size_t es = 2 * sizeof(T);
  // the other operand as [M][K] or [K][M]
  const void* A = ptr(idx);
  int64_t capA = capacity(idx), lda;
  bool ta;
  if (a == Mc + Kx) {
    ta = false;
    lda = Ks;
  } else if (a == Kx + Mc) {
    ta = true;
    lda = Ms;
  } else {
    if (m_[idx].batched) {
      const int slot = cached_permute(idx, a, Mc + Kx, A, capA);
      A = scr_[slot];
      capA = scratch_elems(slot);
    } else {
      void* t = scratch(0, size(a) * es);
      permute_into(A, capA, a, t, scratch_elems(0), Mc + Kx, 1, 0, 0, 0);
      A = t;
      capA = scratch_elems(0);
    }
    ta = false;
    lda = Ks;
  }
  const bool chunked = gK || gN;
  const int64_t gdim = chunked ? dimof(g) : 1;
  int64_t gc = gdim;
  if (chunked) {
    const double per_g = (double)(size(b) / gdim) * (double)es;
    gc = std::max<int64_t>(1, std::min<int64_t>(gdim, (int64_t)((double)vchunk_bytes_ / per_g)));
  }
  void* pc = ptr(op.out);
  const int64_t cc = capacity(op.out);
  OutMap om;
  bool direct = false, mapped = false;
  int64_t gstride = 0;  // stride of g in the output (gN)
  if (gN) {
    // the M digits as output_map merges them; one N digit per letter, g's restricted per chunk
    LRCC_REQUIRE(output_map(Mc, Nc, c, om) && (int)Nc.size() <= kMapRank, LRCC_E_INTERNAL,
                 "virtual contraction: output map");
    std::vector<int64_t> str(c.size());
    int64_t s = 1;
    for (int k = (int)c.size() - 1; k >= 0; --k) str[k] = s, s *= dimof(c[k]);
    om.nn = (int)Nc.size();
    for (int k = 0; k < om.nn; ++k) {
      om.ndim[k] = Nc[k] == g ? gc : dimof(Nc[k]);
      om.nstr[k] = str[c.find(Nc[k])];
    }
    gstride = str[c.find(g)];
    mapped = true;
  } else if (c == Mc + Nc) {
    direct = true;
  } else {
    mapped = output_map(Mc, Nc, c, om);
  }
  void* prod = nullptr;
  int64_t prod_cap = 0;
  if (!direct && !mapped) {
    prod = scratch(2, (size_t)Ms * Ns * es);
    prod_cap = scratch_elems(2);
  }
  const int64_t Krest = gK ? Ks / gdim : Ks, Nrest = gN ? Ns / gdim : Ns;
  for (int64_t g0 = 0; g0 < gdim; g0 += gc) {
    const int64_t gl = std::min(gc, gdim - g0);
    const int64_t Kc = gK ? gl * Krest : Ks, Nch = gN ? gl * Nrest : Ns;
    void* Bm = scratch(3, (size_t)Nch * Kc * es);
    materialize(idg, va ? op.ai : op.bi, Nc + Kx, chunked ? g : 0, g0, chunked ? gl : 0, Bm, scratch_elems(3), 1.0, 0.0,
                false);
    const void* Ac = A;
    int64_t capAc = capA;
    if (gK) {
      const int64_t off = ta ? g0 * Krest * lda : g0 * Krest;
      Ac = (const char*)A + off * es;
      capAc = capA - off;
    }
    const double beta = gK ? (g0 == 0 ? (op.acc ? 1.0 : 0.0) : 1.0) : (op.acc ? 1.0 : 0.0);
    if (direct) {
      gemm(ta, true, Ms, Ns, Kc, op.are, op.aim, Ac, lda, capAc, Bm, Kc, scratch_elems(3), beta, pc, Ns, cc, false);
    } else if (mapped) {
      OutMap oc = om;
      int64_t off = 0;
      if (gN) {
        for (int k = 0; k < oc.nn; ++k)
          if (Nc[k] == g) oc.ndim[k] = gl;
        off = g0 * gstride;
      }
      gemm(ta, true, Ms, Nch, Kc, op.are, op.aim, Ac, lda, capAc, Bm, Kc, scratch_elems(3), beta, (char*)pc + off * es,
           Nch, cc - off, false, &oc);
    } else {
      gemm(ta, true, Ms, Ns, Kc, op.are, op.aim, Ac, lda, capAc, Bm, Kc, scratch_elems(3), g0 == 0 ? 0.0 : 1.0, prod,
           Ns, prod_cap, false);
    }
  }
  if (prod) permute_into(prod, prod_cap, Mc + Nc, pc, cc, c, 1, 0, op.acc ? 1 : 0, 0);
}

template <typename T>
void Executor<T>::add(const Op& op, int nb) {
  (void)nb;
  if (is_virtual(op.a)) {  // a permuted copy of a virtual constant: written straight into the output
    LRCC_REQUIRE(!m_[op.out].batched, LRCC_E_INTERNAL, "add: batch mismatch");
    materialize(op.a, op.ai, op.oi, 0, 0, 0, ptr(op.out), capacity(op.out), op.are, op.aim, op.acc);
    return;
  }
  std::string a = letters(op.a, op.ai), c = letters(op.out, op.oi);
  LRCC_REQUIRE(m_[op.a].batched == m_[op.out].batched, LRCC_E_INTERNAL, "add: batch mismatch");
  permute_into(ptr(op.a), capacity(op.a), a, ptr(op.out), capacity(op.out), c, op.are, op.aim, op.acc ? 1 : 0, 0);
}

// Permute-accumulates into one tensor whose sources are in its index order
// or have its last two indices exchanged (the dressed doubles t2 + t1 t1 -
// (t1 t1) with a <-> b, their adjoints, and the like) run as one summed
// permute: every source is read once and the output written once, not once
// per op.  ops[idx[0]] may be plain or accumulating, the rest must
// accumulate.  A source that is the tensor virt_id_ is evaluated in place
// from its outer products.  Returns false, launching nothing, when the ops
// do not fit; with launch false it only checks.
template <typename T>
bool Executor<T>::fuse_adds(const OpList& ops, const std::vector<size_t>& idx, bool launch) {
  if (idx.size() < 2) return false;
  const Op& o0 = ops[idx[0]];
  const std::string c0 = letters(o0.out, o0.oi);
  const int L = (int)c0.size();
  if (L < 2 || c0[L - 1] == '#' || c0[L - 2] == '#') return false;
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  const int64_t np = dimof(c0[L - 2]), nq = dimof(c0[L - 1]);
  int64_t total = 1;
  for (char l : c0) total *= dimof(l);
  std::vector<int> sw(idx.size());
  for (size_t g = 0; g < idx.size(); ++g) {
    const Op& o = ops[idx[g]];
    if (o.kind != OpKind::Add || o.out != o0.out || o.a == o.out || (g > 0 && !o.acc)) return false;
    if (is_virtual(o.a)) return false;
    if (m_[o.a].batched != m_[o.out].batched) return false;
    const std::string c = letters(o.out, o.oi), a = letters(o.a, o.ai);
    if ((int)c.size() != L || (int)a.size() != L) return false;
    // source position of each output position
    bool ident = true, swap = true;
    for (int k = 0; k < L; ++k) {
      const size_t p = a.find(c[k]);
      if (p == std::string::npos) return false;
      ident = ident && (int)p == k;
      swap = swap && (int)p == (k < L - 2 ? k : (k == L - 2 ? L - 1 : L - 2));
    }
    if (!ident && !swap) return false;
    sw[g] = ident ? 0 : 1;
    if (o.a == virt_id_) {
      if (np != nq || total != (m_[o.a].batched ? g_nb : 1) * virt_.ni * virt_.nj * np * nq) return false;
    } else if (total > capacity(o.a)) {
      return false;
    }
  }
  if (!launch) return true;
  LRCC_REQUIRE(total <= capacity(o0.out), LRCC_E_INTERNAL, "summed permute exceeds its output buffer");
  for (size_t g0 = 0; g0 < idx.size(); g0 += 4) {  // at most four sources per launch
    SumSources s = virt_;
    s.n = 0;
    for (size_t g = g0; g < idx.size() && g < g0 + 4; ++g) {
      const Op& o = ops[idx[g]];
      const bool v = o.a == virt_id_;
      s.p[s.n] = v ? nullptr : ptr(o.a);
      s.virt[s.n] = v ? 1 : 0;
      s.swap[s.n] = sw[g];
      s.re[s.n] = o.are;
      s.im[s.n] = o.aim;
      ++s.n;
    }
    launch_sum_swap<T>(s, ptr(o0.out), g0 == 0 ? o0.acc : true, total / (np * nq), np, nq, st_);
  }
  return true;
}

// Groups of the Add ops ops[i..w) that run_adds executes together.  When no
// op of the run reads a tensor that another op of the run writes, and no
// tensor is first written after ops[i] within the run (so no buffer of the
// liveness pool changes hands inside it), the ops are grouped by output
// tensor, each group keeping its order; otherwise consecutive ops into one
// tensor are grouped.
template <typename T>
std::vector<std::vector<size_t>> Executor<T>::add_groups(const OpList& ops, size_t i, size_t w) const {
  bool regroup = w - i >= 2;
  for (size_t k = i; k < w && regroup; ++k) {
    for (size_t q = i; q < w && regroup; ++q)
      if (q != k && ops[k].a == ops[q].out) regroup = false;
    if (k > i) {
      bool written_before = false;
      for (size_t q = 0; q < k && !written_before; ++q) written_before = ops[q].out == ops[k].out;
      if (!written_before) regroup = false;
    }
  }
  std::vector<std::vector<size_t>> groups;
  for (size_t k = i; k < w; ++k) {
    if (regroup) {
      size_t g = 0;
      while (g < groups.size() && ops[groups[g][0]].out != ops[k].out) ++g;
      if (g == groups.size()) groups.emplace_back();
      groups[g].push_back(k);
    } else {
      if (groups.empty() || ops[groups.back()[0]].out != ops[k].out) groups.emplace_back();
      groups.back().push_back(k);
    }
  }
  return groups;
}

// Runs the Add ops from ops[i] to the next op of another kind, in the groups
// of add_groups; every group that fits runs as one summed permute.  Returns
// the index after the run.
template <typename T>
size_t Executor<T>::run_adds(const OpList& ops, size_t i, int nb) {
  size_t w = i;
  while (w < ops.size() && ops[w].kind == OpKind::Add) ++w;
  for (const auto& g : add_groups(ops, i, w))
    if (!fuse_adds(ops, g)) {
      for (size_t k : g) {
        LRCC_REQUIRE(ops[k].a != virt_id_, LRCC_E_INTERNAL, "in-place tensor read outside a summed permute");
        add(ops[k], nb);
      }
    }
  return w;
}

// An outer product into a 4-index tensor TT[(b)][i][j][p][q] = alpha
// U[(b)][i][p] V[(b)][j][q] (no contracted index): appends it to s.
template <typename T>
bool Executor<T>::outer_product(const Op& o, SumSources& s) {
  if (o.kind != OpKind::Contract || o.a < 0 || o.b < 0 || s.nouter >= 2) return false;
  if (o.a == ladder_const || o.b == ladder_const) return false;
  const std::string c = letters(o.out, o.oi);
  const int L = (int)c.size();
  if (!(L == 4 && !m_[o.out].batched) && !(L == 5 && m_[o.out].batched)) return false;
  const std::string ia = {c[L - 4], c[L - 2]}, jb = {c[L - 3], c[L - 1]};
  int U, V;
  if (o.ai == ia && o.bi == jb) {
    U = o.a, V = o.b;
  } else if (o.bi == ia && o.ai == jb) {
    U = o.b, V = o.a;
  } else {
    return false;
  }
  if (!m_[o.out].batched && (m_[U].batched || m_[V].batched)) return false;
  if (m_[o.out].batched && !m_[U].batched && !m_[V].batched) return false;
  const int64_t ni = dim(c[L - 4]), nj = dim(c[L - 3]), np = dim(c[L - 2]), nq = dim(c[L - 1]);
  if (s.nouter > 0 && (s.ni != ni || s.nj != nj)) return false;
  const int64_t nbU = m_[U].batched ? g_nb : 1, nbV = m_[V].batched ? g_nb : 1;
  if (capacity(U) < nbU * ni * np || capacity(V) < nbV * nj * nq) return false;
  const int c_ = s.nouter++;
  s.U[c_] = ptr(U);
  s.V[c_] = ptr(V);
  s.ustride[c_] = m_[U].batched ? ni * np : 0;
  s.vstride[c_] = m_[V].batched ? nj * nq : 0;
  s.ore[c_] = o.are;
  s.oim[c_] = o.aim;
  s.ni = ni;
  s.nj = nj;
  return true;
}

// The dressed doubles: one or two outer products into a tensor TT (t1 X1
// and X1 t1 in the tangents of the CC residual), read only by the
// permute-accumulate run right after them.  When every group of that run
// that reads TT fits a summed permute, TT is never stored: those groups
// evaluate it in place from the (small) outer-product factors.  Returns the
// index after the ops run, or i when the pattern does not apply.
template <typename T>
size_t Executor<T>::run_dressed(const OpList& ops, size_t i, int nb) {
  const int tt = ops[i].out;
  if (ops[i].kind != OpKind::Contract || ops[i].acc || bound_[tt]) return i;
  for (int k : keep_)
    if (k == tt) return i;
  SumSources outer{};
  size_t j = i;
  while (j < ops.size() && j < i + 2 && ops[j].out == tt && (j == i) != ops[j].acc && outer_product(ops[j], outer)) ++j;
  if (j == i) return i;
  size_t w = j;
  while (w < ops.size() && ops[w].kind == OpKind::Add) ++w;
  if (w == j) return i;
  for (size_t k = j; k < ops.size(); ++k) {
    if (ops[k].out == tt || ops[k].b == tt) return i;
    if (k >= w && ops[k].a == tt) return i;
  }
  virt_id_ = tt;
  virt_ = outer;
  bool ok = true;
  for (const auto& g : add_groups(ops, j, w)) {
    bool reads = false;
    for (size_t k : g) reads = reads || ops[k].a == tt;
    if (reads && !fuse_adds(ops, g, false)) ok = false;
  }
  if (!ok) {
    virt_id_ = -1;
    return i;
  }
  try {
    run_adds(ops, j, nb);
  } catch (...) {
    virt_id_ = -1;
    throw;
  }
  virt_id_ = -1;
  return w;
}

// Align packed letters `pk` with full letters `fl`: for each packed position,
// the first full position it covers and whether it is a pair.
static void align(const std::string& pk, const std::string& fl, std::vector<int>& fpos, std::vector<int>& ispair) {
  size_t p = 0;
  fpos.clear();
  ispair.clear();
  for (char ch : pk) {
    if (p < fl.size() && fl[p] == ch) {
      fpos.push_back((int)p);
      ispair.push_back(0);
      p += 1;
    } else {
      LRCC_REQUIRE(p + 1 < fl.size(), LRCC_E_INTERNAL, "pack alignment");
      fpos.push_back((int)p);
      ispair.push_back(1);
      p += 2;
    }
  }
  LRCC_REQUIRE(p == fl.size(), LRCC_E_INTERNAL, "pack alignment (length)");
}

template <typename T>
void Executor<T>::pack(const Op& op, int nb) {
  (void)nb;
  LRCC_REQUIRE(!is_virtual(op.a), LRCC_E_INTERNAL, "pack of a virtual constant");
  std::string pk = letters(op.out, op.oi), fl = letters(op.a, op.ai);
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  std::vector<int> fpos, isp;
  align(pk, fl, fpos, isp);
  std::vector<int64_t> fstr(fl.size());
  int64_t s = 1;
  for (int k = (int)fl.size() - 1; k >= 0; --k) {
    fstr[k] = s;
    s *= dimof(fl[k]);
  }
  PackDesc d{};
  d.rank = (int)pk.size();
  int np = 0;
  for (int k = 0; k < d.rank; ++k) {
    int p = fpos[k];
    if (!isp[k]) {
      d.dims[k] = dimof(fl[p]);
      d.fstride[k] = fstr[p];
      d.pair[k] = 0;
    } else {
      int64_t n = dimof(fl[p]);
      d.dims[k] = n * (n - 1) / 2;
      d.pair[k] = 1;
      d.npair[k] = n;
      d.fp[k] = fstr[p];
      d.fq[k] = fstr[p + 1];
      d.mode[k] = op.mode[np++];
    }
  }
  int64_t ptot = 1, fmax = 0;
  for (int k = 0; k < d.rank; ++k) {
    ptot *= d.dims[k];
    if (d.pair[k])
      fmax += (d.npair[k] - 1) * (d.fp[k] + d.fq[k]);
    else
      fmax += (d.dims[k] - 1) * d.fstride[k];
  }
  LRCC_REQUIRE(ptot <= capacity(op.out) && fmax < capacity(op.a) && s <= capacity(op.a), LRCC_E_INTERNAL,
               "pack exceeds its buffers");
  launch_pack<T>(ptr(op.a), ptr(op.out), d, op.are, op.aim, op.acc, st_);
}

template <typename T>
void Executor<T>::unpack(const Op& op, int nb) {
  (void)nb;
  LRCC_REQUIRE(!is_virtual(op.a), LRCC_E_INTERNAL, "unpack of a virtual constant");
  std::string pk = letters(op.a, op.ai), fl = letters(op.out, op.oi);
  auto dimof = [&](char l) { return l == '#' ? g_nb : dim(l); };
  std::vector<int> fpos, isp;
  align(pk, fl, fpos, isp);
  PackDesc d{};
  d.rank = (int)pk.size();
  d.frank = (int)fl.size();
  int np = 0;
  for (int k = 0; k < d.rank; ++k) {
    int p = fpos[k];
    int64_t n = dimof(fl[p]);
    if (!isp[k]) {
      d.dims[k] = n;
      d.pair[k] = 0;
      d.fmap[p] = k;
      d.fsec[p] = -1;
    } else {
      d.dims[k] = n * (n - 1) / 2;
      d.pair[k] = 1;
      d.npair[k] = n;
      d.mode[k] = op.mode[np++];
      d.fmap[p] = k;
      d.fsec[p] = 0;
      d.fmap[p + 1] = k;
      d.fsec[p + 1] = 1;
    }
  }
  int64_t s = 1;
  for (int k = d.rank - 1; k >= 0; --k) {
    d.pstride[k] = s;
    s *= d.dims[k];
  }
  d.full_elems = 1;
  for (int k = 0; k < d.frank; ++k) {
    d.fdims[k] = dimof(fl[k]);
    d.full_elems *= d.fdims[k];
  }
  LRCC_REQUIRE(d.full_elems <= capacity(op.out) && s <= capacity(op.a), LRCC_E_INTERNAL,
               "unpack exceeds its buffers");
  launch_unpack<T>(ptr(op.a), ptr(op.out), d, op.are, op.aim, op.acc, st_);
}

int64_t tensor_elems(const Module& m, const Dims& d, int id, int nb) {
  const TensorDecl& t = m[id];
  int64_t n = t.batched ? nb : 1;
  for (char c : t.cls) n *= d.of(c);
  return n;
}

// Tensors a run pools: batched tensors it writes (except those kept or
// bound), and unbatched temporaries it both writes and reads that no other
// program reads (Module::persistent): intermediates of this run only.
// Unbatched tensors a run writes but never reads are its results and stay.
static bool poolable(const Module& m, int t, const std::vector<char>& read_here) {
  const TensorDecl& d = m[t];
  if (d.batched) return true;
  if (!(d.role == Role::Temp || d.role == Role::Adjoint || d.role == Role::Tangent)) return false;
  if (t < (int)m.persistent.size() && m.persistent[t]) return false;
  return read_here[t] != 0;
}

PoolPlan plan_pool(const Module& m, const Dims& d, const OpList& ops, int nb, const std::vector<int>& keep,
                   const std::vector<char>* bound) {
  const int nt = (int)m.tensors.size();
  std::vector<int> first(nt, -1), last(nt, -1);
  std::vector<char> is_keep(nt, 0), read_here(nt, 0);
  for (int k : keep) is_keep[k] = 1;
  for (int k = 0; k < (int)ops.size(); ++k) {
    const Op& op = ops[k];
    if (first[op.out] < 0) first[op.out] = k;
    last[op.out] = std::max(last[op.out], k);
    if (op.a >= 0) last[op.a] = std::max(last[op.a], k), read_here[op.a] = 1;
    if (op.b >= 0) last[op.b] = std::max(last[op.b], k), read_here[op.b] = 1;
  }
  PoolPlan pl;
  std::vector<int> slot_of(nt, -1);
  std::vector<char> busy;
  for (int k = 0; k < (int)ops.size(); ++k) {
    int t = ops[k].out;
    if (first[t] == k && poolable(m, t, read_here) && !is_keep[t] && !(bound && (*bound)[t])) {
      int64_t need = tensor_elems(m, d, t, nb);
      int best = -1;
      for (int s = 0; s < (int)pl.slot_elems.size(); ++s)
        if (!busy[s] && (best < 0 || std::abs(pl.slot_elems[s] - need) < std::abs(pl.slot_elems[best] - need)))
          best = s;
      if (best < 0) {
        best = (int)pl.slot_elems.size();
        pl.slot_elems.push_back(0);
        busy.push_back(0);
      }
      pl.slot_elems[best] = std::max(pl.slot_elems[best], need);
      busy[best] = 1;
      slot_of[t] = best;
      pl.slot.push_back({t, best});
    }
    // release transients whose last use is this op
    const int used[3] = {ops[k].out, ops[k].a, ops[k].b};
    for (int u : used)
      if (u >= 0 && slot_of[u] >= 0 && last[u] == k) busy[slot_of[u]] = 0;
  }
  // number the slots largest first: the executor's pool holds, per slot
  // number, the largest size any program needs there, so that programs
  // whose plans are alike in size share it closely
  std::vector<int> order(pl.slot_elems.size()), rank(pl.slot_elems.size());
  for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return pl.slot_elems[x] > pl.slot_elems[y]; });
  std::vector<int64_t> sizes(order.size());
  for (size_t q = 0; q < order.size(); ++q) {
    rank[order[q]] = (int)q;
    sizes[q] = pl.slot_elems[order[q]];
  }
  pl.slot_elems = sizes;
  for (auto& ts : pl.slot) ts.second = rank[ts.second];
  return pl;
}

template <typename T>
const PoolPlan& Executor<T>::plan_for(const OpList& ops, int nb, const std::vector<int>& keep) {
  auto key = std::make_pair(&ops, nb);
  auto it = plans_.find(key);
  if (it != plans_.end()) return it->second;
  return plans_.emplace(key, plan_pool(m_, d_, ops, nb, keep, &bound_)).first->second;
}

template <typename T>
int64_t Executor<T>::transient_bytes(const OpList& ops, int nb, const std::vector<int>& keep) {
  const PoolPlan& pl = plan_for(ops, nb, keep);
  int64_t e = 0, big = 0;
  for (int64_t x : pl.slot_elems) e += x;
  for (int k : keep)
    if (m_[k].batched) e += elems(k, nb);
  // the three permutation scratch slots hold at most one batched operand each
  for (const Op& op : ops)
    for (int u : {op.out, op.a, op.b})
      if (u >= 0 && m_[u].batched) big = std::max(big, elems(u, nb));
  e += 3 * big;
  return e * 2 * (int64_t)sizeof(T);
}

template <typename T>
size_t Executor<T>::batched_bytes() const {
  size_t s = 0;
  for (size_t k = 0; k < buf_.size(); ++k)
    if (m_[k].batched && !bound_[k] && !pooled_[k]) s += cap_[k] * sizeof(T) * 2;
  for (int64_t c : pool_cap_) s += c * sizeof(T) * 2;
  for (size_t c : scr_cap_) s += c;
  return s;
}

template <typename T>
void Executor<T>::prepare(const OpList& ops, int nb, const std::vector<int>& keep) {
  const PoolPlan& pl = plan_for(ops, nb, keep);
  if (pool_.size() < pl.slot_elems.size()) {
    pool_.resize(pl.slot_elems.size(), nullptr);
    pool_cap_.resize(pl.slot_elems.size(), 0);
  }
  for (size_t s = 0; s < pl.slot_elems.size(); ++s)
    if (pool_cap_[s] < pl.slot_elems[s]) {
      on_realloc();
      if (pool_[s]) {
        HIP_CHECK(hipStreamSynchronize(st_));
        dev_free(pool_[s]);
        pool_[s] = nullptr;
      }
      pool_[s] = dev_alloc(pl.slot_elems[s] * sizeof(T) * 2);
      pool_cap_[s] = pl.slot_elems[s];
    }
  for (auto& ts : pl.slot) {
    int t = ts.first;
    if (buf_[t] && !bound_[t] && !pooled_[t]) {  // drop a private buffer from earlier runs
      on_realloc();
      HIP_CHECK(hipStreamSynchronize(st_));
      dev_free(buf_[t]);
    }
    buf_[t] = pool_[ts.second];
    cap_[t] = pool_cap_[ts.second];
    pooled_[t] = 1;
  }
}

template <typename T>
void Executor<T>::run_ops(const OpList& ops, int nb) {
  pcache_[0] = pcache_[1] = PermEntry();
  for (size_t i = 0; i < ops.size(); ++i) {
    const Op& op = ops[i];
    switch (op.kind) {
      case OpKind::Contract: {
        const size_t j = run_dressed(ops, i, nb);
        if (j > i)
          i = j - 1;
        else
          contract(op, nb);
        break;
      }
      case OpKind::Add: i = run_adds(ops, i, nb) - 1; break;
      case OpKind::Pack: pack(op, nb); break;
      case OpKind::Unpack: unpack(op, nb); break;
      case OpKind::Zero:
        LRCC_REQUIRE(elems(op.out, nb) <= capacity(op.out), LRCC_E_INTERNAL, "zero-fill exceeds its buffer");
        launch_fill_zero<T>(ptr(op.out), elems(op.out, nb), st_);
        break;
    }
  }
}

template <typename T>
void Executor<T>::run(const OpList& ops, int nb, const std::vector<int>& keep) {
  LRCC_REQUIRE(nb >= 1 && nb <= max_nb_, LRCC_E_INTERNAL, "batch exceeds executor maximum");
  g_nb = nb;
  keep_ = keep;
  prepare(ops, nb, keep);
  if (!graphs_on_ || outer_) {
    run_ops(ops, nb);
    return;
  }
  // capture is not possible on the null stream: fork onto the private one
  const hipStream_t caller = st_;
  const bool fork = caller == nullptr;
  if (fork) {
    HIP_CHECK(hipEventRecord(fork_, caller));
    HIP_CHECK(hipStreamWaitEvent(gst_, fork_, 0));
    st_ = gst_;
  }
  try {
    auto it = graphs_.find(make_key(ops, nb, keep));
    if (it == graphs_.end()) {
      run_ops(ops, nb);  // eager: lazy allocations and GEMM tile tuning happen here
      if (graphs_.size() >= 64) clear_graphs();
      graphs_.emplace(make_key(ops, nb, keep), Recorded());
    } else if (it->second.state == 0) {
      capture(it->second, ops, nb);
    } else {
      replay(it->second);
    }
  } catch (...) {
    st_ = caller;
    throw;
  }
  st_ = caller;
  if (fork) {
    HIP_CHECK(hipEventRecord(join_, gst_));
    HIP_CHECK(hipStreamWaitEvent(st_, join_, 0));
  }
}

template <typename T>
bool Executor<T>::RunKey::operator<(const RunKey& o) const {
  return std::tie(ops, nb, timing, keep, addr) < std::tie(o.ops, o.nb, o.timing, o.keep, o.addr);
}

template <typename T>
typename Executor<T>::RunKey Executor<T>::make_key(const OpList& ops, int nb, const std::vector<int>& keep) const {
  RunKey k{&ops, nb, timing_, keep, {}};
  k.addr.reserve(buf_.size() + scr_.size() + pool_.size());
  k.addr.insert(k.addr.end(), buf_.begin(), buf_.end());
  k.addr.insert(k.addr.end(), scr_.begin(), scr_.end());
  k.addr.insert(k.addr.end(), pool_.begin(), pool_.end());
  return k;
}

template <typename T>
void Executor<T>::capture(Recorded& r, const OpList& ops, int nb) {
  ++captures_;
  r.seg.clear();
  r.timed.clear();
  capturing_ = true;
  rec_ = &r;
  try {
    HIP_CHECK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    run_ops(ops, nb);
    end_segment();
  } catch (...) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st_, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(st_, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    capturing_ = false;
    rec_ = nullptr;
    for (hipGraphExec_t e : r.seg)
      if (e) (void)hipGraphExecDestroy(e);
    r.seg.clear();
    r.timed.clear();
    throw;
  }
  capturing_ = false;
  rec_ = nullptr;
  r.state = 1;
}

// Close the current capture, instantiate it and launch it at once (the
// capturing run executes through its own graphs).
template <typename T>
void Executor<T>::end_segment() {
  hipGraph_t g = nullptr;
  HIP_CHECK(hipStreamEndCapture(st_, &g));
  size_t nodes = 0;
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphGetNodes(g, nullptr, &nodes);
  if (e == hipSuccess && nodes > 0) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_CHECK(e);
  rec_->seg.push_back(ex);
  if (ex) HIP_CHECK(hipGraphLaunch(ex, st_));
}

template <typename T>
void Executor<T>::replay(const Recorded& r) {
  ++replays_;
  for (size_t k = 0; k < r.seg.size(); ++k) {
    if (r.seg[k]) HIP_CHECK(hipGraphLaunch(r.seg[k], st_));
    if (k < r.timed.size()) launch_timed(r.timed[k]);
  }
}

template <typename T>
void Executor<T>::clear_graphs() {
  if (graphs_.empty()) return;
  if (gst_) HIP_CHECK(hipStreamSynchronize(gst_));
  if (st_) HIP_CHECK(hipStreamSynchronize(st_));
  for (auto& kv : graphs_)
    for (hipGraphExec_t e : kv.second.seg)
      if (e) (void)hipGraphExecDestroy(e);
  graphs_.clear();
}

template <typename T>
void Executor<T>::on_realloc() {
  LRCC_REQUIRE(!capturing_ && !outer_, LRCC_E_INTERNAL, "allocation while capturing a graph");
  ++epoch_;
  clear_graphs();
}

template <typename T>
void Executor<T>::begin_outer(hipStream_t cs) {
  LRCC_REQUIRE(!outer_ && !capturing_, LRCC_E_INTERNAL, "nested capture");
  saved_st_ = st_;
  st_ = cs;
  outer_ = true;
}

template <typename T>
void Executor<T>::end_outer() {
  if (!outer_) return;
  st_ = saved_st_;
  outer_ = false;
}

template <typename T>
void Executor<T>::set_graphs(bool on) {
  if (on && !gst_) {
    HIP_CHECK(hipStreamCreateWithFlags(&gst_, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&join_, hipEventDisableTiming));
  }
  if (!on) clear_graphs();
  graphs_on_ = on;
}

template class Executor<double>;
template class Executor<float>;

}  // namespace lrcc
