// Executor of contraction programs on one GPU.
//
// Every operation of an OpList becomes HIP kernel launches on one stream:
//   Contract  -> (optional) index permutation of each operand into GEMM
//                order, one complex MFMA GEMM, (optional) permutation of the
//                product into the output order  (transpose-transpose-GEMM-
//                transpose); a full contraction to a scalar is a reduction.
//   Add       -> one permutation kernel (alpha, beta)
//   Pack/Unpack -> one pair (un)packing kernel
//   Zero      -> fill kernel
// Batched tensors (tangents/adjoints of nb right-hand sides) carry a leading
// batch index '#', which the planner folds into the GEMM M dimension.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "program.h"

namespace lrcc {

struct Dims {
  int64_t o = 0, v = 0, O = 0, V = 0;
  int64_t of(char cls) const { return cls == 'o' ? o : cls == 'v' ? v : cls == 'O' ? O : V; }
};

// HIP-event totals per class: 0 = FP32 (3M) ladder GEMM, 1 = FP64 (4M)
// ladder GEMM, 2 = every GEMM (executed real flops: 6 MNK for 3M, 8 MNK for 4M).
struct KernelTimes {
  double ms[3] = {0, 0, 0};
  int64_t launches[3] = {0, 0, 0};
  double flops[3] = {0, 0, 0};
  void clear() { *this = KernelTimes(); }
};

// Liveness plan of the batched transients of one program run: pool slot
// sizes (complex elements) and the (tensor, slot) assignment.  Tensors in
// `keep` and bound tensors are not pooled.
struct PoolPlan {
  std::vector<std::pair<int, int>> slot;
  std::vector<int64_t> slot_elems;
};
int64_t tensor_elems(const Module& m, const Dims& d, int id, int nb);
PoolPlan plan_pool(const Module& m, const Dims& d, const OpList& ops, int nb, const std::vector<int>& keep,
                   const std::vector<char>* bound);

template <typename T>
class Executor {
 public:
  Executor(const Module& m, Dims d, hipStream_t st);
  ~Executor();
  Executor(const Executor&) = delete;
  Executor& operator=(const Executor&) = delete;

  int64_t elems(int id, int nb) const;  // complex elements of tensor id at batch nb
  const Module& module() const { return m_; }
  // Storage: owned (allocated on first use for the current max batch) or bound.
  void* ptr(int id);
  void bind(int id, void* p);
  void unbind(int id);
  void set_max_batch(int nb);
  int max_batch() const { return max_nb_; }
  // Run a program at batch nb.  Batched tensors written by the program
  // (except those listed in `keep`) are transient: they live in a pool whose
  // buffers are reused once a tensor's last reader has run.
  void run(const OpList& ops, int nb, const std::vector<int>& keep = {});
  // Device bytes a run at batch nb needs for pooled transients, kept batched
  // tensors and the permutation scratch slots.
  int64_t transient_bytes(const OpList& ops, int nb, const std::vector<int>& keep);
  // Bytes held now by batch-dependent storage (pool, batched tensors, scratch).
  size_t batched_bytes() const;
  // Free all batch-dependent storage (it is re-allocated on the next run).
  void release_batched();
  // Free the private storage of the unbatched tensors `ops` writes (its
  // results; they are formed again by the next run of `ops`).
  void release_results(const OpList& ops);
  // Free the private storage of one unbatched tensor (allocated again on
  // its next use).
  void release(int id);
  size_t bytes_allocated() const;

  // optional per-launch timing (HIP events on the stream)
  void set_timing(bool on) { timing_ = on; }
  void collect_times(KernelTimes& kt);  // synchronizes; accumulates and clears pending events
  int ladder_const = -1;                // tensor id whose contractions count as the ladder
  // DF-direct ladder: with the virtual-virtual block of the density-fitting
  // factors L[Q][a][e] (naux x v x v, precision T, owned by the caller) set,
  // a contraction with the ladder constant W[P(a,b)][P(e,f)] = <ab||ef>
  // rebuilds W's rows chunk by chunk from L instead of reading a resident W.
  void set_direct_ladder(const void* L, int64_t naux, int64_t v) {
    dl_L_ = L;
    dl_naux_ = naux;
    dl_v_ = v;
  }
  static constexpr size_t kDirectChunkBytes = size_t(512) << 20;  // per scratch buffer of the rebuild
  // Hermitian-triangle ladder: W held as row blocks, block j covering rows
  // [r0, r1) and columns [r0, V) (row length V - r0, precision T, owned by
  // the caller); the entries left of each block follow from W = W^H.
  struct TriBlock {
    int64_t r0, r1;
    const void* p;
  };
  void set_triangle_ladder(const std::vector<TriBlock>& blocks) { tri_ = blocks; }

  // Constants held only through another tensor (no storage of their own).
  // V[vl] = alpha_v * X(src[sl]): sl lists the source's indices in stored
  // order, written with V's letters; the two letters at pair_at (if >= 0)
  // are the source's packed antisymmetric pair P(p, q), p < q; X is complex
  // conjugation when `conj`.  A contraction reading V materializes it into
  // a scratch slot in the order the GEMM wants, in chunks over the index at
  // position `chunk` of vl when that index is contracted or an output index
  // (at most virtual_chunk_bytes per chunk); a permuted copy (Add) writes
  // straight into its output.  Used for <ov||vv> and <vv||vo> (from the
  // packed <ov||vv>) and <vv||oo> (from <oo||vv>), whose dense forms are the
  // largest integral blocks after vvvv.
  struct VirtualDef {
    int src = -1;
    std::string vl, sl;
    int pair_at = -1;
    double sre = 1.0, sim = 0.0;
    bool conj = false;
    int chunk = -1;
  };
  void set_virtual(int id, const VirtualDef& d);
  bool is_virtual(int id) const { return id >= 0 && id < (int)vdef_.size() && vdef_[id].src >= 0; }
  void set_virtual_chunk_bytes(size_t b) { vchunk_bytes_ = std::max<size_t>(b, 1); }

  // HIP graph replay.  With graphs on, a run whose program, batch and every
  // buffer address match an earlier (eager) run is captured into HIP graphs
  // on the second occurrence and replayed from the third on.  On the null
  // stream, graph runs execute on a private stream joined to it by events.
  // With timing on, the ladder GEMMs stay outside the graphs (launched
  // between graph segments) so HIP events can time them; the other GEMMs
  // inside graphs are then not timed.
  void set_graphs(bool on);
  int64_t graph_replays() const { return replays_; }
  int64_t graph_captures() const { return captures_; }
  // Outer capture: launches go to stream cs (which the caller is capturing
  // into a graph of its own) and run eagerly, this executor's own graphs
  // suspended; any allocation change meanwhile throws (it would invalidate
  // the caller's graph).  epoch() counts allocation changes.
  void begin_outer(hipStream_t cs);
  void end_outer();
  int64_t epoch() const { return epoch_; }

 private:
  struct LadderOperands {  // X[M][V] (contracted index last), output C[M][V]
    const void* X;
    void* C;
    int64_t M, V, capX, capC;
    bool over_col;  // C = X W^T (contraction over W's column index), else C = X W
  };
  LadderOperands ladder_operands(const Op& op);
  void ladder_direct(const Op& op);
  void ladder_triangle(const Op& op);
  std::vector<TriBlock> tri_;
  const void* dl_L_ = nullptr;
  int64_t dl_naux_ = 0, dl_v_ = 0;
  struct GemmArgs {
    bool ta, tb;
    int64_t M, N, K;
    double are, aim;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    double bre;
    void* C;
    int64_t ldc;
    bool ladder;
    void* ws;  // split-K partials (scratch slot 4)
    size_t wsb;
    OutMap om;  // output layout when mapped
    bool mapped;
    bool conjb;  // use conj(B)
  };
  struct RunKey {
    const OpList* ops;
    int nb;
    bool timing;
    std::vector<int> keep;
    std::vector<void*> addr;  // every tensor and scratch buffer
    bool operator<(const RunKey& o) const;
  };
  struct Recorded {
    int state = 0;                     // 0: seen once (eager), 1: captured
    std::vector<hipGraphExec_t> seg;   // graph segments, timed GEMMs between them
    std::vector<GemmArgs> timed;
  };
  void prepare(const OpList& ops, int nb, const std::vector<int>& keep);
  void run_ops(const OpList& ops, int nb);
  RunKey make_key(const OpList& ops, int nb, const std::vector<int>& keep) const;
  void capture(Recorded& r, const OpList& ops, int nb);
  void replay(const Recorded& r);
  void end_segment();
  void launch_timed(const GemmArgs& g);
  void clear_graphs();
  void on_realloc();  // every allocation change invalidates recorded graphs
  std::map<RunKey, Recorded> graphs_;
  bool graphs_on_ = false;
  bool capturing_ = false;
  bool outer_ = false;
  hipStream_t saved_st_ = nullptr;
  int64_t epoch_ = 0;
  Recorded* rec_ = nullptr;
  hipStream_t gst_ = nullptr;  // private stream of graph runs
  hipEvent_t fork_ = nullptr, join_ = nullptr;
  int64_t replays_ = 0, captures_ = 0;

  void contract(const Op& op, int nb);
  void contract_virtual(const Op& op);
  // Writes V (letters vlet, as in an op) into dst in the order of `tgt`,
  // restricted to [g0, g0 + gl) along letter g (0: no restriction).
  void materialize(int id, const std::string& vlet, const std::string& tgt, char g, int64_t g0, int64_t gl,
                   void* dst, int64_t dst_cap, double are, double aim, bool acc);
  std::vector<VirtualDef> vdef_;
  size_t vchunk_bytes_ = size_t(1) << 30;
  void add(const Op& op, int nb);
  bool fuse_adds(const OpList& ops, const std::vector<size_t>& idx, bool launch = true);
  std::vector<std::vector<size_t>> add_groups(const OpList& ops, size_t i, size_t w) const;
  size_t run_adds(const OpList& ops, size_t i, int nb);
  bool outer_product(const Op& o, SumSources& s);
  size_t run_dressed(const OpList& ops, size_t i, int nb);
  int virt_id_ = -1;      // tensor evaluated in place by summed permutes (run_dressed)
  SumSources virt_{};     // its outer products
  std::vector<int> keep_;  // tensors the current run keeps
  void pack(const Op& op, int nb);
  void unpack(const Op& op, int nb);
  void permute_into(const void* src, int64_t src_cap, const std::string& sl, void* dst, int64_t dst_cap,
                    const std::string& dl, double are, double aim, double bre, double bim);
  void* scratch(int slot, size_t bytes);
  int64_t scratch_elems(int slot) const { return (int64_t)(scr_cap_[slot] / (2 * sizeof(T))); }
  int64_t capacity(int id);  // complex elements addressable through ptr(id) (allocates if needed)
  int64_t dim(char letter) const;
  std::string letters(int id, const std::string& idx) const;
  void gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double are, double aim, const void* A,
            int64_t lda, int64_t capA, const void* B, int64_t ldb, int64_t capB, double bre, void* C, int64_t ldc,
            int64_t capC, bool ladder, const OutMap* om = nullptr, bool conjb = false);
  bool output_map(const std::string& Mc, const std::string& Nc, const std::string& cl, OutMap& om) const;
  int cached_permute(int id, const std::string& src, const std::string& dst, const void* p, int64_t cap);
  static constexpr int kPermSlot = 5;
  struct PermEntry {
    int tensor = -1;
    std::vector<int> perm;
    int64_t nb = 0;
  };
  PermEntry pcache_[2];
  int pnext_ = 0;

  const PoolPlan& plan_for(const OpList& ops, int nb, const std::vector<int>& keep);
  std::map<std::pair<const OpList*, int>, PoolPlan> plans_;
  std::vector<void*> pool_;
  std::vector<int64_t> pool_cap_;
  std::vector<char> pooled_;

  const Module& m_;
  Dims d_;
  hipStream_t st_;
  int max_nb_ = 1;
  std::vector<void*> buf_;
  std::vector<int64_t> cap_;  // allocated elements
  std::vector<char> bound_;
  std::vector<void*> scr_;
  std::vector<size_t> scr_cap_;
  void* dot_out_ = nullptr;
  void* dot_work_ = nullptr;
  bool timing_ = false;
  struct Pending {
    hipEvent_t a, b;
    int cls;
    double flops;
  };
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> event_pool_;
  hipEvent_t get_event();
  int cur_cls_ = -1;
};

}  // namespace lrcc
