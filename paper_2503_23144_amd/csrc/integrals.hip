// Antisymmetrized spinor-integral blocks from density-fitting factors.
//
//   (pr|qs)  = sum_Q B^Q_pr B^Q_qs
//   <pq||rs> = (pr|qs) - (ps|qr)          (the integrals of Eq. 39)
//
// Each block <PQ||RS> (P, Q, R, S in {occ, vir}) is two MFMA GEMMs over the
// auxiliary index (K = naux) followed by a permute-accumulate, chunked over
// the first index so that no temporary exceeds a fixed budget.  The packed
// vvvv matrix W[P(a,b)][P(e,f)] (a<b, e<f) is built chunk by chunk over a,
// computing (ae|bf) only for b >= the chunk start.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "devmem.h"
#include "integrals.h"
#include "kernels.h"

namespace lrcc {

namespace {

struct DevTmp {
  void* p = nullptr;
  explicit DevTmp(size_t bytes) { p = dev_alloc(std::max<size_t>(bytes, 16)); }
  ~DevTmp() { dev_free(p); }
};

constexpr size_t kChunkBytes = size_t(1) << 30;

}  // namespace

void build_block(const void* Bdev, int64_t naux, int64_t o, int64_t v, const std::string& spec, void* dst,
                 hipStream_t st, bool pack_last) {
  const int64_t nmo = o + v;
  auto start = [&](char c) { return c == 'o' ? int64_t(0) : o; };
  auto len = [&](char c) { return c == 'o' ? o : v; };
  const char P = spec[0], Q = spec[1], R = spec[2], S = spec[3];
  const int64_t np = len(P), nq = len(Q), nr = len(R), ns = len(S);
  if (np * nq * nr * ns == 0) return;
  DevTmp LPR(naux * np * nr * 16), LQS(naux * nq * ns * 16), LPS(naux * np * ns * 16), LQR(naux * nq * nr * 16);
  launch_gather_block(naux, nmo, start(P), np, start(R), nr, Bdev, LPR.p, st);
  launch_gather_block(naux, nmo, start(Q), nq, start(S), ns, Bdev, LQS.p, st);
  launch_gather_block(naux, nmo, start(P), np, start(S), ns, Bdev, LPS.p, st);
  launch_gather_block(naux, nmo, start(Q), nq, start(R), nr, Bdev, LQR.p, st);
  const int64_t per_p = nq * nr * ns * 16;
  int64_t pc = std::max<int64_t>(1, std::min<int64_t>(np, (int64_t)kChunkBytes / per_p));
  DevTmp tmp(pc * per_p);
  // with pack_last, each chunk is formed densely here and packed over (r < s)
  LRCC_REQUIRE(!pack_last || R == S, LRCC_E_INTERNAL, "packed block needs equal last classes");
  DevTmp dense(pack_last ? pc * per_p : 16);
  for (int64_t p0 = 0; p0 < np; p0 += pc) {
    int64_t pn = std::min(pc, np - p0);
    char* out = pack_last ? (char*)dense.p : (char*)dst + p0 * per_p;
    // Coulomb (pr|qs): rows (p, r), columns (q, s)
    launch_gemm<double>(true, false, pn * nr, nq * ns, naux, 1.0, 0.0, (const char*)LPR.p + p0 * nr * 16, np * nr,
                        LQS.p, nq * ns, 0.0, 0.0, tmp.p, nq * ns, st);
    PermDesc d{};
    d.rank = 4;
    d.dims[0] = pn, d.dims[1] = nq, d.dims[2] = nr, d.dims[3] = ns;
    d.istride[0] = nr * nq * ns, d.istride[1] = ns, d.istride[2] = nq * ns, d.istride[3] = 1;
    launch_permute<double>(tmp.p, out, d, 1.0, 0.0, 0.0, 0.0, st);
    // exchange (ps|qr): rows (p, s), columns (q, r)
    launch_gemm<double>(true, false, pn * ns, nq * nr, naux, 1.0, 0.0, (const char*)LPS.p + p0 * ns * 16, np * ns,
                        LQR.p, nq * nr, 0.0, 0.0, tmp.p, nq * nr, st);
    d.istride[0] = ns * nq * nr, d.istride[1] = nr, d.istride[2] = 1, d.istride[3] = nq * nr;
    launch_permute<double>(tmp.p, out, d, -1.0, 0.0, 1.0, 0.0, st);
    if (pack_last) pack_last_pair(out, pn, nq, nr, (char*)dst + p0 * nq * (nr * (nr - 1) / 2) * 16, st);
  }
  HIP_CHECK(hipStreamSynchronize(st));
}

void build_packed_vvvv(const void* Bdev, int64_t naux, int64_t o, int64_t v, void* W, hipStream_t st) {
  const int64_t nmo = o + v;
  if (v < 2) return;
  DevTmp L(naux * v * v * 16);
  launch_gather_block(naux, nmo, o, v, o, v, Bdev, L.p, st);
  int64_t a0 = 0;
  DevTmp tmp(std::min<int64_t>((int64_t)kChunkBytes, v * v * v * v * 16));
  while (a0 < v - 1) {
    int64_t per_a = v * (v - a0) * v * 16;
    int64_t na = std::max<int64_t>(1, std::min<int64_t>(v - 1 - a0, (int64_t)kChunkBytes / per_a));
    LRCC_REQUIRE(na * per_a <= (int64_t)kChunkBytes, LRCC_E_NOMEM, "vvvv chunk exceeds budget (v too large)");
    int64_t a1 = a0 + na;
    // (ae|bf) for a in [a0, a1), b >= a0
    launch_gemm<double>(true, false, na * v, (v - a0) * v, naux, 1.0, 0.0, (const char*)L.p + a0 * v * 16, v * v,
                        (const char*)L.p + a0 * v * 16, v * v, 0.0, 0.0, tmp.p, (v - a0) * v, st);
    launch_pack_vvvv<double>(v, a0, a1, a0, tmp.p, W, st);
    a0 = a1;
  }
  HIP_CHECK(hipStreamSynchronize(st));
}

template <typename TO>
void build_vvvv_triangle(const void* Lvv, int64_t naux, int64_t v, const std::vector<int64_t>& bnd,
                         const std::vector<int64_t>& offs, void* dst, hipStream_t st) {
  const int64_t V = v * (v - 1) / 2;
  auto R = [](int64_t b) { return b * (b - 1) / 2; };
  DevTmp C(kChunkBytes), Wc(kChunkBytes);
  for (size_t j = 0; j + 1 < bnd.size(); ++j) {
    const int64_t r0 = R(bnd[j]), ld = V - r0;
    for (int64_t c0 = bnd[j]; c0 < bnd[j + 1];) {
      // rows of b in [c0, c1): the (ae|bf) block and the rows of W must fit a chunk
      int64_t c1 = c0 + 1;
      auto fits = [&](int64_t cc) {
        return (size_t)((cc - c0) * v) * (size_t)(cc * v) * 16 <= kChunkBytes &&
               (size_t)(R(cc) - R(c0)) * (size_t)V * 16 <= kChunkBytes;
      };
      LRCC_REQUIRE(fits(c1), LRCC_E_NOMEM, "vvvv row chunk exceeds budget (v too large)");
      while (c1 < bnd[j + 1] && fits(c1 + 1)) ++c1;
      // (ae|bf): rows (b, f) for b in [c0, c1), columns (a, e) for a < c1
      launch_gemm<double>(true, false, (c1 - c0) * v, c1 * v, naux, 1.0, 0.0, (const char*)Lvv + c0 * v * 16, v * v,
                          Lvv, v * v, 0.0, 0.0, C.p, c1 * v, st);
      launch_pack_wrows<double>(v, c0, c1, C.p, Wc.p, st);
      launch_copy_rows<double, TO>(R(c1) - R(c0), ld, (const char*)Wc.p + r0 * 16, V,
                                   (char*)dst + (offs[j] + (R(c0) - r0) * ld) * 2 * sizeof(TO), ld, st);
      c0 = c1;
    }
  }
  HIP_CHECK(hipStreamSynchronize(st));
}

template void build_vvvv_triangle<double>(const void*, int64_t, int64_t, const std::vector<int64_t>&,
                                          const std::vector<int64_t>&, void*, hipStream_t);
template void build_vvvv_triangle<float>(const void*, int64_t, int64_t, const std::vector<int64_t>&,
                                         const std::vector<int64_t>&, void*, hipStream_t);

void pack_last_pair(const void* full, int64_t n0, int64_t n1, int64_t n, void* packed, hipStream_t st) {
  // packed[x][y][P(e,f)] = full[x][y][e][f], e < f
  PackDesc d{};
  d.rank = 3;
  d.dims[0] = n0, d.dims[1] = n1, d.dims[2] = n * (n - 1) / 2;
  d.fstride[0] = n1 * n * n, d.fstride[1] = n * n;
  d.pair[0] = d.pair[1] = 0;
  d.pair[2] = 1;
  d.npair[2] = n;
  d.fp[2] = n;
  d.fq[2] = 1;
  d.mode[2] = 0;
  launch_pack<double>(full, packed, d, 1.0, 0.0, false, st);
}

}  // namespace lrcc
