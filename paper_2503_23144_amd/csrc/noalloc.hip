// lrcc_gemm_noalloc: the complex GEMM of lrcc_gemm without any device
// allocation, for callers that cannot allocate (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The only device memory lrcc_gemm allocates is the split-K workspace: deep
// products with few output tiles are split over K into partial products that
// a second kernel reduces in fixed order.  Here those partials live in a
// static device array of kStaticScratchBytes per GPU, which every GPU that
// runs this entry point holds until the process ends.  The library never
// splits a product into more than 256 MiB of partials (gemm_splits caps the
// split at that size), so the array holds the split the library picks for
// every shape; a product that would need more is rejected with
// LRCC_E_INVALID.  The partials are written in full before they are read,
// so nothing has to be cleared between calls.  All calls on one GPU share
// its array: calls that overlap in time on one GPU (on different streams)
// race on it.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "common.h"
#include "kernels.h"
#include "lrcc.h"

static constexpr size_t kStaticScratchBytes = size_t(256) << 20;

// The split-K partials of lrcc_gemm_noalloc.  Host code never passes this
// name to a kernel: it is a host-side stand-in there.  Its device address,
// one per GPU, comes from hipGetSymbolAddress (scratch_on_current_device).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_mu;
std::map<int, void*> g_addr;  // device ordinal -> address of that device's array

// Address of the current device's array, looked up once per device with that
// device current.
void* scratch_on_current_device() {
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_addr.find(dev);
  if (it != g_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  LRCC_REQUIRE(e == hipSuccess && p != nullptr, LRCC_E_HIP,
               std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_addr[dev] = p;
  return p;
}

}  // namespace

extern "C" int lrcc_gemm_noalloc(int precision, int transa, int transb, int64_t m, int64_t n, int64_t k,
                                 const double alpha[2], const void* A, int64_t lda, const void* B, int64_t ldb,
                                 const double beta[2], void* C, int64_t ldc, void* stream) {
  using namespace lrcc;
  try {
    LRCC_REQUIRE(alpha && beta && A && B && C, LRCC_E_INVALID, "null argument");
    LRCC_REQUIRE(precision == LRCC_FP64 || precision == LRCC_MIXED, LRCC_E_INVALID, "bad precision");
    LRCC_REQUIRE(m >= 0 && n >= 0 && k >= 0, LRCC_E_INVALID, "negative size");
    LRCC_REQUIRE(lda >= (transa ? m : k) && ldb >= (transb ? k : n) && ldc >= n, LRCC_E_INVALID, "leading dimension");
    const size_t wsb = precision == LRCC_FP64 ? gemm_workspace_bytes<double>(m, n, k)
                                              : gemm_workspace_bytes<float>(m, n, k);
    LRCC_REQUIRE(wsb <= kStaticScratchBytes, LRCC_E_INVALID,
                 "product needs " + std::to_string(wsb) + " bytes of split-K partials, above the " +
                     std::to_string(kStaticScratchBytes) + "-byte static scratch of lrcc_gemm_noalloc");
    void* ws = wsb ? scratch_on_current_device() : nullptr;
    const hipStream_t st = (hipStream_t)stream;
    if (precision == LRCC_FP64)
      launch_gemm<double>(transa != 0, transb != 0, m, n, k, alpha[0], alpha[1], A, lda, B, ldb, beta[0], beta[1], C,
                          ldc, st, 0, ws, wsb, nullptr, false, false);
    else
      launch_gemm<float>(transa != 0, transb != 0, m, n, k, alpha[0], alpha[1], A, lda, B, ldb, beta[0], beta[1], C,
                         ldc, st, 0, ws, wsb, nullptr, false, false);
    HIP_CHECK(hipGetLastError());
    return LRCC_OK;
  } catch (const Error& e) {
    set_call_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_call_error(e.what());
    return LRCC_E_INTERNAL;
  }
}
