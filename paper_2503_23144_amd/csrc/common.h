// Shared host-side definitions of the lrcc runtime.
#pragma once
#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/lrcc.h"

namespace lrcc {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

#define LRCC_REQUIRE(cond, code, msg)                                    \
  do {                                                                   \
    if (!(cond)) throw ::lrcc::Error((code), std::string(msg));          \
  } while (0)

#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::lrcc::Error(e_ == hipErrorOutOfMemory ? LRCC_E_NOMEM : LRCC_E_HIP,          \
                          std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

// Sets the message lrcc_last_error(NULL) returns on this thread.
void set_call_error(const std::string& msg);

enum class Prec { F64 = 0, F32 = 1 };

inline size_t cbytes(Prec p) { return p == Prec::F64 ? 16 : 8; }

}  // namespace lrcc
