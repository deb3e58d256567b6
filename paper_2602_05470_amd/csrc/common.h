// Internal definitions shared by the host code and the HIP kernels.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>
#include <stdexcept>
#include <string>
#include <hip/hip_runtime.h>
#include "../../include/bbtn.h"

namespace bbtn {

constexpr int32_t NEG = BBTN_NEG;
constexpr int32_t NEG_CUT = BBTN_NEG_CUT;
// Residues a pass may carry per entry: the caller's k (at most
// BBTN_MAX_RESIDUES) plus one certification prime fused into the same pass.
constexpr int KUSER = BBTN_MAX_RESIDUES;
constexpr int KMAX = BBTN_MAX_RESIDUES + 1;

// Error carried from deep host code to the C ABI.
struct Error : std::runtime_error {
  bbtn_status status;
  Error(bbtn_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define BBTN_HIP(expr)                                                         \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::bbtn::Error(BBTN_E_DEVICE, std::string(#expr) + ": " +           \
                                             hipGetErrorString(e_));           \
  } while (0)

// after a kernel launch: a launch error names the kernel
#define BBTN_LAUNCHED(what)                                                    \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess)                                                      \
      throw ::bbtn::Error(BBTN_E_DEVICE, std::string("launch of ") + (what) +  \
                                             ": " + hipGetErrorString(e_));    \
  } while (0)

#define BBTN_REQUIRE(cond, msg)                                                \
  do {                                                                         \
    if (!(cond)) throw ::bbtn::Error(BBTN_E_INVALID_ARG, msg);                 \
  } while (0)

// Moduli of one pass: primes p_i and c_i = 2^32 mod p_i.  For
// 2^31 - 2^20 < p < 2^31, c_i = 2^32 - 2 p_i < 2^21, which lets a 64-bit
// accumulator be folded with one multiply-add: x = hi * 2^32 + lo is
// congruent to hi * c + lo < 2^54.
struct Moduli {
  uint32_t p[KMAX];
  uint32_t c[KMAX];
};

inline bool prime_in_range(uint64_t p) {
  return p > (1ull << 31) - (1ull << 20) && p < (1ull << 31);
}

inline Moduli make_moduli(int k, const uint32_t* primes) {
  Moduli m{};
  for (int i = 0; i < k; ++i) {
    BBTN_REQUIRE(prime_in_range(primes[i]), "prime outside (2^31-2^20, 2^31)");
    m.p[i] = primes[i];
    m.c[i] = (uint32_t)((1ull << 32) % primes[i]);
  }
  for (int i = k; i < KMAX; ++i) { m.p[i] = 2147483647u; m.c[i] = 2; }
  return m;
}

// A tensor buffer on the device: (1 + k) planes of `pstride` 32-bit words.
struct DevTensor {
  uint32_t* ptr = nullptr;
  int64_t pstride = 0;  // entries per plane
};

}  // namespace bbtn
