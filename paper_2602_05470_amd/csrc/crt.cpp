#include "crt.h"

namespace bbtn {

static uint32_t powmod(uint64_t a, uint64_t e, uint32_t p) {
  uint64_t r = 1;
  a %= p;
  while (e) {
    if (e & 1) r = r * a % p;
    a = a * a % p;
    e >>= 1;
  }
  return (uint32_t)r;
}

std::vector<uint32_t> crt_garner(const std::vector<uint32_t>& res,
                                 const std::vector<uint32_t>& pr) {
  const size_t k = pr.size();
  // mixed-radix digits: x = a0 + a1 p0 + a2 p0 p1 + ...
  std::vector<uint32_t> a(k);
  for (size_t i = 0; i < k; ++i) {
    const uint32_t p = pr[i];
    // value of the digits so far, modulo p
    uint64_t v = 0, w = 1;
    for (size_t j = 0; j < i; ++j) {
      v = (v + (uint64_t)a[j] * w) % p;
      w = w * (pr[j] % p) % p;
    }
    const uint64_t diff = ((uint64_t)res[i] % p + p - v) % p;
    a[i] = (uint32_t)(diff * powmod(w, p - 2, p) % p);  // p prime
  }
  // Horner: x = a0 + p0 (a1 + p1 (a2 + ...)); start from the top digit
  std::vector<uint32_t> x{k ? a[k - 1] : 0u};
  for (size_t ii = k - 1; k > 1 && ii-- > 0;) {
    uint64_t carry = a[ii];
    for (auto& wd : x) {
      const uint64_t t = (uint64_t)wd * pr[ii] + carry;
      wd = (uint32_t)t;
      carry = t >> 32;
    }
    while (carry) { x.push_back((uint32_t)carry); carry >>= 32; }
  }
  while (x.size() > 1 && x.back() == 0) x.pop_back();
  return x;
}

uint32_t bigint_mod(const std::vector<uint32_t>& x, uint32_t p) {
  uint64_t r = 0;
  for (size_t i = x.size(); i-- > 0;) r = ((r << 32) | x[i]) % p;
  return (uint32_t)r;
}

int bigint_bits(const std::vector<uint32_t>& x) {
  for (size_t i = x.size(); i-- > 0;)
    if (x[i]) return (int)(32 * i + 32 - __builtin_clz(x[i]));
  return 0;
}

}  // namespace bbtn
