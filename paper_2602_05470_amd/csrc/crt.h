// Exact counts from residues (Chinese remaindering, Garner's mixed radix).
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace bbtn {

// Little-endian 32-bit words of the unique x in [0, prod p_i) with
// x = r_i (mod p_i).  Primes must be distinct.
std::vector<uint32_t> crt_garner(const std::vector<uint32_t>& residues,
                                 const std::vector<uint32_t>& primes);

// x mod p for a little-endian word vector.
uint32_t bigint_mod(const std::vector<uint32_t>& x, uint32_t p);

// Number of bits of x (0 for zero).
int bigint_bits(const std::vector<uint32_t>& x);

}  // namespace bbtn
