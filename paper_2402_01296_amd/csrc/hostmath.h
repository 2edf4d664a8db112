// Host-side number theory for building the RNS tables: 64-bit modular
// arithmetic through 128-bit products, deterministic Miller-Rabin, roots of
// unity and bit reversal.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <vector>

namespace bcn {
namespace host {

typedef unsigned __int128 u128;

inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

inline uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}

// inverse of a mod m (m prime, a not divisible by m), by Fermat
inline uint64_t invmod(uint64_t a, uint64_t m) {
  a %= m;
  if (a == 0) throw std::runtime_error("invmod of zero");
  return powmod(a, m - 2, m);
}

// Miller-Rabin with the first twelve prime bases: deterministic below 3.3e24.
inline bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : bases) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

// The `count` largest primes p < 2^bits with p = 1 mod two_n, descending,
// skipping the values in `skip`.
inline std::vector<uint64_t> ntt_primes(int bits, uint64_t two_n, int count, const std::vector<uint64_t>& skip) {
  std::vector<uint64_t> out;
  uint64_t k = ((1ull << bits) - 2) / two_n;
  while ((int)out.size() < count) {
    uint64_t p = k * two_n + 1;
    if (p < (1ull << (bits - 1))) throw std::runtime_error("not enough NTT-friendly primes");
    bool skipped = false;
    for (uint64_t s : skip) skipped |= (s == p);
    if (!skipped && is_prime(p)) out.push_back(p);
    --k;
  }
  return out;
}

// Smallest x >= 2 with x^n = -1 mod q (n a power of two, 2n | q-1).  The
// solutions are the odd powers of psi0 = g^((q-1)/2n) for a quadratic
// non-residue g, so the smallest is a minimum over n candidates.
inline uint64_t negacyclic_root(uint64_t q, uint64_t n) {
  if ((q - 1) % (2 * n) != 0) throw std::runtime_error("q is not 1 mod 2N");
  uint64_t g = 2;
  while (powmod(g, (q - 1) / 2, q) != q - 1) ++g;
  const uint64_t psi0 = powmod(g, (q - 1) / (2 * n), q);
  const uint64_t sq = mulmod(psi0, psi0, q);
  uint64_t best = q, x = psi0;
  for (uint64_t i = 0; i < n; ++i) {
    if (x < best) best = x;
    x = mulmod(x, sq, q);
  }
  return best;
}

// inverse of an odd k modulo 2^bits (Newton iteration on 2-adic integers)
inline uint64_t inv_pow2(uint64_t k, int bits) {
  uint64_t x = k;                       // correct to 3 bits for odd k
  for (int i = 0; i < 6; ++i) x *= 2 - k * x;
  return bits >= 64 ? x : (x & ((1ull << bits) - 1));
}

inline uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

}  // namespace host
}  // namespace bcn
