// Host check of the library's exact FP64 residue arithmetic (csrc/modarith.h)
// and host number theory (csrc/hostmath.h) against 128-bit integer arithmetic.
// Prints one line per check; exit status 0 when everything agrees.
#include <cstdint>
#include <cstdio>
#include <random>

#include "../../paper_2402_01296_amd/csrc/hostmath.h"
#include "../../paper_2402_01296_amd/csrc/modarith.h"

using namespace bcn;
typedef __int128 i128;
typedef unsigned __int128 u128;

int main(int argc, char** argv) {
  std::mt19937_64 g(12345);
  const uint64_t primes[] = {1073692673ull, 68719230977ull, 1099510054913ull, 1032193ull, 65537ull, 2199023190017ull};
  long bad = 0, checks = 0;
  for (uint64_t q : primes) {
    const Mod m{(double)q, 1.0 / (double)q};
    const bool big = q >= (1ull << 24);
    for (int it = 0; it < 300000; ++it) {
      const int64_t a = (int64_t)(g() % q);
      int64_t b = (int64_t)(g() % (1ull << 47)) - (1ll << 46);     // lazy operand, |b| < 2^46
      if (it & 1) b = (int64_t)(g() % q);
      const double r = mul_lazy((double)a, (double)b, m);
      i128 ex = ((i128)a * b) % (i128)q;
      if (ex < 0) ex += q;
      i128 rr = (i128)(int64_t)r % (i128)q;
      if (rr < 0) rr += q;
      ++checks;
      if (!(r > -(double)q && r < (double)q) || rr != ex) ++bad;
      const int64_t x = (int64_t)(g() % (1ull << 53)) - (1ll << 52) + 1;   // |x| < 2^52
      int64_t ex2 = x % (int64_t)q;
      if (ex2 < 0) ex2 += q;
      ++checks;
      if ((int64_t)reduce((double)x, m) != ex2) ++bad;
      if (big) {
        const uint64_t ta = g() % (1ull << 21), tb = g() % q, tc = g() % (1ull << 21);
        double quo;
        const double rem = mul_add_divmod((double)ta, (double)tb, (double)tc, m, &quo);
        const u128 full = (u128)ta * tb + tc;
        ++checks;
        if ((u128)(uint64_t)quo != full / q || (u128)(uint64_t)rem != full % q) ++bad;
      }
    }
  }
  std::printf("modarith checks=%ld bad=%ld\n", checks, bad);
  // host prime rule and roots (compared with the oracle by the Python test)
  const auto p = host::ntt_primes(36, 16384, 5, {1032193});
  std::printf("primes36_8192");
  for (auto x : p) std::printf(" %llu", (unsigned long long)x);
  std::printf("\nroots %llu %llu %llu\n", (unsigned long long)host::negacyclic_root(65537, 4096),
              (unsigned long long)host::negacyclic_root(1032193, 8192),
              (unsigned long long)host::negacyclic_root(1099510054913ull, 16384));
  std::printf("inv_pow2 %llu\n", (unsigned long long)((host::inv_pow2(3, 15) * 3) & ((1u << 15) - 1)));
  return bad != 0;
}
