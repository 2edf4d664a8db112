// Client-side randomness: ChaCha20 keystreams (the block function of RFC 8439) and
// the samplers of the secret key, the key-switching keys and encryptions drawn
// from them.  Host code only: the client samples and the library uploads.
//
// Stream (seed, purpose, index): key = seed as 8 little-endian bytes then 24 zero
// bytes, nonce = (purpose, index >> 32, index & 0xffffffff), block counter from 0;
// a 64-bit value is two consecutive little-endian keystream words, low word first.
// Samplers: ternary (u mod 3) - 1; uniform mod q ((u_hi 2^64 + u_lo) mod q); Gaussian
// by a cumulative distribution table over k in [-19, 19] with sigma = 3.2,
// T_k = floor(2^64 CDF(k)), e = -19 + #{k : u >= T_k}.  The table is evaluated in
// binary128 (113-bit significand): 2^64 CDF(k) lies at least 2^-20 from an integer
// for every k, so any evaluation to 90 or more bits gives the same floors.
#include <cstdint>
#include <cstring>
#include <vector>

#include "sampler.h"

namespace bcn {

namespace {
inline uint32_t rotl(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

inline void qr(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
  a += b; d = rotl(d ^ a, 16);
  c += d; b = rotl(b ^ c, 12);
  a += b; d = rotl(d ^ a, 8);
  c += d; b = rotl(b ^ c, 7);
}

// exp(x) for x <= 0 in binary128: exp(x / 2^10) by its Taylor series, squared ten times
__float128 exp128(__float128 x) {
  __float128 y = x / 1024;
  __float128 term = 1, sum = 1;
  for (int k = 1; k < 40; ++k) {
    term = term * y / k;
    sum += term;
  }
  for (int i = 0; i < 10; ++i) sum = sum * sum;
  return sum;
}
}  // namespace

void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]) {
  uint32_t init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, key[0], key[1], key[2], key[3],
                       key[4],      key[5],      key[6],      key[7],      counter, nonce[0], nonce[1], nonce[2]};
  uint32_t x[16];
  std::memcpy(x, init, sizeof x);
  for (int r = 0; r < 10; ++r) {
    qr(x[0], x[4], x[8], x[12]);
    qr(x[1], x[5], x[9], x[13]);
    qr(x[2], x[6], x[10], x[14]);
    qr(x[3], x[7], x[11], x[15]);
    qr(x[0], x[5], x[10], x[15]);
    qr(x[1], x[6], x[11], x[12]);
    qr(x[2], x[7], x[8], x[13]);
    qr(x[3], x[4], x[9], x[14]);
  }
  for (int i = 0; i < 16; ++i) out[i] = x[i] + init[i];
}

Stream::Stream(uint64_t seed, uint32_t purpose, uint64_t index) {
  std::memset(key_, 0, sizeof key_);
  key_[0] = (uint32_t)seed;
  key_[1] = (uint32_t)(seed >> 32);
  nonce_[0] = purpose;
  nonce_[1] = (uint32_t)(index >> 32);
  nonce_[2] = (uint32_t)index;
}

uint64_t Stream::next() {
  if (pos_ == 8) {
    uint32_t w[16];
    chacha20_block(key_, counter_++, nonce_, w);
    for (int i = 0; i < 8; ++i) buf_[i] = (uint64_t)w[2 * i] | ((uint64_t)w[2 * i + 1] << 32);
    pos_ = 0;
  }
  return buf_[pos_++];
}

const std::vector<uint64_t>& cdt_table() {
  static const std::vector<uint64_t> table = [] {
    const __float128 two_sigma2 = (__float128)2 * (__float128)32 * (__float128)32 / 100;   // 2 * 3.2^2
    std::vector<__float128> rho;
    __float128 total = 0;
    for (int k = -kErrorBound; k <= kErrorBound; ++k) {
      rho.push_back(exp128(-(__float128)(k * k) / two_sigma2));
      total += rho.back();
    }
    std::vector<uint64_t> t;
    __float128 acc = 0;
    const __float128 two64 = (__float128)18446744073709551616.0;
    for (size_t i = 0; i + 1 < rho.size(); ++i) {
      acc += rho[i];
      t.push_back((uint64_t)(acc / total * two64));
    }
    return t;
  }();
  return table;
}

void sample_ternary(Stream& st, int n, int64_t* out) {
  for (int i = 0; i < n; ++i) out[i] = (int64_t)(st.next() % 3) - 1;
}

void sample_uniform(Stream& st, uint64_t q, int n, uint64_t* out) {
  for (int i = 0; i < n; ++i) {
    const unsigned __int128 hi = st.next();
    const unsigned __int128 lo = st.next();
    out[i] = (uint64_t)(((hi << 64) | lo) % q);
  }
}

void sample_gaussian(Stream& st, int n, int64_t* out) {
  const std::vector<uint64_t>& t = cdt_table();
  for (int i = 0; i < n; ++i) {
    const uint64_t u = st.next();
    int64_t c = 0;
    for (uint64_t x : t) c += u >= x ? 1 : 0;
    out[i] = c - kErrorBound;
  }
}

}  // namespace bcn
