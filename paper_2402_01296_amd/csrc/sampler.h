// Client-side ChaCha20 streams and samplers (sampler.hip).
#pragma once

#include <cstdint>
#include <vector>

namespace bcn {

constexpr int kErrorBound = 19;   // Gaussian support [-19, 19], sigma 3.2
enum : uint32_t { kPurposeSecret = 1, kPurposeKskA = 2, kPurposeKskE = 3, kPurposeEncA = 4, kPurposeEncE = 5 };

void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]);

class Stream {
 public:
  Stream(uint64_t seed, uint32_t purpose, uint64_t index);
  uint64_t next();

 private:
  uint32_t key_[8], nonce_[3];
  uint32_t counter_ = 0;
  uint64_t buf_[8];
  int pos_ = 8;
};

const std::vector<uint64_t>& cdt_table();   // the 38 thresholds
void sample_ternary(Stream& st, int n, int64_t* out);
void sample_uniform(Stream& st, uint64_t q, int n, uint64_t* out);
void sample_gaussian(Stream& st, int n, int64_t* out);

}  // namespace bcn
