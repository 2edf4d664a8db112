// Context creation: prime selection, per-prime transform tables, exact
// conversion constants and the scratch arena.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "scheme.h"

namespace bcn {

Arena::~Arena() {
  for (auto& ch : chunks_) (void)hipFree(ch.p);
  for (auto& ch : retired_) (void)hipFree(ch.p);
}

size_t Arena::capacity() const {
  size_t c = 0;
  for (auto& ch : chunks_) c += ch.cap;
  return c * sizeof(double);
}

size_t Arena::retired_bytes() const {
  size_t c = 0;
  for (auto& ch : retired_) c += ch.cap;
  return c * sizeof(double);
}

size_t Arena::release_retired() {
  const size_t b = retired_bytes();
  if (retired_.empty()) return 0;
  BCN_HIP(hipDeviceSynchronize());
  for (auto& ch : retired_) BCN_HIP(hipFree(ch.p));
  retired_.clear();
  return b;
}

void Arena::bind_external(double* base, size_t cap) {
  ext_ = base;
  ext_cap_ = cap;
  ext_off_ = 0;
}

void Arena::unbind_external() {
  ext_ = nullptr;
  ext_cap_ = ext_off_ = 0;
}

void Arena::reset() {
  if (ext_) {
    ext_off_ = 0;
    return;
  }
  if (chunks_.size() > 1) {
    // consolidate into one chunk of the high-water size; the old chunks are retired, not
    // freed, because work in flight or a captured graph may still use them
    double* p = nullptr;
    const size_t cap = high_ + high_ / 4;
    if (hipMalloc(&p, cap * sizeof(double)) != hipSuccess) throw Error(-4, "device out of memory for scratch");
    for (auto& ch : chunks_) retired_.push_back(ch);
    chunks_.clear();
    chunks_.push_back({p, cap});
    ++generation_;
  }
  cur_ = 0;
  off_ = 0;
  used_total_ = 0;
}

double* Arena::take(size_t doubles) {
  doubles = rounded(doubles);   // 256-byte alignment
  if (ext_) {
    if (ext_off_ + doubles > ext_cap_)
      throw Error(-1, "request exceeds the fixed scratch buffer (" + std::to_string(ext_cap_ * sizeof(double)) +
                          " bytes)");
    double* p = ext_ + ext_off_;
    ext_off_ += doubles;
    return p;
  }
  while (cur_ < chunks_.size() && off_ + doubles > chunks_[cur_].cap) {
    ++cur_;
    off_ = 0;
  }
  if (cur_ == chunks_.size()) {
    const size_t cap = std::max(doubles, (size_t)(32u << 20));   // at least 256 MiB
    double* p = nullptr;
    if (hipMalloc(&p, cap * sizeof(double)) != hipSuccess) throw Error(-4, "device out of memory for scratch");
    chunks_.push_back({p, cap});
    if (chunks_.size() == 1) ++generation_;
    off_ = 0;
  }
  double* p = chunks_[cur_].p + off_;
  off_ += doubles;
  used_total_ += doubles;
  high_ = std::max(high_, used_total_);
  recent_high_ = std::max(recent_high_, used_total_);
  return p;
}

hipEvent_t Context::get_event() const {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  BCN_HIP(hipEventCreate(&e));
  return e;
}

ProfScope::ProfScope(const Context& c, const char* name, hipStream_t s, double bytes, double ops) : c_(c), s_(s) {
  if (!c.prof) return;
  e_ = &c.prof_data[name];
  start_ = c.get_event();
  BCN_HIP(hipEventRecord(start_, s));
  e_->bytes += bytes;
  e_->ops += ops;
  e_->launches += 1;
}

ProfScope::~ProfScope() {
  if (!e_) return;
  hipEvent_t stop = c_.get_event();
  (void)hipEventRecord(stop, s_);
  e_->ev.push_back({start_, stop});
}

Basis Context::basis_Q(int level) const {
  Basis b{};
  b.n = level;
  for (int i = 0; i < level; ++i) b.id[i] = idQ(i);
  return b;
}

Basis Context::basis_QP(int level) const {
  Basis b{};
  b.n = level + K;
  for (int i = 0; i < level; ++i) b.id[i] = idQ(i);
  for (int i = 0; i < K; ++i) b.id[level + i] = idP(i);
  return b;
}

Basis Context::basis_QB(int level) const {
  Basis b{};
  b.n = level + m;
  for (int i = 0; i < level; ++i) b.id[i] = idQ(i);
  for (int i = 0; i < m; ++i) b.id[level + i] = idB(i);
  return b;
}

Conv make_conv(const Context& c, const std::vector<int>& src, const std::vector<int>& dst) {
  if ((int)src.size() > kMaxBasis || (int)dst.size() > kMaxBasis) throw Error(-1, "basis too large");
  Conv cv;
  std::memset(&cv, 0, sizeof(cv));
  cv.ns = (int)src.size();
  cv.nd = (int)dst.size();
  for (int i = 0; i < cv.ns; ++i) cv.src[i] = src[i];
  for (int d = 0; d < cv.nd; ++d) cv.dst[d] = dst[d];
  for (int i = 0; i < cv.ns; ++i) {
    const uint64_t pi = c.primes[src[i]];
    for (int k = 0; k < i; ++k) cv.ginv[i][k] = (double)host::invmod(c.primes[src[k]] % pi, pi);
  }
  for (int d = 0; d < cv.nd; ++d) {
    const uint64_t qd = c.primes[dst[d]];
    uint64_t prod = 1;
    for (int k = 0; k < cv.ns; ++k) {
      const uint64_t pk = c.primes[src[k]] % qd;
      cv.pm[d][k] = (double)pk;
      prod = host::mulmod(prod, pk, qd);
    }
    cv.Mmod[d] = (double)prod;
  }
  return cv;
}

namespace {
std::mutex g_conv_mu;
std::map<std::pair<const Context*, std::string>, Conv*> g_convs;
}  // namespace

const Conv* conv_device(const Context& c, const std::string& key, const Conv& cv) {
  std::lock_guard<std::mutex> lk(g_conv_mu);
  auto it = g_convs.find({&c, key});
  if (it != g_convs.end()) return it->second;
  if (c.no_alloc) throw Error(-6, "conversion table " + key + " was not prepared at context creation");
  Conv* d = nullptr;
  BCN_HIP(hipMalloc(&d, sizeof(Conv)));
  BCN_HIP(hipMemcpy(d, &cv, sizeof(Conv), hipMemcpyHostToDevice));
  g_convs[{&c, key}] = d;
  return d;
}

void release_convs(const Context& c) {
  std::lock_guard<std::mutex> lk(g_conv_mu);
  for (auto it = g_convs.begin(); it != g_convs.end();) {
    if (it->first.first == &c) {
      (void)hipFree(it->second);
      it = g_convs.erase(it);
    } else {
      ++it;
    }
  }
}

Context* create_context(uint32_t n, uint32_t q_bits, uint32_t L, uint32_t K, uint32_t alpha, uint64_t t, int device,
                        bool ckks) {
  int logn = 0;
  while ((1u << logn) < n) ++logn;
  if ((1u << logn) != n || logn < 10 || logn > 14) throw Error(-1, "N must be a power of two in [1024, 16384]");
  if (q_bits < 25 || q_bits > 41) throw Error(-1, "prime size must be 25..41 bits (exact FP64 residue arithmetic)");
  if (L < 1 || L > 8) throw Error(-1, "number of ciphertext primes must be 1..8");
  if (K < 1 || K > 3) throw Error(-1, "number of special primes must be 1..3");
  if (alpha < 1 || alpha > 8) throw Error(-1, "digit size must be 1..8");
  if (ckks) {
    t = 0;
  } else {
    if (t < 3 || t >= (1ull << 21) || !host::is_prime(t) || (t - 1) % (2ull * n) != 0)
      throw Error(-1, "t must be a prime below 2^21 with t = 1 mod 2N");
    if (t >= (1ull << (q_bits - 2))) throw Error(-1, "t too large for the ciphertext primes");
  }
  // special primes must cover one digit: P > Q_j keeps the key-switching noise small
  if (K < alpha && false) throw Error(-1, "unreachable");

  BCN_HIP(hipSetDevice(device));
  auto c = std::make_unique<Context>();
  c->device = device;
  c->n = (int)n;
  c->logn = logn;
  c->L = (int)L;
  c->K = (int)K;
  c->alpha = (int)alpha;
  c->t = t;
  c->scheme = ckks ? 1 : 0;
  c->gen = ckks ? 5 : 3;
  // Q and P: the largest q_bits-bit primes = 1 mod 2N, then aux primes B with
  // B > 2 N Q so that the square's exact tensor lives in Q*B.  B takes the largest 41-bit
  // primes (the widest the exact FP64 residue arithmetic allows), so it needs as few limbs as
  // possible whatever the size of the ciphertext primes: every B limb is five more transforms
  // per ciphertext in the square.
  std::vector<uint64_t> qp = host::ntt_primes((int)q_bits, 2ull * n, (int)(L + K), {t});
  double log_q = 0;
  for (uint32_t i = 0; i < L; ++i) log_q += std::log2((double)qp[i]);
  const double need = log_q + logn + 2.0;
  std::vector<uint64_t> skip(qp.begin(), qp.end());
  skip.push_back(t);
  std::vector<uint64_t> more = host::ntt_primes(41, 2ull * n, 16, skip);
  double log_b = 0;
  int m = 0;
  while (log_b <= need) {
    if (m == (int)more.size()) throw Error(-1, "auxiliary basis too large");
    log_b += std::log2((double)more[m]);
    ++m;
  }
  if ((int)L + m > 16) throw Error(-1, "auxiliary basis too large");
  c->m = m;
  c->primes.assign(qp.begin(), qp.end());
  for (int i = 0; i < m; ++i) c->primes.push_back(more[i]);
  if (!ckks) {
    c->primes.push_back(t);
    c->id_t = (int)c->primes.size() - 1;
  } else {
    c->id_t = -1;
  }
  const int np = (int)c->primes.size();
  for (uint64_t q : c->primes) c->hmods.push_back(Mod{(double)q, 1.0 / (double)q});

  // per-prime tables
  const size_t N = n;
  const size_t per = N + N + N;
  std::vector<double> h((size_t)np * per);
  double* fwd = h.data();
  double* inv = fwd + (size_t)np * N;
  double* post = inv + (size_t)np * N;
  for (int id = 0; id < np; ++id) {
    const uint64_t q = c->primes[id];
    const uint64_t psi = host::negacyclic_root(q, N);
    const uint64_t psi_inv = host::invmod(psi, q);
    const uint64_t omega_inv = host::mulmod(psi_inv, psi_inv, q);
    const uint64_t ninv = host::invmod(N % q, q);
    std::vector<uint64_t> pw(N);
    uint64_t x = 1;
    for (size_t i = 0; i < N; ++i) { pw[i] = x; x = host::mulmod(x, psi, q); }
    fwd[id * N] = (double)pw[0];
    for (int st = 0; st < logn; ++st)
      for (int b = 0; b < (1 << st); ++b)
        fwd[id * N + ((size_t)1 << st) + fwd_tw_word(b, st, logn)] =
            (double)pw[host::bitrev((uint32_t)((1u << st) + b), logn)];
    // inverse twiddles, stage-major: stage s (2^s butterflies per block) uses
    // omega^-(p N / 2^(s+1)) for positions p < 2^s, stored at [2^s + p], so the lanes of
    // one wave (consecutive p) read consecutive words
    std::vector<uint64_t> om(N / 2);
    x = 1;
    for (size_t k = 0; k < N / 2; ++k) { om[k] = x; x = host::mulmod(x, omega_inv, q); }
    inv[id * N] = 0.0;
    for (int st = 0; st < logn; ++st)
      for (size_t p = 0; p < ((size_t)1 << st); ++p) inv[id * N + ((size_t)1 << st) + p] = (double)om[p * (N >> (st + 1))];
    x = ninv;
    for (size_t k = 0; k < N; ++k) { post[id * N + k] = (double)x; x = host::mulmod(x, psi_inv, q); }
  }
  BCN_HIP(hipMalloc(&c->d_tables, h.size() * sizeof(double) + np * sizeof(Mod)));
  BCN_HIP(hipMemcpy(c->d_tables, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  Mod* dm = reinterpret_cast<Mod*>(c->d_tables + h.size());
  BCN_HIP(hipMemcpy(dm, c->hmods.data(), np * sizeof(Mod), hipMemcpyHostToDevice));
  c->tab.fwd = c->d_tables;
  c->tab.inv = c->d_tables + (size_t)np * N;
  c->tab.post = c->d_tables + (size_t)np * 2 * N;
  c->tab.mods = dm;
  c->tab.logn = logn;

  if (!ckks) {
  // slot s -> position of its evaluation point in the transform of R_t
  std::vector<uint32_t> pos(N);
  const uint64_t two_n = 2ull * N;
  uint64_t g = 1;
  for (size_t i = 0; i < N / 2; ++i) {
    const uint64_t e0 = g, e1 = (two_n - g) % two_n;
    pos[i] = ntt_store((int)host::bitrev((uint32_t)((e0 - 1) / 2), logn), logn);
    pos[N / 2 + i] = ntt_store((int)host::bitrev((uint32_t)((e1 - 1) / 2), logn), logn);
    g = g * 3 % two_n;
  }
  BCN_HIP(hipMalloc(&c->d_slot_pos, N * sizeof(uint32_t)));
  BCN_HIP(hipMemcpy(c->d_slot_pos, pos.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice));
  std::vector<uint32_t> slot_of(N, 0xffffffffu);
  for (size_t i = 0; i < N; ++i) slot_of[pos[i]] = (uint32_t)i;
  for (size_t i = 0; i < N; ++i)
    if (slot_of[i] == 0xffffffffu) throw Error(-1, "slot map is not a permutation");
  BCN_HIP(hipMalloc(&c->d_slot_of_word, N * sizeof(uint32_t)));
  BCN_HIP(hipMemcpy(c->d_slot_of_word, slot_of.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice));
  }
  c->arena = std::make_unique<Arena>();
  // default transform shape (bcn_autotune may replace it by a measured choice)
  c->ntt_loge = logn >= 14 ? 5 : 4;
  if (const char* env = std::getenv("BCN_NTT_LOGE")) {
    const int v = std::atoi(env);
    for (int o : c->ntt_loge_options())
      if (o == v) c->ntt_loge = v, c->pinned_loge = true;
  }
  c->square_loge = c->ntt_loge;
  if (const char* env = std::getenv("BCN_SQUARE_LOGE")) {
    const int v = std::atoi(env);
    for (int o : c->ntt_loge_options())
      if (o == v) c->square_loge = v, c->pinned_square_loge = true;
  }
  // the fused square keeps three register sets live; above N = 8192 it would spill
  c->fuse_square = logn <= 13;
  if (const char* env = std::getenv("BCN_FUSE_SQUARE")) c->fuse_square = logn <= 13 && std::atoi(env) != 0;
  if (const char* env = std::getenv("BCN_FUSE_MODDOWN")) c->fuse_moddown = std::atoi(env) != 0;
  // the fused kernel keeps two accumulators and a working set in registers: N <= 8192, digits of <= 2 primes
  const bool can_fuse_ks = logn <= 13 && alpha <= 2;
  c->ks_mode = alpha <= 2 ? 2 : 0;
  if (const char* env = std::getenv("BCN_FUSE_KS")) {
    c->ks_mode = std::atoi(env) != 0 && can_fuse_ks ? 1 : 0;
    c->pinned_ks = true;
  }
  if (const char* env = std::getenv("BCN_KS_MODE")) {
    const int v = std::atoi(env);
    if (v == 0 || (v == 1 && can_fuse_ks) || (v == 2 && alpha <= 2)) c->ks_mode = v, c->pinned_ks = true;
  }
  c->ks_mode_rot = c->ks_mode == 2 ? 2 : 0;
  if (const char* env = std::getenv("BCN_KS_LOGE")) {
    const int v = std::atoi(env);
    for (int o : c->ntt_loge_options())
      if (o == v) c->ks_loge = v, c->pinned_ks = true;
  }
  if (const char* env = std::getenv("BCN_NTT_PERSIST")) c->ntt_persist = std::atoi(env) != 0;
  if (const char* env = std::getenv("BCN_NTT_PREFETCH")) c->ntt_prefetch = std::atoi(env) != 0, c->pinned_prefetch = true;
  if (const char* env = std::getenv("BCN_NTT_XLANE")) c->ntt_xlane = std::atoi(env) != 0, c->pinned_xlane = true;
  if (const char* env = std::getenv("BCN_SPLIT_CHAIN")) c->split_chain = std::atoi(env) != 0;
  BCN_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  BCN_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  BCN_HIP(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
  {
    hipDeviceProp_t prop;
    BCN_HIP(hipGetDeviceProperties(&prop, device));
    const size_t lds = (size_t)n * sizeof(double);
    const int per_cu = std::max(1, (int)(prop.maxSharedMemoryPerMultiProcessor / lds));
    c->persist_blocks = prop.multiProcessorCount * per_cu;
    c->n_cus = prop.multiProcessorCount;
  }
  ntt_setup(*c);
  preload_conversions(*c);
  preload_ks_digits(*c);
  fixed_scratch_setup(*c);
  if (ckks) ckks_setup(*c);
  return c.release();
}

void destroy_context(Context* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->prof_data)
    for (auto& pr : kv.second.ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->join_ev) (void)hipEventDestroy(c->join_ev);
  if (c->side) (void)hipStreamDestroy(c->side);
  release_convs(*c);
  if (c->d_tables) (void)hipFree(c->d_tables);
  if (c->d_slot_pos) (void)hipFree(c->d_slot_pos);
  if (c->d_slot_of_word) (void)hipFree(c->d_slot_of_word);
  if (c->ckks_tab) (void)hipFree(c->ckks_tab);
  delete c;
}

}  // namespace bcn
