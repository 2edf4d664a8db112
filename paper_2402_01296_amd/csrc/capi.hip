// extern "C" entry points: argument checks, error translation, arena reset.
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/bcn.h"
#include "layers.h"
#include "sampler.h"

struct bcn_context { bcn::Context* c; };
struct bcn_secret_key { bcn::SecretKey* k; };
struct bcn_eval_keys { bcn::EvalKeys* k; };
struct bcn_layer { bcn::Layer* l; };

namespace bcn {
Context* create_context(uint32_t n, uint32_t q_bits, uint32_t L, uint32_t K, uint32_t alpha, uint64_t t, int device,
                        bool ckks);
void destroy_context(Context* c);
}  // namespace bcn

namespace {
thread_local std::string g_err;

template <typename F>
int guard(F&& f) {
  try {
    f();
    return BCN_OK;
  } catch (const bcn::Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host out of memory";
    return BCN_ERR_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return BCN_ERR_INTERNAL;
  }
}

bcn::Context& ctxof(bcn_context* c) {
  if (!c || !c->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
  bcn::Context& x = *c->c;
  BCN_HIP(hipSetDevice(x.device));
  x.arena->reset();
  return x;
}

void check_level(const bcn::Context& c, int level) {
  if (level < 1 || level > c.L) throw bcn::Error(BCN_ERR_LEVEL, "level out of range");
}

void check_n(int n) {
  if (n < 0) throw bcn::Error(BCN_ERR_INVALID, "negative count");
}

void check_ptr(const void* p, const char* what) {
  if (!p) throw bcn::Error(BCN_ERR_INVALID, std::string("null pointer: ") + what);
}

void need_scheme(const bcn::Context& c, int scheme) {
  if (c.scheme != scheme)
    throw bcn::Error(BCN_ERR_INVALID, scheme ? "a CKKS operation needs a CKKS context"
                                             : "a BFV operation needs a BFV context (this one is CKKS)");
}
// a [n][level][N] and e [n][N] of encryptions first .. first + n - 1
void encryption_randomness(const bcn::Context& c, uint64_t seed, uint64_t first, int n, int level,
                           std::vector<uint64_t>& a, std::vector<int8_t>& e) {
  if (first + (uint64_t)n > (1ull << 32)) throw bcn::Error(BCN_ERR_INVALID, "encryption index beyond 2^32");
  a.resize((size_t)n * level * c.n);
  e.resize((size_t)n * c.n);
  std::vector<int64_t> tmp(c.n);
  for (int r = 0; r < n; ++r) {
    const uint64_t id = (first + (uint64_t)r) << 32;
    for (int i = 0; i < level; ++i) {
      bcn::Stream st(seed, bcn::kPurposeEncA, id | (uint64_t)i);
      bcn::sample_uniform(st, c.primes[i], c.n, a.data() + ((size_t)r * level + i) * c.n);
    }
    bcn::Stream st(seed, bcn::kPurposeEncE, id);
    bcn::sample_gaussian(st, c.n, tmp.data());
    for (int k = 0; k < c.n; ++k) e[(size_t)r * c.n + k] = (int8_t)tmp[k];
  }
}
}  // namespace

extern "C" {

const char* bcn_last_error(void) { return g_err.c_str(); }

int bcn_context_create(const bcn_params* p, int hip_device, bcn_context** out) {
  return guard([&] {
    check_ptr(p, "params");
    check_ptr(out, "out");
    auto* h = new bcn_context{nullptr};
    try {
      h->c = bcn::create_context(p->n, p->q_bits, p->L, p->K, p->alpha, p->t, hip_device, false);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

void bcn_context_destroy(bcn_context* ctx) {
  if (!ctx) return;
  bcn::destroy_context(ctx->c);
  delete ctx;
}

int bcn_context_primes(const bcn_context* ctx, uint64_t* out, int cap, int* n_q, int* n_p, int* n_aux) {
  return guard([&] {
    if (!ctx || !ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
    const bcn::Context& c = *ctx->c;
    const int total = (int)c.primes.size();
    for (int i = 0; i < total && i < cap; ++i) out[i] = c.primes[i];
    if (n_q) *n_q = c.L;
    if (n_p) *n_p = c.K;
    if (n_aux) *n_aux = c.m;
  });
}

int bcn_secret_key_create(bcn_context* ctx, const int8_t* s, bcn_secret_key** out) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(s, "s");
    check_ptr(out, "out");
    *out = new bcn_secret_key{bcn::secret_key_create(c, s)};
  });
}

void bcn_secret_key_destroy(bcn_secret_key* sk) {
  if (!sk) return;
  delete sk->k;
  delete sk;
}

int bcn_eval_keys_create(bcn_context* ctx, bcn_eval_keys** out) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(out, "out");
    auto* k = new bcn::EvalKeys();
    k->ctx = &c;
    *out = new bcn_eval_keys{k};
  });
}

void bcn_eval_keys_destroy(bcn_eval_keys* ek) {
  if (!ek) return;
  delete ek->k;
  delete ek;
}

int bcn_keygen(bcn_context* ctx, const bcn_secret_key* sk, bcn_eval_keys* ek, int kind, int step, const uint64_t* a,
               const int8_t* e, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(sk, "secret key");
    check_ptr(ek, "eval keys");
    check_ptr(a, "a");
    check_ptr(e, "e");
    if (kind != BCN_KEY_RELIN && kind != BCN_KEY_ROTATION) throw bcn::Error(BCN_ERR_INVALID, "bad key kind");
    if (kind == BCN_KEY_ROTATION && (step == 0 || step <= -c.n / 2 || step >= c.n / 2))
      throw bcn::Error(BCN_ERR_INVALID, "rotation step must be nonzero in (-N/2, N/2)");
    bcn::keygen(c, *sk->k, *ek->k, kind, step, a, e, (hipStream_t)stream);
  });
}

int bcn_eval_key_export(bcn_context* ctx, const bcn_eval_keys* ek, int kind, int step, uint64_t* out,
                        bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(ek, "eval keys");
    check_ptr(out, "out");
    const double* key = kind == BCN_KEY_RELIN ? ek->k->relin : ek->k->rot_key(step);
    if (!key) throw bcn::Error(BCN_ERR_KEY, "missing relinearisation key");
    const bcn::Basis qp = c.basis_QP(c.L);
    const size_t words = ek->k->key_doubles();
    hipStream_t s = (hipStream_t)stream;
    double* tmp = c.arena->take(words);
    BCN_HIP(hipMemcpyAsync(tmp, key, words * sizeof(double), hipMemcpyDeviceToDevice, s));
    bcn::ntt_inverse(c, tmp, (int)(words / ((size_t)qp.n * c.n)), qp, s);
    uint64_t* u = reinterpret_cast<uint64_t*>(c.arena->take(words));
    bcn::f64_to_u64(tmp, u, words, s);
    BCN_HIP(hipMemcpyAsync(out, u, words * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    BCN_HIP(hipStreamSynchronize(s));
  });
}

int bcn_encode_encrypt(bcn_context* ctx, const bcn_secret_key* sk, const int64_t* slots, const uint64_t* a,
                       const int8_t* e, int n, int level, double* ct_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_level(c, level);
    check_n(n);
    check_ptr(sk, "secret key");
    if (n == 0) return;
    check_ptr(slots, "slots");
    check_ptr(a, "a");
    check_ptr(e, "e");
    check_ptr(ct_out, "ct_out");
    bcn::encrypt(c, *sk->k, slots, a, e, n, level, ct_out, (hipStream_t)stream);
  });
}

int bcn_decrypt_decode(bcn_context* ctx, const bcn_secret_key* sk, const double* ct, int n, int level,
                       int64_t* slots_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_level(c, level);
    check_n(n);
    check_ptr(sk, "secret key");
    if (n == 0) return;
    check_ptr(ct, "ct");
    check_ptr(slots_out, "slots_out");
    bcn::decrypt(c, *sk->k, ct, n, level, slots_out, (hipStream_t)stream);
  });
}

int bcn_sample(int kind, uint64_t seed, uint32_t purpose, uint64_t index, uint64_t q, int n, int64_t* out) {
  return guard([&] {
    check_n(n);
    if (n == 0) return;
    check_ptr(out, "out");
    bcn::Stream st(seed, purpose, index);
    if (kind == BCN_SAMPLE_TERNARY) {
      bcn::sample_ternary(st, n, out);
    } else if (kind == BCN_SAMPLE_GAUSSIAN) {
      bcn::sample_gaussian(st, n, out);
    } else if (kind == BCN_SAMPLE_UNIFORM) {
      if (q < 2 || q > (1ull << 62)) throw bcn::Error(BCN_ERR_INVALID, "uniform modulus must be in [2, 2^62]");
      bcn::sample_uniform(st, q, n, reinterpret_cast<uint64_t*>(out));
    } else {
      throw bcn::Error(BCN_ERR_INVALID, "bad sample kind");
    }
  });
}

int bcn_gaussian_table(uint64_t* out) {
  return guard([&] {
    check_ptr(out, "out");
    const std::vector<uint64_t>& t = bcn::cdt_table();
    std::memcpy(out, t.data(), t.size() * sizeof(uint64_t));
  });
}

int bcn_secret_key_generate(bcn_context* ctx, uint64_t seed, bcn_secret_key** out) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(out, "out");
    std::vector<int64_t> v(c.n);
    bcn::Stream st(seed, bcn::kPurposeSecret, 0);
    bcn::sample_ternary(st, c.n, v.data());
    std::vector<int8_t> s(v.begin(), v.end());
    *out = new bcn_secret_key{bcn::secret_key_create(c, s.data())};
  });
}

int bcn_keygen_seeded(bcn_context* ctx, const bcn_secret_key* sk, bcn_eval_keys* ek, int kind, int step,
                      uint64_t seed, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(sk, "secret key");
    check_ptr(ek, "eval keys");
    if (kind != BCN_KEY_RELIN && kind != BCN_KEY_ROTATION) throw bcn::Error(BCN_ERR_INVALID, "bad key kind");
    if (kind == BCN_KEY_ROTATION && (step == 0 || step <= -c.n / 2 || step >= c.n / 2))
      throw bcn::Error(BCN_ERR_INVALID, "rotation step must be nonzero in (-N/2, N/2)");
    const uint64_t key = kind == BCN_KEY_RELIN ? 0 : (uint64_t)bcn::galois_element(c, step);
    const int dnum = c.dnum(c.L), width = c.L + c.K;
    std::vector<uint64_t> a((size_t)dnum * width * c.n);
    std::vector<int8_t> e((size_t)dnum * c.n);
    std::vector<int64_t> tmp(c.n);
    for (int j = 0; j < dnum; ++j) {
      for (int i = 0; i < width; ++i) {
        bcn::Stream st(seed, bcn::kPurposeKskA, (key << 32) | (uint64_t)(j * width + i));
        bcn::sample_uniform(st, c.primes[i], c.n, a.data() + ((size_t)j * width + i) * c.n);
      }
      bcn::Stream st(seed, bcn::kPurposeKskE, (key << 32) | (uint64_t)j);
      bcn::sample_gaussian(st, c.n, tmp.data());
      for (int k = 0; k < c.n; ++k) e[(size_t)j * c.n + k] = (int8_t)tmp[k];
    }
    bcn::keygen(c, *sk->k, *ek->k, kind, step, a.data(), e.data(), (hipStream_t)stream);
  });
}


int bcn_encrypt_seeded(bcn_context* ctx, const bcn_secret_key* sk, const int64_t* slots, uint64_t seed,
                       uint64_t first, int n, int level, double* ct_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_level(c, level);
    check_n(n);
    check_ptr(sk, "secret key");
    if (n == 0) return;
    check_ptr(slots, "slots");
    check_ptr(ct_out, "ct_out");
    std::vector<uint64_t> a;
    std::vector<int8_t> e;
    encryption_randomness(c, seed, first, n, level, a, e);
    bcn::encrypt(c, *sk->k, slots, a.data(), e.data(), n, level, ct_out, (hipStream_t)stream);
  });
}

int bcn_ckks_encrypt_seeded(bcn_context* ctx, const bcn_secret_key* sk, const double* slots, double scale,
                            uint64_t seed, uint64_t first, int n, int level, double* ct_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    check_ptr(sk, "secret key");
    if (n == 0) return;
    check_ptr(slots, "slots");
    check_ptr(ct_out, "ct_out");
    std::vector<uint64_t> a;
    std::vector<int8_t> e;
    encryption_randomness(c, seed, first, n, level, a, e);
    bcn::ckks_encrypt(c, *sk->k, slots, scale, a.data(), e.data(), n, level, ct_out, (hipStream_t)stream);
  });
}

int bcn_ct_export(bcn_context* ctx, const double* ct, int n, int level, uint64_t* host_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(ct, "ct");
    check_ptr(host_out, "host_out");
    const size_t words = (size_t)n * 2 * level * c.n;
    hipStream_t s = (hipStream_t)stream;
    uint64_t* u = reinterpret_cast<uint64_t*>(c.arena->take(words));
    bcn::f64_to_u64(ct, u, words, s);
    BCN_HIP(hipMemcpyAsync(host_out, u, words * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    BCN_HIP(hipStreamSynchronize(s));
  });
}

int bcn_ct_import(bcn_context* ctx, const uint64_t* host_in, int n, int level, double* ct, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(ct, "ct");
    check_ptr(host_in, "host_in");
    const size_t words = (size_t)n * 2 * level * c.n;
    for (int ci = 0; ci < n; ++ci)
      for (int part = 0; part < 2; ++part)
        for (int i = 0; i < level; ++i) {
          const uint64_t q = c.primes[i];
          const uint64_t* row = host_in + (((size_t)ci * 2 + part) * level + i) * c.n;
          for (int k = 0; k < c.n; ++k)
            if (row[k] >= q) throw bcn::Error(BCN_ERR_INVALID, "imported residue not below its prime");
        }
    hipStream_t s = (hipStream_t)stream;
    uint64_t* u = reinterpret_cast<uint64_t*>(c.arena->take(words));
    BCN_HIP(hipMemcpyAsync(u, host_in, words * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    bcn::u64_to_f64(u, ct, words, s);
    BCN_HIP(hipStreamSynchronize(s));
  });
}

int bcn_ntt(bcn_context* ctx, double* data, int n_polys, int n_limbs, int first_prime, int inverse,
            bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_n(n_polys);
    if (n_limbs < 1 || n_limbs > bcn::kMaxBasis) throw bcn::Error(BCN_ERR_INVALID, "bad limb count");
    if (first_prime < 0 || first_prime + n_limbs > (int)c.primes.size())
      throw bcn::Error(BCN_ERR_INVALID, "prime ids out of range");
    if (n_polys == 0) return;
    check_ptr(data, "data");
    bcn::Basis b{};
    b.n = n_limbs;
    for (int i = 0; i < n_limbs; ++i) b.id[i] = first_prime + i;
    if (inverse)
      bcn::ntt_inverse(c, data, n_polys, b, (hipStream_t)stream);
    else
      bcn::ntt_forward(c, data, n_polys, b, (hipStream_t)stream);
  });
}

int bcn_mac(bcn_context* ctx, const double* in, int n_in, double* out, int n_out, int level, const int32_t* w,
            bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_level(c, level);
    if (n_in < 1 || n_out < 0) throw bcn::Error(BCN_ERR_INVALID, "bad MAC shape");
    if (n_out == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    check_ptr(w, "w");
    std::vector<int32_t> W(w, w + (size_t)n_in * n_out);
    int tile = 0;   // automatic
    if (const char* env = std::getenv("BCN_MAC_TILE")) {
      tile = std::atoi(env);
      if (tile < 1 || tile > 64 || (tile & (tile - 1)))
        throw bcn::Error(BCN_ERR_INVALID, "BCN_MAC_TILE must be a power of two in 1..64");
    }
    bcn::MacPlan p = bcn::make_mac_plan(c, W, n_out, n_in, {}, tile);
    try {
      bcn::mac(c, p, in, out, level, (hipStream_t)stream);
      BCN_HIP(hipStreamSynchronize((hipStream_t)stream));
    } catch (...) {
      bcn::free_mac_plan(p);
      throw;
    }
    bcn::free_mac_plan(p);
  });
}

int bcn_add_plain(bcn_context* ctx, double* ct, int n, int level, const int64_t* slots, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(ct, "ct");
    check_ptr(slots, "slots");
    hipStream_t s = (hipStream_t)stream;
    int64_t* sd = reinterpret_cast<int64_t*>(c.arena->take((size_t)n * c.n));
    BCN_HIP(hipMemcpyAsync(sd, slots, (size_t)n * c.n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    double* m = c.arena->take((size_t)n * c.n);
    bcn::encode_device(c, sd, m, n, s);
    bcn::add_delta(c, ct, n, level, m, s);
    BCN_HIP(hipStreamSynchronize(s));
  });
}

int bcn_mul_plain(bcn_context* ctx, const double* in, double* out, int n, int level, const int64_t* slots,
                  bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    check_ptr(slots, "slots");
    hipStream_t s = (hipStream_t)stream;
    double* pt = c.arena->take((size_t)level * c.n);
    bcn::encode_plain_ntt(c, slots, 1, level, pt, s);
    const size_t words = (size_t)n * 2 * level * c.n;
    double* tmp = c.arena->take(words);
    BCN_HIP(hipMemcpyAsync(tmp, in, words * sizeof(double), hipMemcpyDeviceToDevice, s));
    const bcn::Basis q = c.basis_Q(level);
    bcn::ntt_forward(c, tmp, 2 * n, q, s);
    bcn::mul_plain_ntt(c, tmp, tmp, n, level, pt, false, s);
    bcn::ntt_inverse(c, tmp, 2 * n, q, s);
    BCN_HIP(hipMemcpyAsync(out, tmp, words * sizeof(double), hipMemcpyDeviceToDevice, s));
  });
}

int bcn_square_relin(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, double* out, int n, int level,
                     int modswitch, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_level(c, level);
    check_n(n);
    check_ptr(ek, "eval keys");
    if (n == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    bcn::square_relin(c, *ek->k, in, out, n, level, modswitch != 0, (hipStream_t)stream);
  });
}

int bcn_square_relin_noalloc(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, double* out, int n,
                             int level, int modswitch, bcn_stream stream) {
  return guard([&] {
    // no arena reset here: resetting may move the arena to a new block (an allocation)
    if (!ctx || !ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
    bcn::Context& c = *ctx->c;
    need_scheme(c, 0);
    BCN_HIP(hipSetDevice(c.device));
    check_level(c, level);
    check_n(n);
    check_ptr(ek, "eval keys");
    if (n == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    bcn::square_relin_noalloc(c, *ek->k, in, out, n, level, modswitch != 0, (hipStream_t)stream);
  });
}

int bcn_rotate(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, int n_in, int level, const int32_t* steps,
               int n_steps, double* out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_level(c, level);
    check_n(n_in);
    check_ptr(ek, "eval keys");
    if (n_in == 0 || n_steps == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    check_ptr(steps, "steps");
    std::vector<int> st(steps, steps + n_steps);
    for (int x : st) ek->k->rot_key(x);   // throws BCN_ERR_KEY when missing
    bcn::rotate_hoisted(c, *ek->k, in, n_in, level, st, out, (hipStream_t)stream);
  });
}

int bcn_rotate_sum(bcn_context* ctx, const bcn_eval_keys* ek, double* ct, int n, int level, int span,
                   bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_level(c, level);
    check_n(n);
    check_ptr(ek, "eval keys");
    if (span > c.n / 2) throw bcn::Error(BCN_ERR_INVALID, "span beyond the slot row");
    const auto rounds = bcn::rotate_sum_rounds(span);
    if (n == 0) return;
    check_ptr(ct, "ct");
    for (const auto& rs : rounds)
      for (int r : rs) ek->k->rot_key(r);
    bcn::rotate_sum(c, *ek->k, ct, n, level, span, (hipStream_t)stream);
  });
}

int bcn_rotate_sum_steps(int span, int32_t* steps, int cap) {
  int count = 0;
  const int rc = guard([&] {
    const auto rounds = bcn::rotate_sum_rounds(span);
    for (const auto& rs : rounds)
      for (int r : rs) {
        if (steps && count < cap) steps[count] = r;
        ++count;
      }
  });
  return rc == BCN_OK ? count : rc;
}

int bcn_modswitch(bcn_context* ctx, const double* in, double* out, int n, int level, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_level(c, level);
    check_n(n);
    if (level < 2) throw bcn::Error(BCN_ERR_LEVEL, "modulus switch needs two primes");
    if (n == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    bcn::modswitch(c, in, out, n, level, (hipStream_t)stream);
  });
}

int bcn_autotune(bcn_context* ctx, char* report, int cap, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    const std::string r = bcn::autotune_ntt(c, (hipStream_t)stream);
    if (report && cap > 0) {
      std::strncpy(report, r.c_str(), (size_t)cap - 1);
      report[cap - 1] = 0;
    }
  });
}

int bcn_layer_autotune(bcn_context* ctx, bcn_layer* layer, char* report, int cap, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(layer, "layer");
    const std::string r = bcn::autotune_layer_mac(c, *layer->l, (hipStream_t)stream);
    if (report && cap > 0) {
      std::strncpy(report, r.c_str(), (size_t)cap - 1);
      report[cap - 1] = 0;
    }
  });
}

int bcn_profile_enable(bcn_context* ctx, int on) {
  return guard([&] {
    if (!ctx || !ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
    ctx->c->prof = on != 0;
  });
}

int bcn_profile_read(bcn_context* ctx, char* names, int names_cap, int* launches, double* total_ms, double* bytes,
                     double* ops, int cap) {
  int count = 0;
  int rc = guard([&] {
    if (!ctx || !ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
    bcn::Context& c = *ctx->c;
    std::string joined;
    for (auto& kv : c.prof_data) {
      double ms = 0;
      for (auto& pr : kv.second.ev) {
        BCN_HIP(hipEventSynchronize(pr.second));
        float x = 0;
        BCN_HIP(hipEventElapsedTime(&x, pr.first, pr.second));
        ms += x;
        c.event_pool.push_back(pr.first);
        c.event_pool.push_back(pr.second);
      }
      if (count < cap) {
        launches[count] = (int)kv.second.launches;
        total_ms[count] = ms;
        bytes[count] = kv.second.bytes;
        if (ops) ops[count] = kv.second.ops;
      }
      joined += kv.first + "\n";
      ++count;
    }
    c.prof_data.clear();
    if (names && names_cap > 0) {
      std::strncpy(names, joined.c_str(), (size_t)names_cap - 1);
      names[names_cap - 1] = 0;
    }
  });
  return rc < 0 ? rc : count;
}

int bcn_layer_create(bcn_context* ctx, const bcn_layer_desc* desc, int level, bcn_layer** out) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 0);
    check_ptr(desc, "desc");
    check_ptr(out, "out");
    *out = new bcn_layer{bcn::layer_create(c, *desc, level)};
  });
}

void bcn_layer_destroy(bcn_layer* layer) {
  if (!layer) return;
  delete layer->l;
  delete layer;
}

int bcn_layer_rotation_steps(const bcn_layer* layer, int32_t* steps, int cap) {
  if (!layer || !layer->l) {
    g_err = "null layer";
    return BCN_ERR_INVALID;
  }
  const auto& v = layer->l->all_steps;
  for (int i = 0; i < (int)v.size() && i < cap; ++i) steps[i] = v[i];
  return (int)v.size();
}

int bcn_layer_shape(const bcn_layer* layer, int* n_in, int* n_out, int* level_out) {
  if (!layer || !layer->l) {
    g_err = "null layer";
    return BCN_ERR_INVALID;
  }
  if (n_in) *n_in = layer->l->n_in;
  if (n_out) *n_out = layer->l->n_out;
  if (level_out) *level_out = layer->l->level_out;
  return BCN_OK;
}

int bcn_layer_parts(const bcn_layer* layer, int* in_parts, int* out_parts) {
  if (!layer || !layer->l) {
    g_err = "null layer";
    return BCN_ERR_INVALID;
  }
  if (in_parts) *in_parts = layer->l->in_parts;
  if (out_parts) *out_parts = layer->l->defer ? 3 : 2;
  return BCN_OK;
}

int bcn_layer_eval(bcn_context* ctx, const bcn_eval_keys* ek, const bcn_layer* layer, const double* in, double* out,
                   const float* features, bcn_stream stream) {
  return bcn_layer_eval_batch(ctx, ek, layer, in, out, features, 1, stream);
}

int bcn_layer_eval_batch(bcn_context* ctx, const bcn_eval_keys* ek, const bcn_layer* layer, const double* in,
                         double* out, const float* features, int n_requests, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    check_ptr(ek, "eval keys");
    check_ptr(layer, "layer");
    if (n_requests < 0) throw bcn::Error(BCN_ERR_INVALID, "negative request count");
    if (n_requests == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    const bcn::Layer& L = *layer->l;
    if ((L.square || L.in_parts == 3) && !ek->k->relin) throw bcn::Error(BCN_ERR_KEY, "missing relinearisation key");
    for (int st : L.all_steps) ek->k->rot_key(st);
    bcn::layer_eval(c, *ek->k, L, in, out, features, (hipStream_t)stream, n_requests);
  });
}

int bcn_scratch_info(bcn_context* ctx, uint64_t* base, uint64_t* generation, size_t* bytes, size_t* high_bytes,
                     size_t* retired_bytes) {
  return guard([&] {
    if (!ctx || !ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
    bcn::Arena& a = *ctx->c->arena;
    if (base) *base = (uint64_t)(uintptr_t)a.base();
    if (generation) *generation = a.generation();
    if (bytes) *bytes = a.capacity();
    const size_t recent = a.take_recent_high();
    if (high_bytes) *high_bytes = recent;
    if (retired_bytes) *retired_bytes = a.retired_bytes();
  });
}

int bcn_scratch_release(bcn_context* ctx) {
  return guard([&] {
    if (!ctx || !ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context");
    BCN_HIP(hipSetDevice(ctx->c->device));
    ctx->c->arena->release_retired();
  });
}

int bcn_ntt_multi(const bcn_ntt_item* items, int n_items, int inverse, bcn_stream stream) {
  return guard([&] {
    if (n_items < 0 || n_items > bcn::kMaxMultiItems) throw bcn::Error(BCN_ERR_INVALID, "1..16 items per launch");
    if (n_items == 0) return;
    check_ptr(items, "items");
    std::vector<bcn::MultiNttItem> v;
    int device = -1;
    for (int i = 0; i < n_items; ++i) {
      const bcn_ntt_item& it = items[i];
      if (!it.ctx || !it.ctx->c) throw bcn::Error(BCN_ERR_INVALID, "null context in a transform item");
      const bcn::Context& c = *it.ctx->c;
      if (device < 0) device = c.device;
      if (c.device != device) throw bcn::Error(BCN_ERR_INVALID, "transform items on different devices");
      if (it.n_polys < 0 || it.n_limbs < 1 || it.first_prime < 0 ||
          it.first_prime + it.n_limbs > (int)c.primes.size())
        throw bcn::Error(BCN_ERR_INVALID, "bad transform item shape");
      if (it.n_polys > 0) check_ptr(it.data, "item data");
      v.push_back({it.data, c.tab, c.logn, it.n_limbs, it.first_prime, it.n_polys * it.n_limbs});
    }
    BCN_HIP(hipSetDevice(device));
    bcn::ntt_multi(v, inverse != 0, (hipStream_t)stream);
  });
}

// ---- CKKS

int bcn_context_create_ckks(const bcn_params* p, int hip_device, bcn_context** out) {
  return guard([&] {
    check_ptr(p, "params");
    check_ptr(out, "out");
    auto* h = new bcn_context{nullptr};
    try {
      h->c = bcn::create_context(p->n, p->q_bits, p->L, p->K, p->alpha, 0, hip_device, true);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

int bcn_ckks_encode(bcn_context* ctx, const double* slots, int n, int level, double scale, int ntt_domain, double* out,
                    bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(slots, "slots");
    check_ptr(out, "out");
    bcn::ckks_encode(c, slots, n, level, scale, ntt_domain != 0, out, (hipStream_t)stream);
  });
}

int bcn_ckks_encode_encrypt(bcn_context* ctx, const bcn_secret_key* sk, const double* slots, double scale,
                            const uint64_t* a, const int8_t* e, int n, int level, double* ct_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    check_ptr(sk, "secret key");
    if (n == 0) return;
    check_ptr(slots, "slots");
    check_ptr(a, "a");
    check_ptr(e, "e");
    check_ptr(ct_out, "ct_out");
    bcn::ckks_encrypt(c, *sk->k, slots, scale, a, e, n, level, ct_out, (hipStream_t)stream);
  });
}

int bcn_ckks_decrypt_decode(bcn_context* ctx, const bcn_secret_key* sk, const double* ct, int n, int level,
                            double scale, double* slots_out, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    check_ptr(sk, "secret key");
    if (n == 0) return;
    check_ptr(ct, "ct");
    check_ptr(slots_out, "slots_out");
    if (!(scale > 0.0)) throw bcn::Error(BCN_ERR_INVALID, "scale must be positive");
    bcn::ckks_decrypt(c, *sk->k, ct, n, level, scale, slots_out, (hipStream_t)stream);
  });
}

int bcn_ckks_add_plain(bcn_context* ctx, double* ct, int n, int level, const double* pt, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(ct, "ct");
    check_ptr(pt, "pt");
    bcn::ckks_add_plain(c, ct, n, level, pt, (hipStream_t)stream);
  });
}

int bcn_ckks_mul_plain(bcn_context* ctx, const double* in, double* out, int n, int level, const double* pt_ntt,
                       bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    if (n == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    check_ptr(pt_ntt, "pt");
    const size_t words = (size_t)n * 2 * level * c.n;
    double* A = c.arena->take(words);
    bcn::copy_rows(in, 0, A, 0, words, 1, (hipStream_t)stream);
    bcn::ntt_forward(c, A, 2 * n, c.basis_Q(level), (hipStream_t)stream);
    bcn::mul_plain_ntt(c, A, A, n, level, pt_ntt, false, (hipStream_t)stream);
    bcn::ntt_inverse(c, A, 2 * n, c.basis_Q(level), (hipStream_t)stream);
    bcn::copy_rows(A, 0, out, 0, words, 1, (hipStream_t)stream);
  });
}

int bcn_ckks_square_relin_rescale(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, double* out, int n,
                                  int level, bcn_stream stream) {
  return guard([&] {
    bcn::Context& c = ctxof(ctx);
    need_scheme(c, 1);
    check_level(c, level);
    check_n(n);
    check_ptr(ek, "eval keys");
    if (n == 0) return;
    check_ptr(in, "in");
    check_ptr(out, "out");
    bcn::ckks_square_relin_rescale(c, *ek->k, in, out, n, level, (hipStream_t)stream);
  });
}

}  // extern "C"
