// Scheme operations: keys, E / D, square + relinearisation, rotations.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "scheme.h"

namespace bcn {

namespace {
template <typename T>
T* dev_upload(const T* host, size_t count, hipStream_t s, Arena& ar) {
  T* d = reinterpret_cast<T*>(ar.take((count * sizeof(T) + sizeof(double) - 1) / sizeof(double)));
  BCN_HIP(hipMemcpyAsync(d, host, count * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

Basis basis_t(const Context& c) {
  Basis b{};
  b.n = 1;
  b.id[0] = c.id_t;
  return b;
}
}  // namespace

SecretKey::~SecretKey() {
  if (s_hat) (void)hipFree(s_hat);
  if (s_coef) (void)hipFree(s_coef);
}

EvalKeys::~EvalKeys() {
  if (relin) (void)hipFree(relin);
  for (auto& kv : rot) (void)hipFree(kv.second);
  for (auto& kv : tables) {
    (void)hipFree(kv.second.keys);
    (void)hipFree(kv.second.galois);
    (void)hipFree(kv.second.kinv);
  }
}

size_t EvalKeys::key_doubles() const {
  return (size_t)ctx->dnum(ctx->L) * 2 * (ctx->L + ctx->K) * ctx->n;
}

const double* EvalKeys::rot_key(int step) const {
  auto it = rot.find(step);
  if (it == rot.end()) throw Error(-3, "missing rotation key for step " + std::to_string(step));
  return it->second;
}

int galois_element(const Context& c, int step) {
  const uint64_t half = (uint64_t)c.n / 2, two_n = 2ull * c.n;
  const uint64_t r = (uint64_t)(((int64_t)step % (int64_t)half + (int64_t)half) % (int64_t)half);
  return (int)host::powmod((uint64_t)c.gen, r, two_n);
}

int galois_inverse(const Context& c, int k) { return (int)host::inv_pow2((uint64_t)k, c.logn + 1); }

const KeyTable& EvalKeys::table(const std::vector<int>& steps) {
  auto it = tables.find(steps);
  if (it != tables.end()) return it->second;
  std::vector<const double*> kp;
  std::vector<int> g, gi;
  for (int st : steps) {
    kp.push_back(rot_key(st));
    g.push_back(galois_element(*ctx, st));
    gi.push_back(galois_inverse(*ctx, g.back()));
  }
  KeyTable t;
  t.nk = (int)steps.size();
  BCN_HIP(hipMalloc(&t.keys, kp.size() * sizeof(double*)));
  BCN_HIP(hipMalloc(&t.galois, g.size() * sizeof(int)));
  BCN_HIP(hipMalloc(&t.kinv, gi.size() * sizeof(int)));
  BCN_HIP(hipMemcpy(t.keys, kp.data(), kp.size() * sizeof(double*), hipMemcpyHostToDevice));
  BCN_HIP(hipMemcpy(t.galois, g.data(), g.size() * sizeof(int), hipMemcpyHostToDevice));
  BCN_HIP(hipMemcpy(t.kinv, gi.data(), gi.size() * sizeof(int), hipMemcpyHostToDevice));
  return tables.emplace(steps, t).first->second;
}

SecretKey* secret_key_create(Context& c, const int8_t* s_host) {
  for (int i = 0; i < c.n; ++i)
    if (s_host[i] < -1 || s_host[i] > 1) throw Error(-1, "secret key must be ternary");
  auto sk = std::make_unique<SecretKey>();
  sk->ctx = &c;
  const Basis qp = c.basis_QP(c.L);
  const size_t words = (size_t)qp.n * c.n;
  BCN_HIP(hipMalloc(&sk->s_hat, words * sizeof(double)));
  BCN_HIP(hipMalloc(&sk->s_coef, words * sizeof(double)));
  int8_t* d = nullptr;
  BCN_HIP(hipMalloc(&d, c.n));
  BCN_HIP(hipMemcpy(d, s_host, c.n, hipMemcpyHostToDevice));
  // residues of s on every limb: the same int8 row broadcast over the limbs
  for (int i = 0; i < qp.n; ++i) {
    Basis one{};
    one.n = 1;
    one.id[0] = qp.id[i];
    small_to_rns(c, d, sk->s_coef + (size_t)i * c.n, 1, one, nullptr);
  }
  BCN_HIP(hipMemcpy(sk->s_hat, sk->s_coef, words * sizeof(double), hipMemcpyDeviceToDevice));
  ntt_forward(c, sk->s_hat, 1, qp, nullptr);
  BCN_HIP(hipDeviceSynchronize());
  BCN_HIP(hipFree(d));
  return sk.release();
}

void keygen(Context& c, const SecretKey& sk, EvalKeys& ek, int kind, int step, const uint64_t* a_host,
            const int8_t* e_host, hipStream_t s) {
  Arena& ar = *c.arena;
  const Basis qp = c.basis_QP(c.L);
  const int nb = qp.n, dn = c.dnum(c.L);
  const size_t N = c.n, limbw = (size_t)nb * N;
  // a -> transform domain
  const uint64_t* au = dev_upload(a_host, (size_t)dn * limbw, s, ar);
  double* A = ar.take((size_t)dn * limbw);
  u64_to_f64(au, A, (size_t)dn * limbw, s);
  ntt_forward(c, A, dn, qp, s);
  // e -> residues -> transform domain
  const int8_t* ed = dev_upload(e_host, (size_t)dn * N, s, ar);
  double* E = ar.take((size_t)dn * limbw);
  small_to_rns(c, ed, E, dn, qp, s);
  ntt_forward(c, E, dn, qp, s);
  // s' in the transform domain
  double* Sp = ar.take(limbw);
  if (kind == 0) {
    pointwise_mul(c, sk.s_hat, sk.s_hat, Sp, 1, qp, true, s);
  } else {
    automorphism_coeff(c, sk.s_coef, Sp, 1, qp, galois_element(c, step), s);
    ntt_forward(c, Sp, 1, qp, s);
  }
  double* key = nullptr;
  BCN_HIP(hipMalloc(&key, ek.key_doubles() * sizeof(double)));
  double* AS = ar.take(limbw);
  std::vector<double> gval(nb, 0.0);
  for (int i = 0; i < c.L; ++i) {
    uint64_t pm = 1;
    for (int k = 0; k < c.K; ++k) pm = host::mulmod(pm, c.primes[c.idP(k)] % c.primes[i], c.primes[i]);
    gval[i] = (double)pm;
  }
  for (int j = 0; j < dn; ++j) {
    const int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, c.L);
    pointwise_mul(c, A + j * limbw, sk.s_hat, AS, 1, qp, true, s);
    combine_keypart(c, AS, E + j * limbw, Sp, key + (size_t)(2 * j) * limbw, qp, lo, hi, gval.data(), s);
    BCN_HIP(hipMemcpyAsync(key + (size_t)(2 * j + 1) * limbw, A + j * limbw, limbw * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  }
  BCN_HIP(hipStreamSynchronize(s));
  if (kind == 0) {
    if (ek.relin) BCN_HIP(hipFree(ek.relin));
    ek.relin = key;
  } else {
    auto it = ek.rot.find(step);
    if (it != ek.rot.end()) BCN_HIP(hipFree(it->second));
    ek.rot[step] = key;
    // cached tables may hold the old pointer
    for (auto& kv : ek.tables) {
      (void)hipFree(kv.second.keys);
      (void)hipFree(kv.second.galois);
      (void)hipFree(kv.second.kinv);
    }
    ek.tables.clear();
  }
}

void encode_device(Context& c, const int64_t* slots_dev, double* m, int n, hipStream_t s) {
  fill(m, (size_t)n * c.n, 0.0, s);
  slots_to_tdomain(c, slots_dev, m, n, s);
  ntt_inverse(c, m, n, basis_t(c), s);
}

void encode_plain_ntt(Context& c, const int64_t* slots_host, int n, int level, double* out, hipStream_t s,
                      bool over_qp) {
  Arena& ar = *c.arena;
  const int64_t* sd = dev_upload(slots_host, (size_t)n * c.n, s, ar);
  double* m = ar.take((size_t)n * c.n);
  encode_device(c, sd, m, n, s);
  const Basis b = over_qp ? c.basis_QP(level) : c.basis_Q(level);
  lift_plain(c, m, out, n, b.n, s, &b);
  ntt_forward(c, out, n, b, s);
  BCN_HIP(hipStreamSynchronize(s));
}

void encrypt(Context& c, const SecretKey& sk, const int64_t* slots_host, const uint64_t* a_host, const int8_t* e_host,
             int n, int level, double* ct, hipStream_t s) {
  if (level < 1 || level > c.L) throw Error(-2, "bad level");
  Arena& ar = *c.arena;
  const size_t N = c.n, pw = (size_t)level * N;
  const Basis q = c.basis_Q(level);
  const int64_t* sd = dev_upload(slots_host, (size_t)n * N, s, ar);
  double* m = ar.take((size_t)n * N);
  encode_device(c, sd, m, n, s);
  const uint64_t* au = dev_upload(a_host, (size_t)n * pw, s, ar);
  double* A = ar.take((size_t)n * pw);
  u64_to_f64(au, A, (size_t)n * pw, s);
  double* AS = ar.take((size_t)n * pw);
  BCN_HIP(hipMemcpyAsync(AS, A, (size_t)n * pw * sizeof(double), hipMemcpyDeviceToDevice, s));
  ntt_forward(c, AS, n, q, s);
  pointwise_mul(c, AS, sk.s_hat, AS, n, q, true, s);
  ntt_inverse(c, AS, n, q, s);
  const int8_t* ed = dev_upload(e_host, (size_t)n * N, s, ar);
  double* E = ar.take((size_t)n * pw);
  small_to_rns(c, ed, E, n, q, s);
  for (int i = 0; i < n; ++i)
    combine_keypart(c, AS + i * pw, E + i * pw, nullptr, ct + (size_t)i * 2 * pw, q, 0, 0, nullptr, s);
  BCN_HIP(hipMemcpy2DAsync(ct + pw, 2 * pw * sizeof(double), A, pw * sizeof(double), pw * sizeof(double), n,
                           hipMemcpyDeviceToDevice, s));
  add_delta(c, ct, n, level, m, s);
  BCN_HIP(hipStreamSynchronize(s));
}

void decrypt(Context& c, const SecretKey& sk, const double* ct, int n, int level, int64_t* slots_host, hipStream_t s) {
  if (level < 1 || level > c.L) throw Error(-2, "bad level");
  Arena& ar = *c.arena;
  const size_t N = c.n, pw = (size_t)level * N;
  const Basis q = c.basis_Q(level);
  double* C1 = ar.take((size_t)n * pw);
  BCN_HIP(hipMemcpy2DAsync(C1, pw * sizeof(double), ct + pw, 2 * pw * sizeof(double), pw * sizeof(double), n,
                           hipMemcpyDeviceToDevice, s));
  ntt_forward(c, C1, n, q, s);
  pointwise_mul(c, C1, sk.s_hat, C1, n, q, true, s);
  ntt_inverse(c, C1, n, q, s);
  double* X = ar.take((size_t)n * pw);
  BCN_HIP(hipMemcpy2DAsync(X, pw * sizeof(double), ct, 2 * pw * sizeof(double), pw * sizeof(double), n,
                           hipMemcpyDeviceToDevice, s));
  add_inplace(c, X, C1, n, level, s);
  double* M = ar.take((size_t)n * N);
  dec_round(c, X, M, n, level, s);
  ntt_forward(c, M, n, basis_t(c), s);
  int64_t* sd = reinterpret_cast<int64_t*>(ar.take((size_t)n * N));
  tdomain_to_slots(c, M, sd, n, s);
  BCN_HIP(hipMemcpyAsync(slots_host, sd, (size_t)n * N * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BCN_HIP(hipStreamSynchronize(s));
}

namespace {
// square + relinearisation from X [n][2][level+m][N] whose B limbs extend_qb has filled
void square_relin_tail(Context& c, const EvalKeys& ek, double* X, double* out, int n, int level, bool modsw,
                       hipStream_t s) {
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const Basis qb = c.basis_QB(level), qp = c.basis_QP(level);
  const int nb = qb.n, nbp = qp.n, dn = c.dnum(level);
  double* Y = ar.take((size_t)n * 3 * nb * N);
  if (c.fuse_square) {
    square_transform_fused(c, X, Y, n, qb, s);
  } else {
    ntt_forward(c, X, 2 * n, qb, s);
    tensor_square(c, X, Y, n, qb, s);
    ntt_inverse(c, Y, 3 * n, qb, s);
  }
  // d2 = round(t y_2 / Q) feeds the key switch; parts 0 and 1 are either scaled and rounded
  // inside ModDown (fused) or here with d2 (Z holds all three parts)
  const bool fuse = c.fuse_moddown && moddown_scale_round_ok(c, level);
  double* Z = ar.take((size_t)n * (fuse ? 1 : 3) * level * N);
  scale_round(c, Y, Z, n, level, s, fuse);
  const double* z2 = fuse ? Z : Z + 2 * level * N;
  const size_t z2_stride = (size_t)(fuse ? 1 : 3) * level * N;
  double* U = ar.take((size_t)n * 2 * nbp * N);
  KeySel ks;
  ks.key1 = ek.relin;
  if (c.ks_mode == 1) {
    ks_fused(c, z2, z2_stride, n, level, ek.relin, 1, U, s);
  } else if (c.ks_mode == 2) {
    double* D = ar.take((size_t)n * dn * nbp * N);
    ks_split(c, z2, z2_stride, n, level, ks, n, 1, D, U, s);
  } else {
    double* D = ar.take((size_t)n * dn * nbp * N);
    decompose_modup(c, z2, z2_stride, D, n, level, s);
    ntt_forward(c, D, n * dn, qp, s);
    ks_inner(c, D, 1, ks, n, level, U, s);
    ntt_inverse(c, U, 2 * n, qp, s);
  }
  if (fuse) {
    if (!moddown_scale_round(c, U, n, level, Y, modsw, out, s)) throw Error(-1, "no fused ModDown for this shape");
  } else {
    moddown(c, U, n, level, Z, 1, (size_t)3 * level * N, 1, ks, modsw, out, s);
  }
}
}  // namespace

void square_defer(Context& c, double* x, double* out, int n, int level, bool modsw, hipStream_t s, bool b_filled) {
  if (modsw && level < 2) throw Error(-2, "modulus switch needs two primes");
  if (n == 0) return;
  if (!b_filled) extend_qb(c, x, x, n, level, s);
  const Basis qb = c.basis_QB(level);
  double* Y = c.arena->take((size_t)n * 3 * qb.n * c.n);
  if (c.fuse_square) {
    square_transform_fused(c, x, Y, n, qb, s);
  } else {
    ntt_forward(c, x, 2 * n, qb, s);
    tensor_square(c, x, Y, n, qb, s);
    ntt_inverse(c, Y, 3 * n, qb, s);
  }
  scale_round(c, Y, out, n, level, s, false, modsw);
}

void relinearize3(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level, hipStream_t s,
                  bool ext_qb) {
  if (!ek.relin) throw Error(-3, "missing relinearisation key");
  if (n == 0) return;
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const Basis qp = c.basis_QP(level);
  const size_t ct3 = (size_t)3 * level * N;
  double* D = ar.take((size_t)n * c.dnum(level) * qp.n * N);
  double* U = ar.take((size_t)n * 2 * qp.n * N);
  KeySel ks;
  ks.key1 = ek.relin;
  // key switch of d2, then ModDown adds d0 and d1
  ks_split(c, in + 2 * level * N, ct3, n, level, ks, n, 1, D, U, s);
  moddown(c, U, n, level, in, 1, ct3, 1, ks, false, out, s, 0, 0, ext_qb);
}

size_t square_relin_scratch_doubles(const Context& c, int n, int level) {
  // mirrors the arena takes of square_relin and square_relin_tail
  const size_t N = c.n, nb = level + c.m, nbp = level + c.K, dn = c.dnum(level);
  const bool fuse = c.fuse_moddown && moddown_scale_round_ok(c, level);
  size_t d = Arena::rounded((size_t)n * 2 * nb * N) + Arena::rounded((size_t)n * 3 * nb * N) +
             Arena::rounded((size_t)n * (fuse ? 1 : 3) * level * N) + Arena::rounded((size_t)n * 2 * nbp * N);
  if (c.ks_mode != 1) d += Arena::rounded((size_t)n * dn * nbp * N);
  return d;
}

void square_relin(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level, bool modsw,
                  hipStream_t s) {
  if (!ek.relin) throw Error(-3, "missing relinearisation key");
  if (modsw && level < 2) throw Error(-2, "modulus switch needs two primes");
  if (n == 0) return;
  double* X = c.arena->take((size_t)n * 2 * (level + c.m) * c.n);
  extend_qb(c, in, X, n, level, s);
  square_relin_tail(c, ek, X, out, n, level, modsw, s);
}

void square_relin_qb(Context& c, const EvalKeys& ek, double* x, double* out, int n, int level, bool modsw,
                     hipStream_t s, bool b_filled) {
  if (!ek.relin) throw Error(-3, "missing relinearisation key");
  if (modsw && level < 2) throw Error(-2, "modulus switch needs two primes");
  if (n == 0) return;
  if (!b_filled) extend_qb(c, x, x, n, level, s);
  square_relin_tail(c, ek, x, out, n, level, modsw, s);
}

void rotate_hoisted(Context& c, EvalKeys& ek, const double* in, int n_in, int level, const std::vector<int>& steps,
                    double* out, hipStream_t s, int out_div, size_t out_outer) {
  const int ns = (int)steps.size();
  if (n_in == 0 || ns == 0) return;
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const Basis qp = c.basis_QP(level);
  const int nbp = qp.n, dn = c.dnum(level);
  const KeyTable& tb = ek.table(steps);
  double* D = ar.take((size_t)n_in * dn * nbp * N);
  double* U = ar.take((size_t)n_in * ns * 2 * nbp * N);
  KeySel ks;
  ks.keys = tb.keys;
  ks.galois = tb.galois;
  ks.kinv = tb.kinv;
  ks.nk = tb.nk;
  if (c.ks_mode_rot == 2) {
    ks_split(c, in + level * N, (size_t)2 * level * N, n_in, level, ks, n_in * ns, ns, D, U, s);
  } else {
    decompose_modup(c, in + level * N, (size_t)2 * level * N, D, n_in, level, s);
    ntt_forward(c, D, n_in * dn, qp, s);
    ks_inner(c, D, ns, ks, n_in * ns, level, U, s);
    ntt_inverse(c, U, 2 * n_in * ns, qp, s);
  }
  moddown(c, U, n_in * ns, level, in, ns, (size_t)2 * level * N, 2, ks, false, out, s, out_div, out_outer);
}

void taps_extended(Context& c, EvalKeys& ek, const double* in, const double* in_hat, int n_in, int level,
                   const std::vector<int>& steps, double* X, hipStream_t s) {
  if (n_in == 0) return;
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const Basis qp = c.basis_QP(level);
  const int ns = (int)steps.size(), k2 = ns + 1;
  const size_t ctx = (size_t)2 * qp.n * N;
  KsExt ext;
  ext.c0hat = in_hat;
  ext.c0_stride = (size_t)2 * level * N;
  ext.out_div = ns > 0 ? ns : 1;
  ext.out_outer = (size_t)k2 * ctx;
  for (int d = 0; d < level; ++d) {
    const uint64_t q = c.primes[d];
    uint64_t pm = 1;
    for (int i = 0; i < c.K; ++i) pm = host::mulmod(pm, c.primes[c.idP(i)] % q, q);
    ext.pm[d] = (double)pm;
  }
  ext_tap0(c, in_hat, n_in, level, ext, X, ext.out_outer, s);
  if (ns == 0) return;
  const KeyTable& tb = ek.table(steps);
  double* D = ar.take((size_t)n_in * c.dnum(level) * qp.n * N);
  KeySel ks;
  ks.keys = tb.keys;
  ks.galois = tb.galois;
  ks.kinv = tb.kinv;
  ks.nk = tb.nk;
  ks_extended(c, in + level * N, (size_t)2 * level * N, n_in, level, ks, n_in * ns, ns, D, X + ctx, ext, s);
}

std::vector<std::vector<int>> rotate_sum_rounds(int span) {
  if (span < 2 || (span & (span - 1))) throw Error(-1, "rotate-and-sum span must be a power of two >= 2");
  int k = 0;
  while ((1 << k) < span) ++k;
  const int b = 1 << ((k + 1) / 2), g = span / b;
  std::vector<std::vector<int>> rounds(2);
  for (int r = 1; r < b; ++r) rounds[0].push_back(r);
  for (int j = 1; j < g; ++j) rounds[1].push_back(j * b);
  return rounds;
}

void rotate_sum(Context& c, EvalKeys& ek, double* ct, int n, int level, int span, hipStream_t s) {
  const auto rounds = rotate_sum_rounds(span);
  if (n == 0) return;
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const Basis qp = c.basis_QP(level);
  const size_t ctw = (size_t)2 * level * N, ctx = (size_t)2 * qp.n * N;
  // each round: S <- ModDown(sum over its taps of Rot~(S, r)), tap 0 = P S; the taps' inner
  // products run over all of them at once (one digit decomposition of S)
  KsExt ext;
  for (int d = 0; d < level; ++d) {
    const uint64_t q = c.primes[d];
    uint64_t pm = 1;
    for (int i = 0; i < c.K; ++i) pm = host::mulmod(pm, c.primes[c.idP(i)] % q, q);
    ext.pm[d] = (double)pm;
  }
  for (const std::vector<int>& steps : rounds) {
    if (steps.empty()) continue;
    double* H = ar.take((size_t)n * ctw);
    copy_rows(ct, 0, H, 0, (size_t)n * ctw, 1, s);
    ntt_forward(c, H, 2 * n, c.basis_Q(level), s);
    const KeyTable& tb = ek.table(steps);
    KeySel ks;
    ks.keys = tb.keys;
    ks.galois = tb.galois;
    ks.kinv = tb.kinv;
    ks.nk = tb.nk;
    double* D = ar.take((size_t)n * c.dnum(level) * qp.n * N);
    double* U = ar.take((size_t)n * ctx);
    ks_sum_round(c, ct + level * N, ctw, n, level, ks, H, ctw, ext, D, U, s);
    ntt_inverse(c, U, 2 * n, qp, s);
    moddown(c, U, n, level, nullptr, 1, 0, 0, KeySel(), false, ct, s);
  }
}

MacPlan make_mac_plan(const Context& c, const std::vector<int32_t>& w, int n_out, int n_in,
                      const std::vector<int>& order_in, int tile) {
  MacPlan p;
  p.n_in = n_in;
  p.n_out = n_out;
  std::vector<int> order = order_in;
  if (order.empty())
    for (int o = 0; o < n_out; ++o) order.push_back(o);
  if ((int)order.size() != n_out) throw Error(-1, "MAC row order has the wrong length");
  if (tile == 0) {
    tile = 1;
    while (tile < 64 && tile < n_out) tile *= 2;
  }
  p.tile = tile;
  p.n_tiles = (n_out + tile - 1) / tile;
  const size_t slots = (size_t)p.n_tiles * tile;
  std::vector<int> rows(slots, -1);
  std::vector<int> ptr(1, 0), cols;
  std::vector<double> W;   // [entry][tile]
  int32_t wmax = 1;
  for (int t = 0; t < p.n_tiles; ++t) {
    for (int o = 0; o < tile && t * tile + o < n_out; ++o) {
      const int row = order[t * tile + o];
      if (row < 0 || row >= n_out) throw Error(-1, "MAC row order out of range");
      rows[t * tile + o] = row;
    }
    for (int j = 0; j < n_in; ++j) {
      bool any = false;
      for (int o = 0; o < tile; ++o) {
        const int row = rows[t * tile + o];
        if (row >= 0 && w[(size_t)row * n_in + j] != 0) any = true;
      }
      if (!any) continue;
      cols.push_back(j);
      for (int o = 0; o < tile; ++o) {
        const int row = rows[t * tile + o];
        const int32_t v = row >= 0 ? w[(size_t)row * n_in + j] : 0;
        wmax = std::max(wmax, v < 0 ? -v : v);
        p.nnz += v != 0;
        W.push_back((double)v);
      }
    }
    ptr.push_back((int)cols.size());
  }
  if (wmax > (1 << 20)) throw Error(-1, "weights must be below 2^20 in magnitude");
  double qmax = 0;
  for (int i = 0; i < c.L; ++i) qmax = std::max(qmax, (double)c.primes[i]);
  // |acc| <= q/2 + 1 + chunk * wmax * (q-1)/2 must stay below 2^53
  const double room = 9007199254740992.0 - qmax;
  p.chunk = std::max(4, (int)std::min(1e6, std::floor(room / ((double)wmax * qmax * 0.5))));
  if ((double)p.chunk * wmax * qmax * 0.5 >= room) throw Error(-1, "weights too large for exact accumulation");
  // residues in [0, q) need no centring when each tile's sum of |w| times q - 1 stays below 2^53
  double tile_abs_max = 0;
  for (int t = 0; t < p.n_tiles; ++t)
    for (int o = 0; o < tile; ++o) {
      double a = 0;
      for (int e = ptr[t]; e < ptr[t + 1]; ++e) a += std::fabs(W[(size_t)e * tile + o]);
      tile_abs_max = std::max(tile_abs_max, a);
    }
  p.centre = !(tile_abs_max * qmax < room);
  BCN_HIP(hipMalloc(&p.W, std::max<size_t>(1, W.size()) * sizeof(double)));
  BCN_HIP(hipMalloc(&p.rows, rows.size() * sizeof(int)));
  BCN_HIP(hipMalloc(&p.tile_ptr, ptr.size() * sizeof(int)));
  BCN_HIP(hipMalloc(&p.tile_cols, std::max<size_t>(1, cols.size()) * sizeof(int)));
  BCN_HIP(hipMemcpy(p.W, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice));
  BCN_HIP(hipMemcpy(p.rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice));
  BCN_HIP(hipMemcpy(p.tile_ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice));
  if (!cols.empty()) BCN_HIP(hipMemcpy(p.tile_cols, cols.data(), cols.size() * sizeof(int), hipMemcpyHostToDevice));
  return p;
}

void free_mac_plan(MacPlan& p) {
  if (p.W) (void)hipFree(p.W);
  if (p.rows) (void)hipFree(p.rows);
  if (p.tile_ptr) (void)hipFree(p.tile_ptr);
  if (p.tile_cols) (void)hipFree(p.tile_cols);
  p.W = nullptr;
  p.rows = p.tile_ptr = p.tile_cols = nullptr;
}
}  // namespace bcn
