// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "hostmath.h"
#include "modarith.h"

namespace bcn {

constexpr int kMaxBasis = 24;   // limbs in one RNS basis (Q + P + B)

// Limb -> prime-id map of one RNS buffer, passed to kernels by value.
struct Basis {
  int n;
  int id[kMaxBasis];
};

// Device-resident per-prime tables (all binary64 integers).
struct Tables {
  const double* fwd;   // [np][N]   forward twiddles psi^bitrev(2^s + b) at [2^s + fwd_tw_word(b, s)]
  const double* inv;   // [np][N]   stage-major: [2^s + p] = omega^-(p N / 2^(s+1)), omega = psi^2
  const double* post;  // [np][N]   N^-1 psi^-k: untwist of the inverse transform
  const Mod* mods;     // [np]
  int logn;
};

// Storage order of transform-domain limbs.  Transform index i (evaluation point
// psi^(2 bitrev(i) + 1)) is stored at word (i mod 16) * N/16 + floor(i / 16): the
// forward transform's last pass, in which every thread holds 2^LOGE consecutive
// indices, then writes lane-consecutive words, and the inverse transform's first
// pass reads them the same way (with i stored at word i, every lane of a wave
// touched its own cache line).  Requires N >= 16.
BCN_HD int ntt_store(int i, int logn) { return ((i & 15) << (logn - 4)) + (i >> 4); }
BCN_HD int ntt_index(int p, int logn) { return ((p & ((1 << (logn - 4)) - 1)) << 4) + (p >> (logn - 4)); }

// Forward twiddles: stage s (2^s blocks) keeps psi^bitrev(2^s + b) for block b at
// word 2^s + fwd_tw_word(b, s, logn).  In the last four stages the blocks of one
// thread are consecutive and the lanes of a wave step by 2^(s - logn + 4); within
// those stages the words are stored transposed (b mod M, b / M with M = 2^(s - logn + 4))
// so that a wave's loads are lane-consecutive.
BCN_HD int fwd_tw_word(int b, int s, int logn) {
  const int lm = s - (logn - 4);
  if (lm <= 0) return b;
  return ((b & ((1 << lm) - 1)) << (s - lm)) + (b >> lm);
}

__device__ __forceinline__ int bitrev_n(int x, int logn) { return (int)(__brev((unsigned)x) >> (32 - logn)); }

// Transform-domain automorphism: sigma_k(a)^ at transform index i is a^ at the
// returned transform index (evaluation point psi^(2 bitrev(i) + 1) maps to its k-th power).
__device__ __forceinline__ int ntt_perm(int i, int galois, int logn) {
  const int N = 1 << logn;
  const int j = bitrev_n(i, logn);
  const int e = (int)(((long long)(2 * j + 1) * galois) & (2 * N - 1));
  return bitrev_n((e - 1) >> 1, logn);
}

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define BCN_HIP(x)                                                                 \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess)                                                          \
      throw ::bcn::Error(-5, std::string("HIP error: ") + hipGetErrorString(e_) +  \
                                 " at " + __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

// Grow-only device scratch arena owned by a context.  take() hands out
// stream-ordered scratch that stays valid until the next reset(); reset() is
// called at the start of every public entry point.  When a call needed more
// than one chunk, the next reset() replaces them by one chunk of 1.25x the
// high-water size, so from the second call of a shape on there is one chunk
// and no hipMalloc on the hot path.  The replaced chunks are not freed: a
// hipGraph captured earlier may still read and write them.  They stay
// allocated (retired) until release_retired() or the arena's destruction.
//
// While bound to caller memory (bind_external), take() bumps through that
// buffer only and throws when it is exhausted: no allocation of any kind.
class Arena {
 public:
  ~Arena();
  double* take(size_t doubles);
  void reset();
  size_t capacity() const;
  // the most scratch one call has used since the previous take_recent_high()
  size_t take_recent_high() {
    const size_t b = recent_high_ * sizeof(double);
    recent_high_ = 0;
    return b;
  }
  size_t retired_bytes() const;
  // frees the retired chunks; the caller guarantees no pending work or graph uses them
  size_t release_retired();
  const double* base() const { return chunks_.empty() ? nullptr : chunks_[0].p; }
  uint64_t generation() const { return generation_; }
  void bind_external(double* base, size_t cap);
  void unbind_external();
  // doubles that take(d_1), ..., take(d_k) consume from an empty arena
  static size_t rounded(size_t doubles) { return (doubles + 31) & ~(size_t)31; }

 private:
  struct Chunk { double* p; size_t cap; };
  std::vector<Chunk> chunks_, retired_;
  size_t cur_ = 0, off_ = 0, used_total_ = 0, high_ = 0, recent_high_ = 0;
  uint64_t generation_ = 0;
  double* ext_ = nullptr;
  size_t ext_cap_ = 0, ext_off_ = 0;
};

// Optional per-kernel timing: hipEvents recorded around launches on the
// launch stream while profiling is enabled; algorithmic bytes accumulate per
// kernel name.
struct ProfEntry {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double bytes = 0;   // algorithmic HBM bytes
  double ops = 0;     // algorithmic FP64 VALU lane operations (0 when not tracked)
  long launches = 0;
};

struct Context {
  int device = 0;
  mutable bool prof = false;
  mutable std::map<std::string, ProfEntry> prof_data;
  mutable std::vector<hipEvent_t> event_pool;
  hipEvent_t get_event() const;
  int n = 0, logn = 0;
  int L = 0, K = 0, alpha = 0, m = 0;   // Q primes, P primes, digit size, aux primes
  uint64_t t = 0;                        // BFV plaintext modulus (0 for CKKS)
  int scheme = 0;                        // 0 BFV, 1 CKKS
  int gen = 3;                           // slot rotation generator: Rot(c, r) = sigma_{gen^r}
  double* ckks_tab = nullptr;            // CKKS encoder tables (ckks.hip)
  std::vector<uint64_t> primes;          // ids: Q [0,L), P [L,L+K), B [L+K,L+K+m), t last
  std::vector<Mod> hmods;
  int id_t = 0;
  double* d_tables = nullptr;            // one allocation for all tables
  Tables tab{};
  uint32_t* d_slot_pos = nullptr;        // [N] position of slot s in the transform of R_t
  uint32_t* d_slot_of_word = nullptr;    // [N] inverse of d_slot_pos: the slot held at each word
  std::unique_ptr<Arena> arena;
  mutable bool no_alloc = false;         // set while an entry point that must not allocate runs
  double* fixed_scratch = nullptr;       // this device's static scratch array (device address)
  size_t fixed_scratch_doubles = 0;

  int ntt_loge = 0;                      // registers per thread = 2^ntt_loge in the transform
  int square_loge = 0;                   // the same for the fused square's transforms
  bool pinned_loge = false, pinned_square_loge = false, pinned_prefetch = false;   // fixed by the environment
  bool fuse_square = true;               // square's transforms and tensor in one kernel
  bool fuse_moddown = true;              // relinearisation's ModDown also scales and rounds d0, d1
  bool ntt_persist = false;              // persistent, prefetching transform kernel
  bool ntt_prefetch = false;             // transform loads the next pass's twiddles before each exchange
  bool ntt_xlane = false;                // exchanges that are row transposes run on cross-lane moves (2^4 per thread)
  bool pinned_xlane = false;
  int persist_blocks = 512;              // its grid: workgroups resident at once
  int n_cus = 256;                       // compute units of the device
  int ks_mode = 2;                       // key switching: 0 ModUp + NTT + inner product + INTT (four kernels),
                                         // 1 one fused kernel, 2 digits+NTT and inner product+INTT (two kernels)
  int ks_mode_rot = 2;                   // the same for hoisted rotations (0 or 2)
  int ks_loge = 4;                       // transform shape of the two-kernel key switch
  bool pinned_ks = false;
  // A layer's per-ciphertext chain after a slot-batched MAC (square, its relinearisation or
  // scale-and-round) may run as two halves on two streams, so one half's kernels fill the CUs
  // the other half's tails leave idle.  Not while profiling (per-kernel times stay serial).
  bool split_chain = true;
  hipStream_t side = nullptr;            // the second stream (default priority)
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  std::vector<int> ntt_loge_options() const;

  int idQ(int i) const { return i; }
  int idP(int i) const { return L + i; }
  int idB(int i) const { return L + K + i; }
  int dnum(int level) const { return (level + alpha - 1) / alpha; }
  Basis basis_Q(int level) const;
  Basis basis_QP(int level) const;       // Q_level then P
  Basis basis_QB(int level) const;       // Q_level then B
  Mod mod(int id) const { return hmods[id]; }
};

class ProfScope {
 public:
  ProfScope(const Context& c, const char* name, hipStream_t s, double bytes, double ops = 0.0);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const Context& c_;
  hipStream_t s_;
  ProfEntry* e_ = nullptr;
  hipEvent_t start_ = nullptr;
};

// ---- transforms (ntt.hip)
// one item of a multi-context transform launch: limbs [n_polys][n_limbs][N] of one context,
// limb i with prime id first_prime + i
constexpr int kMaxMultiItems = 16;
struct MultiNttItem {
  double* data;
  Tables tb;
  int logn, n_limbs, first_prime, units;
};
struct MultiNttWork {
  MultiNttItem it[kMaxMultiItems];
  int n_items, total;
};
void ntt_multi(const std::vector<MultiNttItem>& items, bool inverse, hipStream_t s);
// data: [n_polys][basis.n][N]; each limb transformed in place with its prime.
void ntt_forward(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s);
void ntt_inverse(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s);
void ntt_setup(const Context& c);
// in [n][2][b.n][N] coefficient form -> out [n][3][b.n][N]: the square's tensor
// d0 = a0^2, d1 = 2 a0 a1, d2 = a1^2 in R_q for every limb, via fused transforms
void square_transform_fused(const Context& c, const double* in, double* out, int n, const Basis& b, hipStream_t s);
// key switching of n source polynomials (coefficient form, [level][N] at src + i*src_stride) with one
// key ([dnum][2][L+K][N], transform domain); galois = k applies X -> X^k to the source first.
// u [n][2][level+K][N] coefficient form (before the division by P).
void ks_fused(const Context& c, const double* src, size_t src_stride, int n, int level, const double* key, int galois,
              double* u, hipStream_t s);

}  // namespace bcn

namespace bcn {

// Exact basis conversion tables (mixed-radix / Garner).  A source basis
// p_0..p_{ns-1} gives digits v with x = v_0 + p_0 (v_1 + p_1 (v_2 + ...)),
// 0 <= v_k < p_k; comparing the digits with those of (M-1)/2, which are
// (p_k - 1)/2, decides whether the centred value is x or x - M.
struct Conv {
  int ns, nd;
  int src[kMaxBasis], dst[kMaxBasis];
  double ginv[kMaxBasis][kMaxBasis];   // [i][k] = p_k^-1 mod p_i   (k < i)
  double pm[kMaxBasis][kMaxBasis];     // [d][k] = p_k mod dst_d
  double Mmod[kMaxBasis];              // prod_k p_k mod dst_d
  double aux[kMaxBasis];               // per-destination extra constant (see users)
  double aux2[kMaxBasis];
};

Conv make_conv(const Context& c, const std::vector<int>& src, const std::vector<int>& dst);
// device copy of a conversion table, cached per (context, key); allocates on a miss
const Conv* conv_device(const Context& c, const std::string& key, const Conv& cv);
// fill that cache for every level at context creation (kernels.hip, ntt.hip)
void preload_conversions(const Context& c);
void preload_ks_digits(const Context& c);

// ---- element kernels (kernels.hip); all buffers are limb-major [..][limb][N]
// out[o] = sum_j W[o][j] * in[j]; W dense f64 [n_out][n_in] (device),
// tiles: per tile of TO rows the list of columns with a nonzero weight.
struct MacPlan {
  int n_in = 0, n_out = 0, tile = 0, n_tiles = 0;
  double* W = nullptr;          // device [entries][tile]: weights of each tile column entry
  int* rows = nullptr;          // device [n_tiles*tile]: output row of each tile slot, -1 = none
  int* tile_ptr = nullptr;      // device [n_tiles+1]
  int* tile_cols = nullptr;     // device: columns with a nonzero weight in the tile
  int chunk = 0;                // inputs between two partial reductions
  long nnz = 0;                 // nonzero weights
  bool centre = true;           // false: every tile's sum of |w| * (q-1) fits 2^53 uncentred
};
// requests > 1: independent requests at in + r*in_req, out + r*out_req (doubles)
// out_ct, out_part (doubles): output row r's part k starts at out + r * out_ct + k * out_part
// (0: contiguous [rows][2][level][N]); e.g. the Q limbs of a [rows][2][level+m][N] buffer
// basis: the limbs of each part when they are not Q_level (e.g. Q_level then P); then
// `level` only selects the delta constants and delta_msg must be null.
// parts = 3: rows of three-part products [3][level][N] (no delta add)
// mul_pt: every output word is multiplied by this transform-domain plaintext [limbs][N] (the
// inputs being in the transform domain); exclusive with delta_msg
void mac(const Context& c, const MacPlan& p, const double* in, double* out, int level, hipStream_t s, int requests = 1,
         size_t in_req = 0, size_t out_req = 0, const double* delta_msg = nullptr, size_t out_ct = 0,
         size_t out_part = 0, const Basis* basis = nullptr, int parts = 2, const double* mul_pt = nullptr);

// The MAC of a slot-batched layer feeding a square, writing out rows [2][level + m][N] over
// Q_level then B (the extension fused into the MAC's stores); out_ct, out_part as for mac.
// Returns false (and does nothing) when the plan's tile or centring is not supported.
bool mac_qb_supported(const MacPlan& p, int level);
bool mac_qb(const Context& c, const MacPlan& p, const double* in, double* out, int level, hipStream_t s, int requests,
            size_t in_req, size_t out_req, const double* delta_msg, size_t out_ct, size_t out_part);

// c0 of each ciphertext += Delta(m_i), m_i in [0, t) coefficient form, [n][N]
void add_delta(const Context& c, double* ct, int n, int level, const double* m, hipStream_t s);
// out[k] = in[k] (.) pt  (NTT domain); pt [level][N] shared, or [n][level][N] when per_ct
// (basis: the limbs when they are not Q_level)
void mul_plain_ntt(const Context& c, const double* in, double* out, int n, int level, const double* pt,
                   bool per_ct, hipStream_t s, const Basis* basis = nullptr);
// out[k] = sum_c in[c] (.) pt[k][c]  (NTT domain); pt [n_out][n_in][level][N]
void ptvec_mac_ntt(const Context& c, const double* in, int n_in, double* out, int n_out, int level,
                   const double* pt, hipStream_t s, int requests = 1);
// square in the NTT domain over `nb` limbs: [n][2][nb][N] -> [n][3][nb][N]
void tensor_square(const Context& c, const double* in, double* out, int n, const Basis& b, hipStream_t s);
// exact centred extension of [n][2][level][N] (coeff) into [n][2][level+m][N] over Q_level then B
void extend_qb(const Context& c, const double* in, double* out, int n, int level, hipStream_t s);
// round(t x / Q_level) for [n][3][level+m][N] (coeff, Q then B) -> [n][3][level][N], or with
// only_d2 just part 2 of each ciphertext -> [n][level][N]; modsw: then the modulus switch to
// level - 1 limbs
void scale_round(const Context& c, const double* in, double* out, int n, int level, hipStream_t s,
                 bool only_d2 = false, bool modsw = false);
// centred digits of x [n][level][N] (coeff) raised to Q_level+P: [n][dnum][level+K][N]
void decompose_modup(const Context& c, const double* in, size_t in_stride, double* out, int n, int level,
                     hipStream_t s);
// u[p] = sum_j D_j (.) key_j[p] over Q_level+P (NTT domain); output o uses digit block o / d_div
// of D ([*][dnum][level+K][N]), the key keys[o] (device [dnum][2][L+K][N]) and, when galois is not
// null, first permutes the digits by the automorphism X -> X^galois[o].  out [n][2][level+K][N].
// Key selection for a batch of key switches: output o uses table entry o % nk, or the single
// key1/galois1/kinv1 when keys is null.  galois = 1 means no automorphism.
struct KeySel {
  const double* const* keys = nullptr;
  const int* galois = nullptr;
  const int* kinv = nullptr;
  int nk = 1;
  const double* key1 = nullptr;
  int galois1 = 1;
  int kinv1 = 1;
};
void ks_inner(const Context& c, const double* D, int d_div, const KeySel& ks, int n, int level, double* out,
              hipStream_t s);
// Key switching in two kernels: digits of n_src sources formed and transformed into D
// ([n_src][dnum][level + K][N], transform domain), then for each of n_out outputs the
// inner product with its key (output o uses source o / d_div) and both inverse
// transforms into u ([n_out][2][level + K][N], coefficient form).
// src_galois != 1 switches sigma_k(source) (k = src_galois): the digits are stored through
// the transform-domain permutation, and ks must then carry none (galois 1).
void ks_split(const Context& c, const double* src, size_t src_stride, int n_src, int level, const KeySel& ks,
              int n_out, int d_div, double* D, double* u, hipStream_t s, int src_galois = 1);
// Rotations kept over Q_l P before ModDown (the taps of a convolution whose weighted sum
// is divided by P once): output o = P sigma(c0) + sum_j sigma(D_j) key_j[0] on the Q limbs
// (the key term alone on the P limbs) and sum_j sigma(D_j) key_j[1], in the transform
// domain, written at u + (o / out_div) * out_outer + (o % out_div) * 2 (level + K) N.
// c0hat: the sources' part 0 transformed over Q_level, source i at c0hat + i * c0_stride.
struct KsExt {
  const double* c0hat = nullptr;
  size_t c0_stride = 0;
  int out_div = 1;
  size_t out_outer = 0;
  double pm[kMaxBasis] = {};   // P mod q_i, i < level
};
void ks_extended(const Context& c, const double* src, size_t src_stride, int n_src, int level, const KeySel& ks,
                 int n_out, int d_div, double* D, double* u, const KsExt& ext, hipStream_t s);
// Tap 0 of ks_extended's layout: P c^ on the Q limbs and 0 on the P limbs of each part, for
// n sources c^ ([n][2][level][N], transform domain) into X + i * out_outer ([2][level + K][N]).
void ext_tap0(const Context& c, const double* chat, int n, int level, const KsExt& ext, double* X, size_t out_outer,
              hipStream_t s);
// One rotate-and-sum round over n sources (c1 parts at src + i * src_stride, coefficient form):
// digits into D, then u[i] = P c^ + sum over the table's steps of Rot~(c, step) over Q_level P
// in the transform domain ([n][2][level + K][N]); chat: the sources transformed over Q_level
// ([2][level][N] at chat + i * c_stride); ext.pm as for ks_extended.
void ks_sum_round(const Context& c, const double* src, size_t src_stride, int n, int level, const KeySel& ks,
                  const double* chat, size_t c_stride, const KsExt& ext, double* D, double* u, hipStream_t s);
// out = sum of `slabs` slabs of `words` residues each (slab k at in + k * words), reduced mod the
// basis' primes; the words are n_polys polynomials [n_polys][b.n][N]
void sum_slabs(const Context& c, const double* in, int slabs, size_t words, int n_polys, const Basis& b, double* out,
               hipStream_t s);
// exact round(u/P) of u [n][2][level+K][N] (coeff) -> [n][2][level][N], plus an addend:
// add_mode 0: none; 1: add [n][2][level][N]; 2: add sigma_k(add) to part 0 only (add [n][2][level][N]);
// 3: add add itself and sigma_k of its part 0 (rotate-and-add; out must not alias add).
// With modswitch the result is further rounded by q_level to level-1 limbs.
// The addend of output o is add + (o / add_div) * add_stride; mode 2 gathers it through the
// inverse Galois element kinv[o].
// Output o is written at out + (o / out_div) * out_outer + (o % out_div) * (ciphertext size);
// out_div = 0 means contiguous outputs.
// ext_qb (no modulus switch, contiguous outputs): out is [n][2][level+m][N] over Q_level then B,
// and the B limbs receive the centred lift of the result (the steps of extend_qb).
void moddown(const Context& c, const double* u, int n, int level, const double* add, int add_div, size_t add_stride,
             int add_mode, const KeySel& ks, bool modswitch, double* out, hipStream_t s, int out_div = 0,
             size_t out_outer = 0, bool ext_qb = false);
// Relinearisation's ModDown with the addend scaled and rounded inline: out = round(u/P) +
// round(t y_k / Q_level) for parts k = 0, 1 of the square's tensor y ([n][3][level+m][N], coeff,
// Q_level then B), optionally modulus-switched.  Returns false (nothing launched) when the
// shape (special, ciphertext and auxiliary prime counts) has no compiled variant.
bool moddown_scale_round(const Context& c, const double* u, int n, int level, const double* y, bool modswitch,
                         double* out, hipStream_t s);
bool moddown_scale_round_ok(const Context& c, int level);
// out = a + b over [count] words whose limb is (word >> logn) % nl
// a += b over n polynomials of `level` limbs ([n][level][N], limb = row % level)
void add_inplace(const Context& c, double* a, const double* b, int npoly, int level, hipStream_t s);
// [n][2][level][N] -> [n][2][level-1][N]
void modswitch(const Context& c, const double* in, double* out, int n, int level, hipStream_t s);
// coefficient-domain automorphism of [n][limbs][N]
void automorphism_coeff(const Context& c, const double* in, double* out, int n, const Basis& b, int k,
                        hipStream_t s);
// m [n][N] in [0, t): residues of lift_c(m) on each limb of Q_level -> [n][level][N]
void lift_plain(const Context& c, const double* m, double* out, int n, int level, hipStream_t s,
                const Basis* basis = nullptr);
// slot values (int64, any representative) -> transform-domain vector mod t at the slot positions
void slots_to_tdomain(const Context& c, const int64_t* slots, double* out, int n, hipStream_t s);
// slot-batched FP32 features [requests][batch][stride_b] -> quantised plaintexts in the
// transform domain of R_t [n_pt][N] (n_pt = requests * stride_b)
void features_to_tdomain(const Context& c, const float* f, int n_pt, int batch, int stride_b, float scale, int clampv,
                         double* out, hipStream_t s);
void tdomain_to_slots(const Context& c, const double* in, int64_t* slots, int n, hipStream_t s);
// decryption rounding: x [n][level][N] (coeff) -> m [n][N] = round(t x / Q) mod t
void dec_round(const Context& c, const double* x, double* m, int n, int level, hipStream_t s);
// elementwise helpers on [n][limbs][N]
void pointwise_mul(const Context& c, const double* a, const double* b, double* out, int n, const Basis& bs,
                   bool b_shared, hipStream_t s);
void small_to_rns(const Context& c, const int8_t* e, double* out, int n, const Basis& b, hipStream_t s);
void u64_to_f64(const uint64_t* in, double* out, size_t count, hipStream_t s);
// graph-capturable fills and strided copies (kernels, not memset / memcpy nodes)
void fill(double* p, size_t count, double v, hipStream_t s);
void copy_rows(const double* src, size_t spitch, double* dst, size_t dpitch, size_t width, size_t rows, hipStream_t s);
void f64_to_u64(const double* in, uint64_t* out, size_t count, hipStream_t s);
// out = -x + e (+ g * sp on the limbs in [g_lo, g_hi)) elementwise over [limbs][N]; g_val per limb
void combine_keypart(const Context& c, const double* x, const double* e, const double* sp, double* out,
                     const Basis& b, int g_lo, int g_hi, const double* g_val_host, hipStream_t s);
// quantise FP32 features: q(f) = clamp(rint(8 f), -127, 127), gathered into slot vectors.
// mode 0 (batch packing): plaintext p = r*stride_b + j, slots[p][b] = q(f[(r*batch + b)*stride_b + j]);
// mode 1 (HW packing): slots[p][slot_of[k]] = q(f[p*per + k]) for k < per.
void quantise_features(const Context& c, const float* f, int n_pt, int mode, int batch, int stride_b,
                       const int* slot_of, int per, float scale, int clampv, int64_t* slots, hipStream_t s);

}  // namespace bcn
