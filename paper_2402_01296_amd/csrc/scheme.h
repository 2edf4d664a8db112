// Scheme-level objects and operations built from the kernels.
#pragma once

#include "internal.h"

namespace bcn {

struct SecretKey {
  const Context* ctx = nullptr;
  double* s_hat = nullptr;    // [L+K][N] transform of s over Q then P
  double* s_coef = nullptr;   // [L+K][N] residues of s
  ~SecretKey();
};

struct KeyTable {
  const double** keys = nullptr;  // device
  int* galois = nullptr;          // device
  int* kinv = nullptr;            // device
  int nk = 0;
};

struct EvalKeys {
  const Context* ctx = nullptr;
  double* relin = nullptr;                 // [dnum][2][L+K][N], transform domain
  std::map<int, double*> rot;              // step -> key
  std::map<std::vector<int>, KeyTable> tables;
  ~EvalKeys();
  size_t key_doubles() const;
  const double* rot_key(int step) const;
  const KeyTable& table(const std::vector<int>& steps);   // cached device arrays for a step list
};

int galois_element(const Context& c, int step);
int galois_inverse(const Context& c, int k);

SecretKey* secret_key_create(Context& c, const int8_t* s_host);
void keygen(Context& c, const SecretKey& sk, EvalKeys& ek, int kind, int step, const uint64_t* a_host,
            const int8_t* e_host, hipStream_t s);
void encrypt(Context& c, const SecretKey& sk, const int64_t* slots_host, const uint64_t* a_host, const int8_t* e_host,
             int n, int level, double* ct, hipStream_t s);
void decrypt(Context& c, const SecretKey& sk, const double* ct, int n, int level, int64_t* slots_host, hipStream_t s);

// m [n][N] in [0, t) from slot vectors already on the device (int64 [n][N])
void encode_device(Context& c, const int64_t* slots_dev, double* m, int n, hipStream_t s);
// NTT over Q_level of lift_c(encode(slots)) for host slot vectors [n][N] -> out [n][level][N]
// over_qp: the transform over Q_level then P ([n][level + K][N])
void encode_plain_ntt(Context& c, const int64_t* slots_host, int n, int level, double* out, hipStream_t s,
                      bool over_qp = false);

void square_relin(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level, bool modsw,
                  hipStream_t s);
// scratch doubles square_relin takes from the arena for n ciphertexts at `level`
size_t square_relin_scratch_doubles(const Context& c, int n, int level);
// square_relin with its scratch in the fixed per-device array (noalloc.hip): no allocation
void square_relin_noalloc(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level, bool modsw,
                          hipStream_t s);
void fixed_scratch_setup(Context& c);

// ---- CKKS (ckks.hip): the paper's scheme on the same rings, keys and key switching
void ckks_setup(Context& c);
// slots z (device, real, [n][N/2]) -> round(scale * m) as residues over Q_level ([n][level][N],
// coefficient form; with ntt_domain, transformed)
void ckks_encode(const Context& c, const double* z, int n, int level, double scale, bool ntt_domain, double* out,
                 hipStream_t s);
void ckks_encrypt(Context& c, const SecretKey& sk, const double* z_host, double scale, const uint64_t* a_host,
                  const int8_t* e_host, int n, int level, double* ct, hipStream_t s);
void ckks_decrypt(Context& c, const SecretKey& sk, const double* ct, int n, int level, double scale, double* z_host,
                  hipStream_t s);
// c0 += pt (coefficient residues [n][level][N], one per ciphertext)
void ckks_add_plain(const Context& c, double* ct, int n, int level, const double* pt, hipStream_t s);
// Mult(c1, c2) with c1 = c2, relinearised, then rescaled by q_level: [n][2][level][N] -> [n][2][level-1][N]
void ckks_square_relin_rescale(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level,
                               hipStream_t s);
// the same from x [n][2][level+m][N] whose Q limbs hold the input; x's B limbs are filled in place
void square_relin_qb(Context& c, const EvalKeys& ek, double* x, double* out, int n, int level, bool modsw,
                     hipStream_t s, bool b_filled = false);
// The square with its relinearisation deferred: x as for square_relin_qb; out [n][3][level'][N]
// holds (d0, d1, d2) = round(t (x (x) x) / Q_level), then modulus-switched when modsw
// (level' = level - 1).  Relinearisation is linear, so the next linear layer may run over the
// three parts and relinearise its outputs (relinearize3).
void square_defer(Context& c, double* x, double* out, int n, int level, bool modsw, hipStream_t s,
                  bool b_filled = false);
// (d0, d1, d2) [n][3][level][N] -> (d0 + KS(d2)_0, d1 + KS(d2)_1) [n][2][level][N]
// ext_qb: out is [n][2][level+m][N] over Q_level then B, the B limbs the result's centred lift
void relinearize3(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level, hipStream_t s,
                  bool ext_qb = false);
// out placement as in moddown (out_div = 0: contiguous [n_in][n_steps])
void rotate_hoisted(Context& c, EvalKeys& ek, const double* in, int n_in, int level, const std::vector<int>& steps,
                    double* out, hipStream_t s, int out_div = 0, size_t out_outer = 0);
// In place: the sum of Rot(c, r) over r < span, in two rounds (rotate_sum_rounds: baby steps
// 1 .. b-1, giant steps b .. (g-1) b, b = 2^ceil(k/2) for span = 2^k), each a hoisted set of
// rotations kept over Q_level P, summed, and brought down by one ModDown.
std::vector<std::vector<int>> rotate_sum_rounds(int span);
void rotate_sum(Context& c, EvalKeys& ek, double* ct, int n, int level, int span, hipStream_t s);
// The k2 taps of each of n_in inputs kept over Q_level P before ModDown, in the transform
// domain: X [n_in][k2][2][level + K][N], tap 0 = P * input, tap 1 + r = Rot~(input, steps[r]).
// in: the inputs (coefficient form), in_hat: the same transformed over Q_level.
void taps_extended(Context& c, EvalKeys& ek, const double* in, const double* in_hat, int n_in, int level,
                   const std::vector<int>& steps, double* X, hipStream_t s);

// w: [n_out][n_in]; order: output rows in tiling order (empty = natural); tile: outputs per
// tile (power of two <= 64, 0 = automatic)
MacPlan make_mac_plan(const Context& c, const std::vector<int32_t>& w, int n_out, int n_in,
                      const std::vector<int>& order = {}, int tile = 0);
void free_mac_plan(MacPlan& p);

}  // namespace bcn
