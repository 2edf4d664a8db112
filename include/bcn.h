/*
 * bcn.h -- C ABI of the MI355X ciphertext-branch engine for bi-CryptoNets
 * (arXiv 2402.01296): homomorphic evaluation of the ciphertext branch in
 * RNS-BFV over R_Q = Z_Q[X]/(X^N+1), Q = q_1...q_L.
 *
 * The paper's operation set (appendix "CKKS Scheme"): E, D, Add(c,u),
 * Add(c1,c2), Mult(c,u), Mult(c1,c2), Rot(c,r), with Rot a cyclic left shift
 * of the slot vector by r.  Its layers (appendix "Implementation Details"):
 * HW-packed convolution by rotate / scalar-multiply / sum / mask, sum
 * pooling, fully connected layers; batch packing puts one image per slot.
 * Plaintext-branch features enter by Add(c,u) after a convolution (section
 * "The unidirectional connections"); activations are squares.
 *
 * Conventions
 *  - All functions return 0 (BCN_OK) or a negative BCN_ERR_* code; the
 *    message of the last failure on the calling thread is bcn_last_error().
 *  - A ciphertext at level l (l primes) is caller-owned device memory of
 *    2*l*N doubles, layout [2][l][N]: part, limb, coefficient.  Each entry
 *    is a binary64 holding an integer residue in [0, q_i) of the coefficient
 *    form.  A batch of n ciphertexts is n such blocks back to back.
 *  - Slot vectors are int64 [N]; slot s = rho*N/2 + i sits in row rho,
 *    column i.  Values are taken mod t; decoded values are centred in
 *    (-t/2, t/2).
 *  - Device pointers must be valid for the stream passed; host pointers are
 *    read before the call returns unless stated otherwise.
 *  - Calls on one context must be issued from one host thread on one stream
 *    (or be externally serialised): they share the context's scratch arena.
 *  - Work is ordered on the stream passed.  Layer evaluation may fork part of
 *    its work onto a second stream the context owns (default priority): it
 *    forks after the work already queued on the caller's stream and joins
 *    back into it before returning, so stream order and hipGraph capture of
 *    the caller's stream hold as for single-stream work.
 *  - The secret key lives in client-side objects (bcn_secret_key) used only
 *    by encryption, decryption and key generation; evaluation never sees it.
 */
#ifndef BCN_H
#define BCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* bcn_stream; /* a hipStream_t; NULL = default stream */

enum {
  BCN_OK = 0,
  BCN_ERR_INVALID = -1,  /* bad parameters, sizes or layer description */
  BCN_ERR_LEVEL = -2,    /* level mismatch / not enough primes left */
  BCN_ERR_KEY = -3,      /* a needed relinearisation or Galois key is missing */
  BCN_ERR_NOMEM = -4,    /* device allocation failed */
  BCN_ERR_HIP = -5,      /* HIP runtime error */
  BCN_ERR_INTERNAL = -6
};

typedef struct bcn_context bcn_context;
typedef struct bcn_secret_key bcn_secret_key;
typedef struct bcn_eval_keys bcn_eval_keys;
typedef struct bcn_layer bcn_layer;

/* Scheme parameters.  Primes are chosen by rule: the largest q_bits-bit
 * primes q = 1 mod 2N in descending order (skipping t); the first L form Q,
 * the next K form the special modulus P; internal auxiliary primes follow.
 * Key-switching digits are groups of `alpha` consecutive primes of Q. */
typedef struct {
  uint32_t n;      /* ring degree N: 1024 .. 16384, power of two */
  uint32_t q_bits; /* prime size, 25 .. 41 bits */
  uint32_t L;      /* ciphertext primes, 1 .. 8 */
  uint32_t K;      /* special primes, 1 .. 3 */
  uint32_t alpha;  /* primes per key-switching digit */
  uint64_t t;      /* plaintext modulus: prime < 2^21, t = 1 mod 2N */
} bcn_params;

const char* bcn_last_error(void);

/* Builds the prime tables on `hip_device` (transform twiddles, slot map). */
int bcn_context_create(const bcn_params* p, int hip_device, bcn_context** out);
void bcn_context_destroy(bcn_context* ctx);
/* Writes the primes (Q, then P, then auxiliary) to out[cap]; counts to n_q, n_p, n_aux. */
int bcn_context_primes(const bcn_context* ctx, uint64_t* out, int cap, int* n_q, int* n_p, int* n_aux);

/* ---- client side: keys, E and D (appendix "CKKS Scheme": E(.), D(.)) ---- */

/* s: host int8 [N] ternary secret. */
int bcn_secret_key_create(bcn_context* ctx, const int8_t* s, bcn_secret_key** out);
void bcn_secret_key_destroy(bcn_secret_key* sk);

int bcn_eval_keys_create(bcn_context* ctx, bcn_eval_keys** out);
void bcn_eval_keys_destroy(bcn_eval_keys* ek);

enum { BCN_KEY_RELIN = 0, BCN_KEY_ROTATION = 1 };
/* Generates one key-switching key into ek: kind BCN_KEY_RELIN (s^2 -> s, used
 * by Mult(c1,c2)) or BCN_KEY_ROTATION for a left rotation by `step` (sigma_k(s)
 * -> s, k = g^step mod 2N with g = 3 (BFV) or 5 (CKKS), used by Rot(c, step)); a
 * negative step (> -N/2) is a right rotation and keeps its own key.
 * For digit j: b_j = -a_j s + e_j + P g_j s' mod Q P with g_j = 1 mod the
 * primes of digit j and 0 mod the rest of Q.
 * a: host uint64 [dnum][L+K][N] uniform residues over (Q primes, P primes),
 * e: host int8 [dnum][N] errors; dnum = ceil(L / alpha).  The caller supplies
 * the randomness (from its CSPRNG); the library does not sample. */
int bcn_keygen(bcn_context* ctx, const bcn_secret_key* sk, bcn_eval_keys* ek, int kind, int step,
               const uint64_t* a, const int8_t* e, bcn_stream stream);
/* Copies a key out in coefficient form: host uint64 [dnum][2][L+K][N]. */
int bcn_eval_key_export(bcn_context* ctx, const bcn_eval_keys* ek, int kind, int step, uint64_t* out,
                        bcn_stream stream);

/* E: encodes n slot vectors (host int64 [n][N]) and encrypts each at `level`:
 * c = (-a s + e + round(Q_level [m]_t / t), a).  a: host uint64 [n][level][N]
 * uniform residues, e: host int8 [n][N].  ct_out: device [n][2][level][N]. */
int bcn_encode_encrypt(bcn_context* ctx, const bcn_secret_key* sk, const int64_t* slots, const uint64_t* a,
                       const int8_t* e, int n, int level, double* ct_out, bcn_stream stream);
/* D: m = [round(t [c0 + c1 s]_Q / Q)]_t, decoded to host int64 [n][N] (centred). */
int bcn_decrypt_decode(bcn_context* ctx, const bcn_secret_key* sk, const double* ct, int n, int level,
                       int64_t* slots_out, bcn_stream stream);

/* ---- client side: seeded randomness ----
 * The paper leaves the randomness of keys and encryptions to the scheme
 * (appendix "CKKS Scheme": a uniform, s and e small).  These calls draw it
 * from ChaCha20 keystreams (the block function of RFC 8439, section 2.3) so
 * that a seed fixes every key and ciphertext bit for bit.  Stream
 * (seed, purpose, index): key = seed as 8 little-endian bytes then 24 zero
 * bytes; nonce = the 32-bit words (purpose, index >> 32, index & 0xffffffff);
 * block counter from 0; each 64-bit value is two consecutive little-endian
 * keystream words, low word first.  Samplers (fixed consumption):
 *   ternary   (u mod 3) - 1
 *   uniform q (u_hi 2^64 + u_lo) mod q from two consecutive values
 *   Gaussian  sigma = 3.2 on [-19, 19] by a cumulative table:
 *             T_k = floor(2^64 CDF(k)), k = -19..18; e = -19 + #{k : u >= T_k}
 * Host-only; the result depends on nothing but the arguments. */
enum { BCN_SAMPLE_TERNARY = 0, BCN_SAMPLE_UNIFORM = 1, BCN_SAMPLE_GAUSSIAN = 2 };
enum {
  BCN_PURPOSE_SECRET = 1, /* index 0: the secret key s */
  BCN_PURPOSE_KSK_A = 2,  /* index (key << 32) | (digit (L+K) + prime): a of a key-switching key */
  BCN_PURPOSE_KSK_E = 3,  /* index (key << 32) | digit: its error; key = 0 (relin) or the Galois element k */
  BCN_PURPOSE_ENC_A = 4,  /* index (ct << 32) | prime: a of encryption number ct, residues mod q_prime */
  BCN_PURPOSE_ENC_E = 5   /* index ct << 32: its error */
};
/* Writes n samples of `kind` from stream (seed, purpose, index) to out (host int64 [n]);
 * q is the modulus of BCN_SAMPLE_UNIFORM (2 .. 2^62), ignored otherwise. */
int bcn_sample(int kind, uint64_t seed, uint32_t purpose, uint64_t index, uint64_t q, int n, int64_t* out);
/* The 38 Gaussian thresholds T_k (host uint64 out[38]). */
int bcn_gaussian_table(uint64_t* out);
/* s = ternary from stream (seed, BCN_PURPOSE_SECRET, 0); same object as bcn_secret_key_create. */
int bcn_secret_key_generate(bcn_context* ctx, uint64_t seed, bcn_secret_key** out);
/* bcn_keygen with a_j (residue over prime i of Q then P) uniform from stream
 * (seed, BCN_PURPOSE_KSK_A, (key << 32) | (j (L+K) + i)) and e_j Gaussian from
 * (seed, BCN_PURPOSE_KSK_E, (key << 32) | j); key = 0 for BCN_KEY_RELIN, else
 * the Galois element of `step`.  The host buffers are the library's own. */
int bcn_keygen_seeded(bcn_context* ctx, const bcn_secret_key* sk, bcn_eval_keys* ek, int kind, int step,
                      uint64_t seed, bcn_stream stream);
/* bcn_encode_encrypt (BFV context) or bcn_ckks_encode_encrypt (CKKS context; slots
 * host double [n][N/2] at `scale`) with the randomness of ciphertext r taken from
 * index ct = first + r: a over q_1..q_level uniform from (seed, BCN_PURPOSE_ENC_A,
 * (ct << 32) | i), e Gaussian from (seed, BCN_PURPOSE_ENC_E, ct << 32); first + n
 * must not exceed 2^32. */
int bcn_encrypt_seeded(bcn_context* ctx, const bcn_secret_key* sk, const int64_t* slots, uint64_t seed,
                       uint64_t first, int n, int level, double* ct_out, bcn_stream stream);
int bcn_ckks_encrypt_seeded(bcn_context* ctx, const bcn_secret_key* sk, const double* slots, double scale,
                            uint64_t seed, uint64_t first, int n, int level, double* ct_out, bcn_stream stream);

/* Coefficient-form transfer: host uint64 [n][2][level][N] <-> device ciphertexts. */
int bcn_ct_export(bcn_context* ctx, const double* ct, int n, int level, uint64_t* host_out, bcn_stream stream);
int bcn_ct_import(bcn_context* ctx, const uint64_t* host_in, int n, int level, double* ct, bcn_stream stream);

/* ---- server side: evaluation (no secret key) ---- */

/* Negacyclic NTT of raw limbs in place: data device [n_polys][n_limbs][N] doubles,
 * limb i uses prime id first_prime + i (ids as in bcn_context_primes; the plaintext
 * modulus t has id n_q + n_p + n_aux).  Forward output word p holds a(psi^(2j+1))
 * with j = bitreverse(i), i = (p mod N/16) * 16 + floor(p / (N/16)) (index i is
 * stored at word (i mod 16) * N/16 + floor(i / 16)), psi the smallest x >= 2 with
 * x^N = -1.  inverse != 0 applies the exact inverse (that order in, natural out). */
int bcn_ntt(bcn_context* ctx, double* data, int n_polys, int n_limbs, int first_prime, int inverse,
            bcn_stream stream);

/* Batching across parameter sets: one persistent launch transforms the limbs of
 * several contexts (N = 4096, 8192 or 16384; each with its own primes), e.g.
 * requests of uneven ring degree and prime count.  Item i: data device
 * [n_polys][n_limbs][N] of context ctx, limb j with prime id first_prime + j;
 * the result is exactly bcn_ntt of each item.  At most 16 items, all contexts
 * on one device; calls on overlapping data race. */
typedef struct {
  bcn_context* ctx;
  double* data;
  int32_t n_polys, n_limbs, first_prime;
} bcn_ntt_item;
int bcn_ntt_multi(const bcn_ntt_item* items, int n_items, int inverse, bcn_stream stream);

/* out[o] = sum_j w[o][j] in[j] (Mult(c,u) by scalars, Add(c1,c2)); w host int32 [n_out][n_in].
 * The environment variable BCN_MAC_TILE (a power of two, 1..64) pins the number of
 * outputs per tile; results are the same for every tile size. */
int bcn_mac(bcn_context* ctx, const double* in, int n_in, double* out, int n_out, int level, const int32_t* w,
            bcn_stream stream);
/* Add(c, u): c0 += round(Q_level [m]_t / t), m = encode(slots[i]); slots host int64 [n][N]. */
int bcn_add_plain(bcn_context* ctx, double* ct, int n, int level, const int64_t* slots, bcn_stream stream);
/* Mult(c, u): c_k * lift_c(m), m = encode(slots) (host int64 [N], shared by the n ciphertexts). */
int bcn_mul_plain(bcn_context* ctx, const double* in, double* out, int n, int level, const int64_t* slots,
                  bcn_stream stream);
/* Mult(c, c) + relinearisation (exact BFV tensor and rounding, hybrid key switching);
 * with modswitch != 0 the result is also switched down one prime (level-1 limbs). */
int bcn_square_relin(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, double* out, int n, int level,
                     int modswitch, bcn_stream stream);
/* For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): bcn_square_relin with
 * the same arguments, semantics and bit-identical results, but no allocation,
 * free or allocating library call of any kind.  Its scratch is a fixed 64 MiB
 * array of device memory per GPU, held by the library until the process ends.
 * A call whose scratch would exceed it (about 13 ciphertexts at N = 8192 with
 * four primes, 4 at N = 16384 with six) returns BCN_ERR_INVALID before
 * launching anything.  Every call on one GPU, from any context, stream or host
 * thread, uses that one array, so calls that overlap in time on one GPU race:
 * the caller must serialise them.  Nothing in the array needs to start at zero
 * (every word is written before it is read). */
int bcn_square_relin_noalloc(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, double* out, int n,
                             int level, int modswitch, bcn_stream stream);
/* Rot(c, r) for each input and each step, sharing one digit decomposition per input
 * (hoisting; bit-identical to one-at-a-time).  out device [n_in][n_steps][2][level][N]. */
int bcn_rotate(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, int n_in, int level,
               const int32_t* steps, int n_steps, double* out, bcn_stream stream);
/* In place: c <- sum of Rot(c, r) over r = 0 .. span-1 (span = 2^k >= 2): slot 0 of each
 * row receives the sum of its first span slots (the global sum pooling of appendix
 * "Implementation Details").  Two rounds, each a set of hoisted rotations kept over Q_l P,
 * summed and divided by P once: baby steps 1 .. b-1, then giant steps b, 2b, .., (g-1) b of
 * the first round's result, b = 2^ceil(k/2), g = span / b.  Every step needs its rotation
 * key (bcn_rotate_sum_steps lists them); BCN_ERR_KEY if one is missing. */
int bcn_rotate_sum(bcn_context* ctx, const bcn_eval_keys* ek, double* ct, int n, int level, int span,
                   bcn_stream stream);
/* The rotation steps bcn_rotate_sum(span) uses: writes up to cap of them to steps (may be
 * NULL) and returns their count, or BCN_ERR_INVALID for a span that is not a power of two >= 2. */
int bcn_rotate_sum_steps(int span, int32_t* steps, int cap);
/* Exact modulus switch: c' = (c - lift_c([c]_{q_l})) / q_l mod Q_{l-1}. */
int bcn_modswitch(bcn_context* ctx, const double* in, double* out, int n, int level, bcn_stream stream);

/* ---- layers ---- */
enum { BCN_CONV2D = 0, BCN_DENSE = 1, BCN_POOL = 2 };
enum { BCN_DENSE_WEIGHT_VECTORS = 0, BCN_DENSE_DIAGONAL = 1 };
enum { BCN_PACK_BATCH = 0, BCN_PACK_HW = 1 };

/* One layer of the ciphertext branch: linear part, then (HW conv) the mask of
 * valid outputs, then the optional feature injection, square+relinearisation,
 * modulus switch and (HW) global sum.
 *
 * BATCH packing (slot b = image b): inputs are one ciphertext per input
 *   element in (c, y, x) order; CONV2D outputs one ciphertext per (o, i, j),
 *   b_{o,i,j} = sum_{c,di,dj} w[o][c][di][dj] a_{c, s i+di-p, s j+dj-p};
 *   DENSE: out[o] = sum_j w[o][j] in[j] (also the scalar layer over
 *   ciphertexts that each carry one value).
 * HW packing (one ciphertext per channel, input position (y, x) at slot
 *   pos_stride*(row*y + x)); BHW packing (appendix "Implementation Details",
 *   BHW packing) is HW packing with `batch` images per ciphertext, image b's
 *   positions offset by base(b) = (b mod P) * block + floor(b / P) * N/2,
 *   P = (N/2) / block (blocks fill slot row 0, then row 1): CONV2D (valid, pad 0) rotates each input by
 *   pos_stride*(row*di + dj), multiplies by w[o][c][di][dj], sums and keeps the
 *   outputs at slots pos_stride*stride*(row*i + j) with a mask; DENSE weights
 *   w[o][c*in_h*in_w + y*in_w + x] multiply the slot of (y, x) of input c,
 *   products are summed and then summed over slots (rotate-and-sum), leaving
 *   out[o] in slot 0.  DENSE with method BCN_DENSE_DIAGONAL (appendix
 *   "Implementation Details", fully connected layer): each input channel holds
 *   its n1 = in_h*in_w inputs at slots 0..n1-1 (pos_stride 1, in_w = row or
 *   in_h = 1); for r = 1-n2 .. n1-1 (n2 = out_c; n1 + n2 - 1 hoisted rotations)
 *   Rot(in[c], r) is multiplied by the vector whose slot j holds
 *   w[j][c*n1 + j + r] (0 where j + r falls outside 0..n1-1) and everything is
 *   summed: one output ciphertext with out[j] in slot j.  POOL (local sum
 *   pooling, "similar to the convolution without weights"): channel by channel,
 *   the sum of each k x k window at the stride, then the mask; in_c = out_c,
 *   weights unused.
 * Features (has_features): FP32 device array; q(f) = clamp(rint(scale f),
 *   -clamp, clamp) in FP32 arithmetic is added as a plaintext.  BATCH: layout
 *   [batch][n_out] (image-major); HW: [out_c][oh][ow]; BHW: [out_c][batch][oh][ow].
 */
typedef struct {
  int32_t kind;          /* BCN_CONV2D or BCN_DENSE */
  int32_t packing;       /* BCN_PACK_BATCH or BCN_PACK_HW */
  int32_t in_c, in_h, in_w;
  int32_t out_c;
  int32_t k, stride, pad;/* CONV2D geometry (HW: pad must be 0) */
  int32_t row;           /* HW: slots per image row */
  int32_t pos_stride;    /* HW: spacing of the valid input positions */
  const int32_t* weights;/* host; CONV2D [out_c][in_c][k][k], DENSE [out_c][in_c*in_h*in_w] */
  int32_t has_features;
  float feature_scale;   /* 8.0 in the three workloads */
  int32_t feature_clamp; /* 127 */
  int32_t batch;         /* BATCH: images (slots) carrying data; HW with block > 0: images per ciphertext */
  int32_t square;        /* square + relinearise after the linear part (+features) */
  int32_t modswitch;     /* after the square, switch down one prime (needs level >= 2) */
  int32_t sum;           /* HW CONV2D: nonzero = global sum of each output map, left in slot 0;
                            BATCH DENSE (scalar weights): 0, or a span S (power of two): each
                            output is then rotated-and-summed over S slots (a global sum moved
                            after the dense layer, which commutes with it) */
  int32_t block;         /* HW: 0 (one image at base 0), or the slot distance between the blocks of
                            `batch` images packed in one ciphertext (BHW packing) */
  int32_t method;        /* HW DENSE: BCN_DENSE_WEIGHT_VECTORS (default) or BCN_DENSE_DIAGONAL */
  int32_t defer_relin;   /* BATCH with square: 1 = leave the square unrelinearised, out rows are
                            [3][level_out][N] (d0, d1, d2: decrypts as d0 + d1 s + d2 s^2) */
  int32_t in_parts;      /* BATCH: 2 (0 = 2), or 3 when the inputs are such unrelinearised products:
                            the layer's weighted sums run over the three parts and each output is
                            relinearised once before the rest of the layer */
} bcn_layer_desc;

/* Prepares a layer for inputs at `level`: uploads weights, encodes masks and
 * weight vectors, fixes the rotation steps.  The keys must hold every Galois
 * key the layer needs (bcn_layer_rotation_steps lists them). */
int bcn_layer_create(bcn_context* ctx, const bcn_layer_desc* desc, int level, bcn_layer** out);
void bcn_layer_destroy(bcn_layer* layer);
/* Rotation steps the layer uses; returns the count (or an error), writes up to cap. */
int bcn_layer_rotation_steps(const bcn_layer* layer, int32_t* steps, int cap);
/* Input/output ciphertext counts and the output level. */
int bcn_layer_shape(const bcn_layer* layer, int* n_in, int* n_out, int* level_out);
/* Parts per input and per output row: 2, or 3 for unrelinearised products (desc in_parts,
 * defer_relin). */
int bcn_layer_parts(const bcn_layer* layer, int* in_parts, int* out_parts);
/* Evaluates the layer: in device [n_in][in_parts][level][N] -> out device
 * [n_out][out_parts][level_out][N] (parts 2 unless deferred relinearisation is asked for);
 * features: device float or NULL when the layer has none. */
int bcn_layer_eval(bcn_context* ctx, const bcn_eval_keys* ek, const bcn_layer* layer, const double* in,
                   double* out, const float* features, bcn_stream stream);
/* The same layer over n_requests independent requests in one set of launches:
 * in [n_requests][n_in][in_parts][level][N], out [n_requests][n_out][out_parts][level_out][N],
 * features [n_requests][...] in the per-request layout above.  Request r's
 * results are bit-identical to evaluating it alone.  From the second call of
 * a shape on it issues no host synchronisation, allocation or memset, so it
 * can then be captured into a hipGraph (the first call may grow the context's
 * scratch arena, the second consolidates it into one block). */
int bcn_layer_eval_batch(bcn_context* ctx, const bcn_eval_keys* ek, const bcn_layer* layer, const double* in,
                         double* out, const float* features, int n_requests, bcn_stream stream);

/* ---- tuning ---- */
/* Times the candidate transform shapes (registers per thread, hence LDS passes
 * per transform) on this device and keeps the fastest for the context.  A text
 * report of the timings is written to report[cap] (may be NULL).  Results are
 * unaffected: every shape computes the same exact transform. */
int bcn_autotune(bcn_context* ctx, char* report, int cap, bcn_stream stream);
/* Times the layer's multiply-accumulate with each candidate output-tile size and
 * keeps the fastest (exact for every tile size). */
int bcn_layer_autotune(bcn_context* ctx, bcn_layer* layer, char* report, int cap, bcn_stream stream);

/* ---- measurement ---- */
/* While enabled, launches of the main kernels are bracketed by hipEvents on
 * their stream and their algorithmic HBM bytes are accumulated per kernel
 * name (ntt_forward, ntt_inverse, mac, extend_qb, scale_round, modup,
 * ks_inner, moddown, tensor_square). */
int bcn_profile_enable(bcn_context* ctx, int on);
/* Resolves and clears the recorded timings (synchronises their events).  Writes
 * newline-separated kernel names into names[names_cap] and, per name, the launch
 * count, summed launch time (ms), algorithmic HBM bytes and algorithmic FP64 VALU
 * lane operations (0 where not tracked; ops may be NULL) into the arrays (cap
 * entries).  Returns the number of names, or an error code. */
int bcn_profile_read(bcn_context* ctx, char* names, int names_cap, int* launches, double* total_ms, double* bytes,
                     double* ops, int cap);

/* ---- CKKS: the paper's scheme (section "Experiments": CKKS with N = 2^14;
 * appendix "CKKS Scheme") on the same RNS rings, transforms, keys and key
 * switching.  A ciphertext [2][l][N] (same layout as above) holds N/2 real
 * slot values at a scale Delta the caller tracks: slot i sits at the
 * evaluation point zeta^(5^i mod 2N), zeta = exp(i pi / N).  Rot(c, r)
 * (bcn_rotate, bcn_rotate_sum) shifts the N/2 slots left by r; keys come from
 * bcn_keygen (relinearisation key s^2 -> s, rotation keys with k = 5^r).
 * bcn_mac multiplies by integer scalars (the scale is unchanged);
 * bcn_modswitch is the rescale (exact nearest division by the last prime:
 * the scale divides by that prime).  The BFV-only calls (bcn_encode_encrypt,
 * bcn_decrypt_decode, bcn_add_plain, bcn_mul_plain, bcn_square_relin*,
 * bcn_layer_create) refuse a CKKS context with BCN_ERR_INVALID. */

/* A CKKS context: p->t is ignored (no plaintext modulus). */
int bcn_context_create_ckks(const bcn_params* p, int hip_device, bcn_context** out);
/* Encoding: slots device double [n][N/2] (real) -> round(scale * m), m the real
 * polynomial with m(zeta^(5^i)) = z_i, as residues over Q_level: out device
 * [n][level][N], coefficient form, or transformed (bcn_ntt order) when
 * ntt_domain != 0.  Requires scale in (0, 2^52) and |scale * m_k| < 2^52. */
int bcn_ckks_encode(bcn_context* ctx, const double* slots, int n, int level, double scale, int ntt_domain,
                    double* out, bcn_stream stream);
/* E: encodes host slots [n][N/2] at `scale` and encrypts at `level`:
 * c = (-a s + e + m, a); a: host uint64 [n][level][N], e: host int8 [n][N]. */
int bcn_ckks_encode_encrypt(bcn_context* ctx, const bcn_secret_key* sk, const double* slots, double scale,
                            const uint64_t* a, const int8_t* e, int n, int level, double* ct_out, bcn_stream stream);
/* D: m = lift_c([c0 + c1 s]_Q), decoded: slots_out host double [n][N/2] = m(zeta^(5^i)) / scale (real parts). */
int bcn_ckks_decrypt_decode(bcn_context* ctx, const bcn_secret_key* sk, const double* ct, int n, int level,
                            double scale, double* slots_out, bcn_stream stream);
/* Add(c, u): c0 += pt for each ciphertext, pt device [n][level][N] coefficient residues
 * (bcn_ckks_encode at the ciphertext's scale). */
int bcn_ckks_add_plain(bcn_context* ctx, double* ct, int n, int level, const double* pt, bcn_stream stream);
/* Mult(c, u): out = in * pt, pt device [level][N] transformed (bcn_ckks_encode with
 * ntt_domain), shared by the n ciphertexts; the scales multiply. */
int bcn_ckks_mul_plain(bcn_context* ctx, const double* in, double* out, int n, int level, const double* pt_ntt,
                       bcn_stream stream);
/* Mult(c, c): the exact tensor mod Q_level, relinearised, then rescaled by q_level:
 * in [n][2][level][N] at scale D -> out [n][2][level-1][N] at scale D^2 / q_level. */
int bcn_ckks_square_relin_rescale(bcn_context* ctx, const bcn_eval_keys* ek, const double* in, double* out, int n,
                                  int level, bcn_stream stream);

/* ---- scratch arena ----
 * Each context owns a grow-only device scratch arena used by every call.  When
 * a call outgrows it, the next call moves to one larger block; the blocks it
 * replaces are retired, not freed, because a hipGraph captured earlier may
 * still use them.  Retired blocks are freed only by bcn_scratch_release or
 * bcn_context_destroy. */
/* Current block's device address, a counter that changes whenever the block
 * changes, its size, the most scratch any one call has used since the previous
 * bcn_scratch_info (the mark restarts at each query), and the bytes held by
 * retired blocks.  Any output pointer may be NULL. */
int bcn_scratch_info(bcn_context* ctx, uint64_t* base, uint64_t* generation, size_t* bytes, size_t* high_bytes,
                     size_t* retired_bytes);
/* Frees the retired blocks (synchronises the device first).  The caller must
 * hold no captured graph that was recorded before the last block change. */
int bcn_scratch_release(bcn_context* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BCN_H */
