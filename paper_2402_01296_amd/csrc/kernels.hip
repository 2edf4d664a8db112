// Element-wise and per-coefficient kernels of the ciphertext branch.
//
// Layout: every RNS buffer is limb-major, [..][limb][N] binary64 residues in
// [0, q).  Per-coefficient kernels (base conversion, rounding, modulus
// switching) give one thread one coefficient of one polynomial and read its
// limbs at stride N, so consecutive threads touch consecutive words.
#include "convert.h"

namespace bcn {
namespace {

constexpr int TPB = 256;

inline unsigned nblocks(size_t work) { return (unsigned)((work + TPB - 1) / TPB); }

// ------------------------------------------------------------------ MAC

// out[rows[tile*TO + o]] = sum over the tile's column entries e of Wp[e][o] * in[cols[e]].
// Wp holds, per column entry, the TO weights of the tile contiguously, so the
// uniform weights of one column arrive as a few wide scalar loads.  Every partial
// sum is an exact FP64 integer: with CENTRE, inputs are centred (|x| <= (q-1)/2)
// and `chunk` bounds the inputs between two partial reductions; without it (the
// plan has checked that a whole tile's sum of |w| * (q-1) stays below 2^53) the
// residues in [0, q) are accumulated as they are, with no reduction until the end.
// Optional plaintext add folded into the MAC's stores (the unidirectional feature
// connection): part 0 of output row r gains round(Q_level m_r / t) for the encoded
// plaintext m_r (msg[r][N], values mod t), exactly as the separate Add(c, u) kernel.
struct DeltaAdd {
  const double* msg = nullptr;  // [requests][rows][N]; null: no add
  size_t msg_req = 0;           // words between requests
  double qmodt = 0.0;           // Q_level mod t
  Mod mt{};                     // t
  double negtinv[kMaxBasis];    // -t^-1 mod q_i
  const double* mulpt = nullptr;  // [limbs][N] transform-domain plaintext multiplied into every output word
};

// Four inputs of a MAC column list: word w of inputs cols[0..3] (xin = in + w).
__device__ __forceinline__ void mac_load4(double (&x)[4], const double* __restrict__ xin, const int* __restrict__ cols,
                                          int words) {
#pragma unroll
  for (int u = 0; u < 4; ++u) x[u] = xin[(size_t)cols[u] * words];
}

// acc[o] += wr[u * TO + o] * x[u] over a group of four inputs (exact FP64 integer sums; with
// CENTRE the inputs are centred and the partial sums reduced before `chunk` inputs accumulate).
template <int TO, bool CENTRE>
__device__ __forceinline__ void mac_group4(double (&acc)[TO], const double (&x)[4], const double* wr,
                                           int& cnt, int chunk, Mod m, double halfq) {
  if (CENTRE && cnt > chunk - 4) {
#pragma unroll
    for (int o = 0; o < TO; ++o) acc[o] = reduce_lazy(acc[o], m);
    cnt = 0;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double xv = CENTRE && x[u] > halfq ? x[u] - m.q : x[u];
#pragma unroll
    for (int o = 0; o < TO; ++o) acc[o] = fma(wr[u * TO + o], xv, acc[o]);
  }
  cnt += 4;
}

template <int TO, bool CENTRE>
__global__ void __launch_bounds__(TPB)
k_mac(const double* __restrict__ in, double* __restrict__ out, int words, int logn, int level,
      const double* __restrict__ Wp, const int* __restrict__ rows, const int* __restrict__ tptr,
      const int* __restrict__ tcols, int chunk, Basis b, const Mod* __restrict__ mods, size_t in_req,
      size_t out_req, size_t out_ct, size_t out_part, DeltaAdd da) {
  // word-block-major work list walked per XCD (the tiles of one block of words read the same
  // inputs and share that XCD's L2); dispatch order is x fastest
  const int wq = xcd_order(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bx = wq / gridDim.y, tile = wq - bx * gridDim.y;
  const int w = bx * TPB + threadIdx.x;
  if (w >= words) return;
  in += blockIdx.z * in_req;     // request blockIdx.z of a batch of independent requests
  out += blockIdx.z * out_req;
  const Mod m = mods[b.id[(w >> logn) % level]];
  const double halfq = (m.q - 1.0) * 0.5;
  double acc[TO];
#pragma unroll
  for (int o = 0; o < TO; ++o) acc[o] = 0.0;
  const int beg = tptr[tile], end = tptr[tile + 1];
  const double* __restrict__ xin = in + w;
  int cnt = 0;
  int e = beg;
  if constexpr (TO <= 16) {
    // Inputs go in groups of four through two register buffers: the loads of the next group
    // are issued before the products of the current one, so one group's memory latency
    // overlaps the other's FMAs.  Wider tiles keep the plain loop: one input's weights already
    // fill 2 * TO scalar registers, and the second buffer's addresses push them into spills
    // (and a scratch segment, which costs the launch its occupancy).
    double xa[4], xb[4];
    if (e + 4 <= end) mac_load4(xa, xin, tcols + e, words);   // invariant: xa holds group e whenever e + 4 <= end
    for (; e + 8 <= end; e += 8) {
      mac_load4(xb, xin, tcols + e + 4, words);
      __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the products
      mac_group4<TO, CENTRE>(acc, xa, Wp + (size_t)e * TO, cnt, chunk, m, halfq);
      // unconditional (a repeat of group e at the end): a branch here lets the compiler sink
      // the products below it and keep every weight of the group live in scalar registers
      mac_load4(xa, xin, tcols + (e + 12 <= end ? e + 8 : e), words);
      __builtin_amdgcn_sched_barrier(0);
      mac_group4<TO, CENTRE>(acc, xb, Wp + (size_t)(e + 4) * TO, cnt, chunk, m, halfq);
    }
    if (e + 4 <= end) {
      mac_group4<TO, CENTRE>(acc, xa, Wp + (size_t)e * TO, cnt, chunk, m, halfq);
      e += 4;
    }
  } else {
    for (; e + 4 <= end; e += 4) {
      if (CENTRE && cnt > chunk - 4) {
#pragma unroll
        for (int o = 0; o < TO; ++o) acc[o] = reduce_lazy(acc[o], m);
        cnt = 0;
      }
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = xin[(size_t)tcols[e + u] * words];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double xv = CENTRE && x[u] > halfq ? x[u] - m.q : x[u];
        const double* __restrict__ wr = Wp + (size_t)(e + u) * TO;
#pragma unroll
        for (int o = 0; o < TO; ++o) acc[o] = fma(wr[o], xv, acc[o]);
      }
      cnt += 4;
    }
  }
  for (; e < end; ++e) {
    if (CENTRE && cnt >= chunk) {
#pragma unroll
      for (int o = 0; o < TO; ++o) acc[o] = reduce_lazy(acc[o], m);
      cnt = 0;
    }
    double x = xin[(size_t)tcols[e] * words];
    if (CENTRE) x = x > halfq ? x - m.q : x;
    const double* __restrict__ wr = Wp + (size_t)e * TO;
#pragma unroll
    for (int o = 0; o < TO; ++o) acc[o] = fma(wr[o], x, acc[o]);
    ++cnt;
  }
  const bool add_part = w < (words >> 1);                             // part 0 words
  const bool add = da.msg != nullptr && add_part;
  const int limb = (w >> logn) % level;
  const size_t k = (size_t)w & (((size_t)1 << logn) - 1);
  const double pmul = da.mulpt ? da.mulpt[((size_t)limb << logn) + k] : 0.0;
#pragma unroll
  for (int o = 0; o < TO; ++o) {
    const int row = rows[tile * TO + o];
    if (row < 0) continue;
    double r = reduce(acc[o], m);
    if (da.mulpt) r = mul_mod(r, pmul, m);
    if (add) {
      const double mv = da.msg[blockIdx.z * da.msg_req + ((size_t)row << logn) + k];
      const double rt = mul_mod(da.qmodt, mv, da.mt);                 // [Q m]_t
      double d = norm(mul_lazy(rt, da.negtinv[limb], m), m);         // floor(Q m / t) mod q
      if (2.0 * rt > da.mt.q) d = add_mod(d, 1.0, m);                 // nearest, never a tie (t odd)
      r = add_mod(r, d, m);
    }
    out[(size_t)row * out_ct + (add_part ? 0 : out_part) + (size_t)(add_part ? w : w - (words >> 1))] = r;
  }
}

// The same MAC feeding a square (slot batching): thread (part, coefficient k) accumulates all
// NQ limbs of the tile's TO outputs, so after the reduction (and the feature add on part 0) it
// holds every residue of the coefficient and writes the B limbs of its centred lift too (the
// steps of k_extend_qb): out row r is [2][NQ + m][N] over Q_level then B.  Uncentred plans only.
// The NQ limbs of input `col` at coefficient k (xin = in + part * NQ * N + k).
template <int NQ>
__device__ __forceinline__ void qb_load(double (&x)[NQ], const double* __restrict__ xin, int col, size_t words,
                                        size_t N) {
#pragma unroll
  for (int l = 0; l < NQ; ++l) x[l] = xin[(size_t)col * words + (size_t)l * N];
}

template <int TO, int NQ>
__device__ __forceinline__ void qb_input(double (&acc)[TO][NQ], const double (&x)[NQ], const double* __restrict__ wr) {
#pragma unroll
  for (int o = 0; o < TO; ++o)
#pragma unroll
    for (int l = 0; l < NQ; ++l) acc[o][l] = fma(wr[o], x[l], acc[o][l]);
}

template <int TO, int NQ>
__global__ void __launch_bounds__(TPB)
k_mac_qb(const double* __restrict__ in, double* __restrict__ out, int logn, const double* __restrict__ Wp,
         const int* __restrict__ rows, const int* __restrict__ tptr, const int* __restrict__ tcols, Basis b,
         const Mod* __restrict__ mods, size_t in_req, size_t out_req, size_t out_ct, size_t out_part, DeltaAdd da,
         const Conv* __restrict__ cvp) {
  const size_t N = (size_t)1 << logn;
  // (the word-block-major order of k_mac measured slower here: dispatch order is kept)
  const size_t w = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (w >= 2 * N) return;
  in += blockIdx.z * in_req;
  out += blockIdx.z * out_req;
  const int tile = blockIdx.y;
  const int part = (int)(w >> logn);
  const size_t k = w & (N - 1);
  const size_t words = 2 * NQ * N;
  double acc[TO][NQ];
#pragma unroll
  for (int o = 0; o < TO; ++o)
#pragma unroll
    for (int l = 0; l < NQ; ++l) acc[o][l] = 0.0;
  const double* __restrict__ xin = in + (size_t)part * NQ * N + k;
  const int beg = tptr[tile], end = tptr[tile + 1];
  int e = beg;
  // One input (its NQ limbs) per register buffer, two buffers: the next input's loads are in
  // flight while the current one's products run.
  double xa[NQ], xb[NQ];
  if (e < end) qb_load(xa, xin, tcols[e], words, N);   // invariant: xa holds input e whenever e < end
  for (; e + 2 <= end; e += 2) {
    qb_load(xb, xin, tcols[e + 1], words, N);
    __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the products
    qb_input<TO, NQ>(acc, xa, Wp + (size_t)e * TO);
    qb_load(xa, xin, tcols[e + 3 <= end ? e + 2 : e], words, N);   // unconditional, as in k_mac
    __builtin_amdgcn_sched_barrier(0);
    qb_input<TO, NQ>(acc, xb, Wp + (size_t)(e + 1) * TO);
  }
  if (e < end) qb_input<TO, NQ>(acc, xa, Wp + (size_t)e * TO);
  const Conv& cv = *cvp;
  const bool add = da.msg != nullptr && part == 0;
#pragma unroll
  for (int o = 0; o < TO; ++o) {
    const int row = rows[tile * TO + o];
    if (row < 0) continue;
    double r[NQ], v[NQ];
    double rt = 0.0;
    if (add) rt = mul_mod(da.qmodt, da.msg[blockIdx.z * da.msg_req + ((size_t)row << logn) + k], da.mt);  // [Q m]_t
    double* dst = out + (size_t)row * out_ct + (size_t)part * out_part + k;
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
      const Mod m = mods[b.id[l]];
      double x = reduce(acc[o][l], m);
      if (add) {
        double d = norm(mul_lazy(rt, da.negtinv[l], m), m);           // floor(Q m / t) mod q
        if (2.0 * rt > da.mt.q) d = add_mod(d, 1.0, m);                // nearest, never a tie (t odd)
        x = add_mod(x, d, m);
      }
      r[l] = x;
      dst[(size_t)l * N] = x;
    }
    garner<NQ>(r, v, cv, mods);
    const bool neg = above_half<NQ>(v, NQ, cv, mods);
    for (int d = 0; d < cv.nd; ++d) {
      const Mod md = mods[cv.dst[d]];
      double a = v[NQ - 1];
#pragma unroll
      for (int kk = NQ - 2; kk >= 0; --kk) a = mul_lazy(a, cv.pm[d][kk], md) + v[kk];
      if (neg) a -= cv.Mmod[d];
      dst[(size_t)(NQ + d) * N] = reduce(a, md);
    }
  }
}

// ------------------------------------------------------------------ plaintext ops

struct LimbConsts {
  double v[kMaxBasis];
};

__global__ void k_add_delta(double* __restrict__ ct, int n, int level, int logn, const double* __restrict__ msg,
                            double qmodt, Mod mt, Basis b, const Mod* __restrict__ mods, LimbConsts negtinv) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * level * N) return;
  const size_t ci = idx / (level * N);
  const int limb = (int)((idx >> logn) % level);
  const size_t k = idx & (N - 1);
  const double r = mul_mod(qmodt, msg[ci * N + k], mt);          // [Q m]_t
  const Mod mq = mods[b.id[limb]];
  double d = norm(mul_lazy(r, negtinv.v[limb], mq), mq);         // floor(Q m / t) mod q
  if (2.0 * r > mt.q) d = add_mod(d, 1.0, mq);                   // nearest, never a tie (t odd)
  double* p = ct + ci * 2 * level * N + (size_t)limb * N + k;   // part 0
  *p = add_mod(*p, d, mq);
}

__global__ void k_mul_plain(const double* __restrict__ in, double* __restrict__ out, int n, int level, int logn,
                            const double* __restrict__ pt, int per_ct, Basis b, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * 2 * level * N) return;
  const size_t ci = idx / (2 * level * N);
  const size_t lk = idx % (level * N);                            // limb*N + k
  const Mod m = mods[b.id[lk >> logn]];
  const double p = pt[(per_ct ? ci * level * N : 0) + lk];
  out[idx] = mul_mod(in[idx], p, m);
}

// P c^ on the Q limbs, 0 on the P limbs (tap 0 of the extended taps)
__global__ void k_ext_tap0(const double* __restrict__ chat, int n, int level, int nb, int logn, KsExt ext, Basis b,
                           const Mod* __restrict__ mods, double* __restrict__ X, size_t out_outer) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * 2 * nb * N) return;
  const size_t i = idx / (2 * nb * N);
  const size_t r = idx % (2 * nb * N);
  const int part = (int)(r / (nb * N));
  const int limb = (int)((r >> logn) % nb);
  const size_t k = idx & (N - 1);
  double v = 0.0;
  if (limb < level) v = mul_mod(chat[(i * 2 + part) * level * N + (size_t)limb * N + k], ext.pm[limb], mods[b.id[limb]]);
  X[i * out_outer + r] = v;
}

__global__ void k_sum_slabs(const double* __restrict__ in, int slabs, size_t words, int nb, int logn, Basis b,
                            const Mod* __restrict__ mods, double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= words) return;
  const Mod m = mods[b.id[(idx >> logn) % nb]];
  double a = 0.0;                       // slabs <= 2^11 residues below 2^41: exact
  for (int k = 0; k < slabs; ++k) a += in[(size_t)k * words + idx];
  out[idx] = reduce(a, m);
}

__global__ void k_ptvec_mac(const double* __restrict__ in, int n_in, double* __restrict__ out, int n_out,
                            int level, int logn, const double* __restrict__ pt, Basis b,
                            const Mod* __restrict__ mods, int requests) {
  const size_t N = (size_t)1 << logn;
  const size_t words = 2 * level * N;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)requests * n_out * words) return;
  const size_t kr = idx / words, w = idx % words;
  const size_t req = kr / n_out, ko = kr % n_out;
  const size_t lk = w % (level * N);
  const Mod m = mods[b.id[lk >> logn]];
  const double* inr = in + req * n_in * words;
  double acc = 0.0;
  for (int cc = 0; cc < n_in; ++cc) {
    acc += mul_lazy(inr[(size_t)cc * words + w], pt[(ko * n_in + cc) * level * N + lk], m);
    if ((cc & 1023) == 1023) acc = reduce_lazy(acc, m);
  }
  out[idx] = reduce(acc, m);
}

__global__ void k_tensor_square(const double* __restrict__ in, double* __restrict__ out, int n, int nb, int logn,
                                Basis b, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * nb * N) return;
  const size_t ci = idx / (nb * N), lk = idx % (nb * N);
  const Mod m = mods[b.id[lk >> logn]];
  const double a0 = in[(ci * 2) * nb * N + lk], a1 = in[(ci * 2 + 1) * nb * N + lk];
  const double x = mul_mod(a0, a1, m);
  out[(ci * 3) * nb * N + lk] = mul_mod(a0, a0, m);
  out[(ci * 3 + 1) * nb * N + lk] = add_mod(x, x, m);
  out[(ci * 3 + 2) * nb * N + lk] = mul_mod(a1, a1, m);
}

// ------------------------------------------------------------------ exact base conversions

// [n][2][level][N] over Q_level -> [n][2][level+m][N] over Q_level then B (centred lift)
template <int NS>
__global__ void __launch_bounds__(TPB)
k_extend_qb(const double* in, double* out, int npoly, int logn, int in_place, const Conv* __restrict__ cvp,
            const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)npoly * N) return;
  const Conv& cv = *cvp;
  const size_t poly = idx >> logn, k = idx & (N - 1);
  const int nd = cv.nd;
  double* dst = out + poly * (NS + nd) * N + k;
  // in place: the Q limbs are already the first NS limbs of each output polynomial
  const double* src = in_place ? dst : in + poly * NS * N + k;
  double x[NS], v[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    x[i] = src[i * N];
    if (!in_place) dst[i * N] = x[i];
  }
  garner<NS>(x, v, cv, mods);
  const bool neg = above_half<NS>(v, NS, cv, mods);
  for (int d = 0; d < nd; ++d) {
    const Mod md = mods[cv.dst[d]];
    double acc = v[NS - 1];
#pragma unroll
    for (int kk = NS - 2; kk >= 0; --kk) acc = mul_lazy(acc, cv.pm[d][kk], md) + v[kk];
    if (neg) acc -= cv.Mmod[d];
    dst[(NS + d) * N] = reduce(acc, md);
  }
}

// round(t x / Q_level) mod q_d, d < nq, for one coefficient x given by its NS residues
// src[i * N] over Q_level then B (x centred, |x| < Q_level B / 2).
// cv.src = Q_level + B, cv.dst = Q_level, cv.pm[d][k] = src_k mod q_d, cv.aux[d] = B mod q_d,
// cv.aux2[0] = t.
template <int NS>
__device__ __forceinline__ void scale_round_coeff(const double* __restrict__ src, size_t N, int nq, const Conv& cv,
                                                  const Mod* __restrict__ mods, double (&res)[NS]) {
  const double t = cv.aux2[0];
  double x[NS], v[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = src[i * N];
  garner<NS>(x, v, cv, mods);
  const bool neg = above_half<NS>(v, NS, cv, mods);
  // t * r = sum_k w_k M_k + c * Q_level over the Q digits (exact carry chain)
  double c = 0.0;
  double wdig[NS];
#pragma unroll
  for (int kk = 0; kk < NS; ++kk) {
    if (kk < nq) {
      const Mod mk = mods[cv.src[kk]];
      double quo;
      wdig[kk] = mul_add_divmod(t, v[kk], c, mk, &quo);
      c = quo;
    } else {
      wdig[kk] = 0.0;
    }
  }
  const bool up = above_half<NS>(wdig, nq, cv, mods);
  const double R = c + (up ? 1.0 : 0.0);                          // round(t r / Q) in [0, t]
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    if (d >= nq) break;
    const Mod md = mods[cv.dst[d]];
    // K = floor(x / Q) from the B digits, minus B when the centred value is negative
    double acc = v[NS - 1];
#pragma unroll
    for (int kk = NS - 2; kk >= 0; --kk)
      if (kk >= nq) acc = mul_lazy(acc, cv.pm[d][kk], md) + v[kk];
    if (neg) acc -= cv.aux[d];
    const double y = mul_lazy(t, reduce(acc, md), md) + R;
    res[d] = reduce(y, md);
  }
}

// [n][3][level+m][N] (Q_level then B) -> [n*][level][N]: round(t x / Q_level) mod q_i for the
// polynomials poly_mul * i + poly_add of the input (1, 0: all three parts; 3, 2: only part 2).
template <int NS>
__global__ void __launch_bounds__(TPB)
k_scale_round(const double* __restrict__ in, double* __restrict__ out, int npoly, int logn, int nq, int poly_mul,
              int poly_add, const Conv* __restrict__ cvp, const Mod* __restrict__ mods, int modsw, LimbConsts linv) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)npoly * N) return;
  const size_t poly = idx >> logn, k = idx & (N - 1);
  double res[NS];
  scale_round_coeff<NS>(in + (poly * poly_mul + poly_add) * NS * N + k, N, nq, *cvp, mods, res);
  if (modsw) {
    // then drop q_{nq-1}: (r - lift_c([r]_{q_last})) / q_last, as the modulus switch
    const Conv& cv = *cvp;
    const Mod ml = mods[cv.dst[nq - 1]];
    const double last = res[nq - 1];
    const double lc = last > (ml.q - 1.0) * 0.5 ? last - ml.q : last;
    double* dst = out + poly * (nq - 1) * N + k;
#pragma unroll
    for (int d = 0; d < NS; ++d) {
      if (d >= nq - 1) break;
      const Mod md = mods[cv.dst[d]];
      dst[d * N] = norm(mul_lazy(res[d] - lc, linv.v[d], md), md);
    }
    return;
  }
  double* dst = out + poly * nq * N + k;
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    if (d >= nq) break;
    dst[d * N] = res[d];
  }
}

// digit j of x [n][level][N]: centred residue over the digit's primes, raised to Q_level + P.
// cv.src = digit primes (NS of them), cv.dst = Q_level + P; cv.aux[d] = 1 when dst d is in the digit
// (then the value is copied), with the source limb index in cv.aux2[d].
template <int NS>
__global__ void __launch_bounds__(TPB)
k_modup(const double* __restrict__ in, size_t in_stride, double* __restrict__ out, int npoly, int logn, int digit,
        int dnum, const Conv* __restrict__ cvp, const Mod* __restrict__ mods, int first_limb) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)npoly * N) return;
  const Conv& cv = *cvp;
  const size_t poly = idx >> logn, k = idx & (N - 1);
  const double* src = in + poly * in_stride + k;
  double x[NS], v[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = src[(first_limb + i) * N];
  garner<NS>(x, v, cv, mods);
  const bool neg = above_half<NS>(v, NS, cv, mods);
  const int nd = cv.nd;
  double* dst = out + (poly * dnum + digit) * nd * N + k;
  for (int d = 0; d < nd; ++d) {
    if (cv.aux[d] != 0.0) {
      dst[d * N] = x[(int)cv.aux2[d]];
      continue;
    }
    const Mod md = mods[cv.dst[d]];
    double acc = v[NS - 1];
#pragma unroll
    for (int kk = NS - 2; kk >= 0; --kk) acc = mul_lazy(acc, cv.pm[d][kk], md) + v[kk];
    if (neg) acc -= cv.Mmod[d];
    dst[d * N] = reduce(acc, md);
  }
}



__global__ void __launch_bounds__(TPB)
k_ks_inner(const double* __restrict__ D, KeySel ka, int n, int d_div, int level, int nb, int dnum, int L,
           int logn, Basis b, const Mod* __restrict__ mods, double* __restrict__ out) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * nb * N) return;
  const size_t o = idx / (nb * N);
  const int limb = (int)((idx >> logn) % nb);
  const int k = (int)(idx & (N - 1));
  const Mod m = mods[b.id[limb]];
  const int sel = (int)(o % ka.nk);
  const int g = ka.keys ? ka.galois[sel] : ka.galois1;
  // positions are in transform-domain storage order; the permutation acts on transform indices
  const int src = g == 1 ? k : ntt_store(ntt_perm(ntt_index(k, logn), g, logn), logn);
  const double* dd = D + (o / d_div) * dnum * nb * N + (size_t)limb * N + src;
  const double* key = ka.keys ? ka.keys[sel] : ka.key1;
  const int klimb = limb < level ? limb : L + (limb - level);
  const int KL = nb - level + L;                                   // limbs of a key part (L + K)
  double a0 = 0.0, a1 = 0.0;
  for (int j = 0; j < dnum; ++j) {
    const double dj = dd[(size_t)j * nb * N];
    a0 += mul_lazy(dj, key[((size_t)(j * 2) * KL + klimb) * N + k], m);
    a1 += mul_lazy(dj, key[((size_t)(j * 2 + 1) * KL + klimb) * N + k], m);
  }
  out[(o * 2) * nb * N + (size_t)limb * N + k] = reduce(a0, m);
  out[(o * 2 + 1) * nb * N + (size_t)limb * N + k] = reduce(a1, m);
}

// gather form of the coefficient automorphism X -> X^k: value at n comes from i = n k^-1 mod 2N
__device__ __forceinline__ double auto_gather(const double* __restrict__ a, int n, int kinv, int logn, Mod m) {
  const int N = 1 << logn;
  const int i = (int)(((long long)n * kinv) & (2 * N - 1));
  if (i < N) return a[i];
  const double x = a[i - N];
  return x == 0.0 ? 0.0 : m.q - x;
}

// exact round(u/P) mod q_i, optional addend, optional modulus switch.
// cv.src = P primes (NK), cv.dst = Q_level; cv.pm/Mmod as for conversions;
// cv.aux[d] = P^-1 mod q_d; cv.aux2[d] = q_{level-1}^-1 mod q_d.
// NS > 0 (relinearisation): the addend is parts 0 and 1 of the square's tensor y
// ([n][3][NS][N] over Q_level then B), scaled and rounded here by the same per-coefficient
// steps as k_scale_round, so those two parts never round-trip through HBM.
template <int NK, int NQ, int NS = 0>
__global__ void __launch_bounds__(TPB)
k_moddown(const double* __restrict__ u, int n, int logn, const double* __restrict__ add, int add_div,
          size_t add_stride, int add_mode, KeySel ks, int modsw, const Conv* __restrict__ cvp,
          const Mod* __restrict__ mods, double* __restrict__ out, int out_div, size_t out_outer,
          const double* __restrict__ y = nullptr, const Conv* __restrict__ srcv = nullptr,
          const Conv* __restrict__ extv = nullptr) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * 2 * N) return;
  const Conv& cv = *cvp;
  const size_t ci = idx / (2 * N);
  const int part = (int)((idx >> logn) & 1);
  const int k = (int)(idx & (N - 1));
  constexpr int NB = NQ + NK;
  const double* up = u + (ci * 2 + part) * NB * N + k;
  double x[NK], v[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) x[i] = up[(NQ + i) * N];
  garner<NK>(x, v, cv, mods);
  const bool neg = above_half<NK>(v, NK, cv, mods);
  double sr[NS > 0 ? NS : 1];
  if constexpr (NS > 0) scale_round_coeff<NS>(y + (ci * 3 + part) * (size_t)NS * N + k, N, NQ, *srcv, mods, sr);
  double res[NQ];
#pragma unroll
  for (int d = 0; d < NQ; ++d) {
    const Mod md = mods[cv.dst[d]];
    double acc = v[NK - 1];
#pragma unroll
    for (int kk = NK - 2; kk >= 0; --kk) acc = mul_lazy(acc, cv.pm[d][kk], md) + v[kk];
    if (neg) acc -= cv.Mmod[d];                                    // |acc| < 2^43: lift_c([u]_P) mod q_d
    double r = norm(mul_lazy(up[d * N] - reduce(acc, md), cv.aux[d], md), md);
    if constexpr (NS > 0) {
      r = add_mod(r, sr[d], md);
    } else if (add_mode == 1) {
      r = add_mod(r, add[(ci / add_div) * add_stride + (size_t)(part * NQ + d) * N + k], md);
    } else if (add_mode == 2 && part == 0) {
      const int kinv = ks.kinv ? ks.kinv[ci % ks.nk] : ks.kinv1;
      r = add_mod(r, auto_gather(add + (ci / add_div) * add_stride + (size_t)d * N, k, kinv, logn, md), md);
    } else if (add_mode == 3) {
      // rotate-and-add: the result is add + Rot(add) (add itself, plus sigma_k of its part 0)
      const double* ab = add + (ci / add_div) * add_stride;
      double a = ab[(size_t)(part * NQ + d) * N + k];
      if (part == 0) {
        const int kinv = ks.kinv ? ks.kinv[ci % ks.nk] : ks.kinv1;
        a = add_mod(a, auto_gather(ab + (size_t)d * N, k, kinv, logn, md), md);
      }
      r = add_mod(r, a, md);
    }
    res[d] = r;
  }
  if constexpr (NS == 0) {
    if (extv) {
      // the result over Q_level then its centred lift to B (as k_extend_qb): out [n][2][NQ+m][N]
      const Conv& ev = *extv;
      double* eb = out + ci * out_outer + (size_t)part * (NQ + ev.nd) * N + k;
#pragma unroll
      for (int d = 0; d < NQ; ++d) eb[(size_t)d * N] = res[d];
      double w[NQ];
      garner<NQ>(res, w, ev, mods);
      const bool eneg = above_half<NQ>(w, NQ, ev, mods);
      for (int d = 0; d < ev.nd; ++d) {
        const Mod md = mods[ev.dst[d]];
        double acc = w[NQ - 1];
#pragma unroll
        for (int kk = NQ - 2; kk >= 0; --kk) acc = mul_lazy(acc, ev.pm[d][kk], md) + w[kk];
        if (eneg) acc -= ev.Mmod[d];
        eb[(size_t)(NQ + d) * N] = reduce(acc, md);
      }
      return;
    }
  }
  const int NQO = modsw ? NQ - 1 : NQ;
  double* ob = out + (ci / out_div) * out_outer + (ci % out_div) * 2 * NQO * N + (size_t)part * NQO * N + k;
  if (!modsw) {
#pragma unroll
    for (int d = 0; d < NQ; ++d) ob[(size_t)d * N] = res[d];
    return;
  }
  const Mod ml = mods[cv.dst[NQ - 1]];
  const double last = res[NQ - 1];
  const double lc = last > (ml.q - 1.0) * 0.5 ? last - ml.q : last;
#pragma unroll
  for (int d = 0; d < NQ - 1; ++d) {
    const Mod md = mods[cv.dst[d]];
    ob[(size_t)d * N] = norm(mul_lazy(res[d] - lc, cv.aux2[d], md), md);
  }
}

// [n][2][level][N] -> [n][2][level-1][N]; linv[d] = q_{level-1}^-1 mod q_d
__global__ void k_modswitch(const double* __restrict__ in, double* __restrict__ out, int n, int level, int logn,
                            Basis b, const Mod* __restrict__ mods, LimbConsts linv) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * 2 * N) return;
  const size_t pp = idx >> logn;        // ciphertext*2 + part
  const size_t k = idx & (N - 1);
  const Mod ml = mods[b.id[level - 1]];
  const double last = in[(pp * level + level - 1) * N + k];
  const double lc = last > (ml.q - 1.0) * 0.5 ? last - ml.q : last;
  for (int d = 0; d < level - 1; ++d) {
    const Mod md = mods[b.id[d]];
    out[(pp * (level - 1) + d) * N + k] = norm(mul_lazy(in[(pp * level + d) * N + k] - lc, linv.v[d], md), md);
  }
}

__global__ void k_automorphism(const double* __restrict__ in, double* __restrict__ out, int npoly, int nl, int logn,
                               int kinv, Basis b, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)npoly * nl * N) return;
  const size_t row = idx >> logn;
  const int k = (int)(idx & (N - 1));
  const Mod m = mods[b.id[row % nl]];
  out[idx] = auto_gather(in + row * N, k, kinv, logn, m);
}

__global__ void k_lift_plain(const double* __restrict__ msg, double* __restrict__ out, int n, int level, int logn,
                             double t, Basis b, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * level * N) return;
  const size_t ci = idx / (level * N);
  const int limb = (int)((idx >> logn) % level);
  const size_t k = idx & (N - 1);
  const double mv = msg[ci * N + k];
  const double mc = mv > (t - 1.0) * 0.5 ? mv - t : mv;
  const Mod m = mods[b.id[limb]];
  out[idx] = mc < 0.0 ? mc + m.q : mc;
}

__global__ void k_slots_to_t(const int64_t* __restrict__ slots, double* __restrict__ out, int n, int logn,
                             long long t, const uint32_t* __restrict__ pos) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * N) return;
  const size_t ci = idx >> logn, s = idx & (N - 1);
  long long v = (long long)(slots[idx] % t);
  if (v < 0) v += t;
  out[ci * N + pos[s]] = (double)v;
}

__global__ void k_t_to_slots(const double* __restrict__ in, int64_t* __restrict__ slots, int n, int logn,
                             double t, const uint32_t* __restrict__ pos) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * N) return;
  const size_t ci = idx >> logn, s = idx & (N - 1);
  const double v = in[ci * N + pos[s]];
  slots[idx] = (int64_t)(v > (t - 1.0) * 0.5 ? v - t : v);
}

// m = round(t x / Q) mod t from x over Q_level (coefficient form)
template <int NS>
__global__ void __launch_bounds__(TPB)
k_dec_round(const double* __restrict__ xin, double* __restrict__ msg, int n, int logn, double t,
            const Conv* __restrict__ cvp, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * N) return;
  const Conv& cv = *cvp;
  const size_t ci = idx >> logn, k = idx & (N - 1);
  double x[NS], v[NS], wdig[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = xin[(ci * NS + i) * N + k];
  garner<NS>(x, v, cv, mods);
  double c = 0.0;
#pragma unroll
  for (int kk = 0; kk < NS; ++kk) {
    double quo;
    wdig[kk] = mul_add_divmod(t, v[kk], c, mods[cv.src[kk]], &quo);
    c = quo;
  }
  double r = c + (above_half<NS>(wdig, NS, cv, mods) ? 1.0 : 0.0);
  if (r >= t) r -= t;
  msg[idx] = r;
}

__global__ void k_pointwise(const double* __restrict__ a, const double* __restrict__ bb, double* __restrict__ out,
                            int n, int nl, int logn, int b_shared, Basis b, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * nl * N) return;
  const size_t lk = idx % (nl * N);
  const Mod m = mods[b.id[lk >> logn]];
  out[idx] = mul_mod(a[idx], bb[b_shared ? lk : idx], m);
}

__global__ void k_small_to_rns(const int8_t* __restrict__ e, double* __restrict__ out, int n, int nl, int logn,
                               Basis b, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)n * nl * N) return;
  const size_t ci = idx / (nl * N);
  const int limb = (int)((idx >> logn) % nl);
  const double v = (double)e[ci * N + (idx & (N - 1))];
  const Mod m = mods[b.id[limb]];
  out[idx] = v < 0.0 ? v + m.q : v;
}

__global__ void k_add_inplace(double* __restrict__ a, const double* __restrict__ b, size_t count, int level, int logn,
                              Basis bs, const Mod* __restrict__ mods) {
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= count) return;
  const Mod m = mods[bs.id[(idx >> logn) % level]];
  a[idx] = add_mod(a[idx], b[idx], m);
}

__global__ void k_fill(double* __restrict__ p, size_t count, double v) {
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx < count) p[idx] = v;
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, size_t width, size_t spitch,
                       size_t dpitch, size_t rows) {
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= width * rows) return;
  const size_t r = idx / width, c = idx % width;
  dst[r * dpitch + c] = src[r * spitch + c];
}

__global__ void k_u64_to_f64(const uint64_t* __restrict__ in, double* __restrict__ out, size_t count) {
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx < count) out[idx] = (double)in[idx];
}

__global__ void k_f64_to_u64(const double* __restrict__ in, uint64_t* __restrict__ out, size_t count) {
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx < count) out[idx] = (uint64_t)in[idx];
}

__global__ void k_keypart(const double* __restrict__ x, const double* __restrict__ e, const double* __restrict__ sp,
                          double* __restrict__ out, int nl, int logn, int g_lo, int g_hi, LimbConsts gval, Basis b,
                          const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (idx >= (size_t)nl * N) return;
  const int limb = (int)(idx >> logn);
  const Mod m = mods[b.id[limb]];
  double r = sub_mod(e[idx], x[idx], m);
  if (limb >= g_lo && limb < g_hi) r = add_mod(r, mul_mod(gval.v[limb], sp[idx], m), m);
  out[idx] = r;
}

__global__ void k_quantise(const float* __restrict__ f, int n_pt, int mode, int batch, int stride_b,
                           const int* __restrict__ slot_of, int per, float scale, int clampv,
                           int64_t* __restrict__ slots, int logn) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (mode == 0) {
    // plaintext p = r * stride_b + j of request r reads f[r][b][j] (image-major features)
    if (idx >= (size_t)n_pt * batch) return;
    const size_t p = idx / batch, bi = idx % batch;
    const size_t r = p / stride_b, j = p % stride_b;
    float q = rintf(scale * f[(r * batch + bi) * (size_t)stride_b + j]);
    q = fminf(fmaxf(q, (float)-clampv), (float)clampv);
    slots[p * N + bi] = (int64_t)q;
  } else {
    if (idx >= (size_t)n_pt * per) return;
    const size_t p = idx / per, kk = idx % per;
    float q = rintf(scale * f[p * per + kk]);
    q = fminf(fmaxf(q, (float)-clampv), (float)clampv);
    slots[p * N + slot_of[kk]] = (int64_t)q;
  }
}

// Slot-batched features straight to the transform domain of R_t: plaintext p =
// r * stride_b + j (request r, feature j) takes, at slot b < batch, the quantised
// feature f[r][b][j] (zero at the other slots), reduced mod t and written at the
// transform position of slot b.  Every position is written, so no clearing pass.
// Consecutive plaintexts are consecutive floats of one image, so a block takes 64
// consecutive transform-domain words (their slots from the inverse slot map) x 32
// plaintexts: it reads each slot's 32 features as one run, quantises, and
// transposes through LDS so that every plaintext row is written as one run.
// Quantised values lie in [-clampv, clampv] with clampv < t, so q mod t is q or q + t.
__global__ void __launch_bounds__(TPB)
k_features_to_t(const float* __restrict__ f, int n_pt, int batch, int stride_b, float scale, int clampv, double t,
                double* __restrict__ out, int logn, const uint32_t* __restrict__ slot_of_word) {
  __shared__ double tile[32][65];
  const size_t N = (size_t)1 << logn;
  const int tid = threadIdx.x;
  const size_t w0 = (size_t)blockIdx.x * 64;
  const int p0 = blockIdx.y * 32;
  {
    const int jj = tid & 31;
    const int p = p0 + jj;
    const int r = p / stride_b, j = p - r * stride_b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = (tid >> 5) + 8 * k;
      const uint32_t b = slot_of_word[w0 + i];
      double v = 0.0;
      if (p < n_pt && b < (uint32_t)batch) {
        float q = rintf(scale * f[((size_t)r * batch + b) * (size_t)stride_b + j]);
        q = fminf(fmaxf(q, (float)-clampv), (float)clampv);
        v = q < 0.0f ? (double)q + t : (double)q;
      }
      tile[jj][i] = v;
    }
  }
  __syncthreads();
  const int i = tid & 63;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int jj = (tid >> 6) + 4 * k;
    if (p0 + jj < n_pt) out[(size_t)(p0 + jj) * N + w0 + i] = tile[jj][i];
  }
}

#define BCN_DISPATCH_NS(ns, MACRO)                                                                  \
  switch (ns) {                                                                                     \
    case 1: MACRO(1); break; case 2: MACRO(2); break; case 3: MACRO(3); break; case 4: MACRO(4); break; \
    case 5: MACRO(5); break; case 6: MACRO(6); break; case 7: MACRO(7); break; case 8: MACRO(8); break; \
    case 9: MACRO(9); break; case 10: MACRO(10); break; case 11: MACRO(11); break;                  \
    case 12: MACRO(12); break; case 13: MACRO(13); break; case 14: MACRO(14); break;                \
    case 15: MACRO(15); break; case 16: MACRO(16); break;                                            \
    default: throw Error(-1, "basis too large for the conversion kernels");                         \
  }

}  // namespace

// ------------------------------------------------------------------ host wrappers

namespace {
// Q_level mod t and -t^-1 mod q_i: the constants of round(Q_level m / t) mod q_i
void delta_consts(const Context& c, int level, double* qmodt_out, double* neg) {
  uint64_t qmodt = 1;
  for (int i = 0; i < level; ++i) {
    qmodt = host::mulmod(qmodt, c.primes[i] % c.t, c.t);
    const uint64_t q = c.primes[i];
    neg[i] = (double)((q - host::invmod(c.t % q, q)) % q);
  }
  *qmodt_out = (double)qmodt;
}
}  // namespace

void mac(const Context& c, const MacPlan& p, const double* in, double* out, int level, hipStream_t s, int requests,
         size_t in_req, size_t out_req, const double* delta_msg, size_t out_ct, size_t out_part, const Basis* basis,
         int parts, const double* mul_pt) {
  if (basis && delta_msg) throw Error(-1, "the delta add needs the Q_level basis");
  if (parts != 2 && (parts != 3 || delta_msg)) throw Error(-1, "MAC over two parts, or three without a delta add");
  const Basis b = basis ? *basis : c.basis_Q(level);
  const int nl = b.n;
  const int words = parts * nl * c.n;
  if (out_ct == 0) {
    out_ct = (size_t)words;
    out_part = (size_t)(words >> 1);          // contiguous rows
  }
  if (p.n_out == 0 || requests == 0) return;
  DeltaAdd da;
  if (delta_msg) {
    da.msg = delta_msg;
    da.msg_req = (size_t)p.n_out * c.n;
    da.mt = c.mod(c.id_t);
    delta_consts(c, level, &da.qmodt, da.negtinv);
  }
  if (mul_pt && delta_msg) throw Error(-1, "the MAC multiplies by a plaintext or adds one, not both");
  da.mulpt = mul_pt;
  // algorithmic work: one FMA per word for each nonzero (output, input) weight
  ProfScope ps(c, "mac", s, 8.0 * words * ((double)p.n_in + p.n_out) * requests, (double)words * p.nnz * requests);
  dim3 grid(nblocks(words), p.n_tiles, requests);
  switch (p.tile) {
#define BCN_MAC_CASE(TO)                                                                                  \
  case TO:                                                                                                \
    if (p.centre)                                                                                         \
      hipLaunchKernelGGL((k_mac<TO, true>), grid, dim3(TPB), 0, s, in, out, words, c.logn, nl, p.W, p.rows, \
                         p.tile_ptr, p.tile_cols, p.chunk, b, c.tab.mods, in_req, out_req, out_ct, out_part, da); \
    else                                                                                                  \
      hipLaunchKernelGGL((k_mac<TO, false>), grid, dim3(TPB), 0, s, in, out, words, c.logn, nl, p.W,       \
                         p.rows, p.tile_ptr, p.tile_cols, p.chunk, b, c.tab.mods, in_req, out_req, out_ct,   \
                         out_part, da);                                                                       \
    break;
    BCN_MAC_CASE(1) BCN_MAC_CASE(2) BCN_MAC_CASE(4) BCN_MAC_CASE(8) BCN_MAC_CASE(16) BCN_MAC_CASE(32)
    BCN_MAC_CASE(64)
#undef BCN_MAC_CASE
    default: throw Error(-1, "bad MAC tile");
  }
  BCN_HIP(hipGetLastError());
}

void ext_tap0(const Context& c, const double* chat, int n, int level, const KsExt& ext, double* X, size_t out_outer,
              hipStream_t s) {
  if (n == 0) return;
  const Basis b = c.basis_QP(level);
  const size_t work = (size_t)n * 2 * b.n * c.n;
  ProfScope ps(c, "ext_tap0", s, 8.0 * (double)n * 2 * c.n * (level + b.n));
  hipLaunchKernelGGL(k_ext_tap0, dim3(nblocks(work)), dim3(TPB), 0, s, chat, n, level, b.n, c.logn, ext, b, c.tab.mods,
                     X, out_outer);
  BCN_HIP(hipGetLastError());
}

static const Conv* extend_conv(const Context& c, int level);

bool mac_qb_supported(const MacPlan& p, int level) {
  return !p.centre && level >= 2 && level <= 6 && (p.tile == 2 || p.tile == 4 || p.tile == 8 || p.tile == 16) &&
         p.tile * level <= 64;
}

bool mac_qb(const Context& c, const MacPlan& p, const double* in, double* out, int level, hipStream_t s, int requests,
            size_t in_req, size_t out_req, const double* delta_msg, size_t out_ct, size_t out_part) {
  if (!mac_qb_supported(p, level)) return false;
  if (p.n_out == 0 || requests == 0) return true;
  DeltaAdd da;
  if (delta_msg) {
    da.msg = delta_msg;
    da.msg_req = (size_t)p.n_out * c.n;
    da.mt = c.mod(c.id_t);
    delta_consts(c, level, &da.qmodt, da.negtinv);
  }
  const Conv* cv = extend_conv(c, level);
  const double words = 2.0 * level * c.n;
  // inputs and the Q limbs out as for the MAC, plus the B limbs the extension would have written
  ProfScope ps(c, "mac", s, 8.0 * requests * (words * ((double)p.n_in + p.n_out) + 2.0 * c.m * c.n * p.n_out),
               words * p.nnz * requests);
  dim3 grid(nblocks((size_t)2 * c.n), p.n_tiles, requests);
  const Basis b = c.basis_Q(level);
#define BCN_MQB(TO, NQ)                                                                                            \
  hipLaunchKernelGGL((k_mac_qb<TO, NQ>), grid, dim3(TPB), 0, s, in, out, c.logn, p.W, p.rows, p.tile_ptr, p.tile_cols, \
                     b, c.tab.mods, in_req, out_req, out_ct, out_part, da, cv)
#define BCN_MQB_T(NQ)                                    \
  switch (p.tile) {                                      \
    case 2: BCN_MQB(2, NQ); break;                       \
    case 4: BCN_MQB(4, NQ); break;                       \
    case 8: BCN_MQB(8, NQ); break;                       \
  }
#define BCN_MQB_T16(NQ)                                  \
  if (p.tile == 16) {                                    \
    BCN_MQB(16, NQ);                                     \
  } else {                                               \
    BCN_MQB_T(NQ)                                        \
  }
  // accumulators: tile * level <= 64
  switch (level) {
    case 2: BCN_MQB_T16(2) break;
    case 3: BCN_MQB_T16(3) break;
    case 4: BCN_MQB_T16(4) break;
    case 5: BCN_MQB_T(5) break;
    case 6: BCN_MQB_T(6) break;
  }
#undef BCN_MQB_T16
#undef BCN_MQB_T
#undef BCN_MQB
  BCN_HIP(hipGetLastError());
  return true;
}

void sum_slabs(const Context& c, const double* in, int slabs, size_t words, int n_polys, const Basis& b, double* out,
               hipStream_t s) {
  if (words == 0) return;
  if (slabs > 2048) throw Error(-1, "too many slabs to sum exactly");
  if (words != (size_t)n_polys * b.n * c.n) throw Error(-1, "slab size does not match the basis");
  ProfScope ps(c, "sum_slabs", s, 8.0 * (double)words * (slabs + 1));
  hipLaunchKernelGGL(k_sum_slabs, dim3(nblocks(words)), dim3(TPB), 0, s, in, slabs, words, b.n, c.logn, b, c.tab.mods,
                     out);
  BCN_HIP(hipGetLastError());
}

void add_delta(const Context& c, double* ct, int n, int level, const double* m, hipStream_t s) {
  if (n == 0) return;
  const Mod mt = c.mod(c.id_t);
  double qmodt = 0.0;
  LimbConsts neg{};
  delta_consts(c, level, &qmodt, neg.v);
  hipLaunchKernelGGL(k_add_delta, dim3(nblocks((size_t)n * level * c.n)), dim3(TPB), 0, s, ct, n, level, c.logn, m,
                     qmodt, mt, c.basis_Q(level), c.tab.mods, neg);
  BCN_HIP(hipGetLastError());
}

void mul_plain_ntt(const Context& c, const double* in, double* out, int n, int level, const double* pt, bool per_ct,
                   hipStream_t s, const Basis* basis) {
  if (n == 0) return;
  const Basis b = basis ? *basis : c.basis_Q(level);
  hipLaunchKernelGGL(k_mul_plain, dim3(nblocks((size_t)n * 2 * b.n * c.n)), dim3(TPB), 0, s, in, out, n, b.n,
                     c.logn, pt, per_ct ? 1 : 0, b, c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void ptvec_mac_ntt(const Context& c, const double* in, int n_in, double* out, int n_out, int level, const double* pt,
                   hipStream_t s, int requests) {
  if (n_out == 0 || requests == 0) return;
  hipLaunchKernelGGL(k_ptvec_mac, dim3(nblocks((size_t)requests * n_out * 2 * level * c.n)), dim3(TPB), 0, s, in, n_in,
                     out, n_out, level, c.logn, pt, c.basis_Q(level), c.tab.mods, requests);
  BCN_HIP(hipGetLastError());
}

void tensor_square(const Context& c, const double* in, double* out, int n, const Basis& b, hipStream_t s) {
  if (n == 0) return;
  ProfScope ps(c, "tensor_square", s, 8.0 * n * (double)b.n * c.n * 5);
  hipLaunchKernelGGL(k_tensor_square, dim3(nblocks((size_t)n * b.n * c.n)), dim3(TPB), 0, s, in, out, n, b.n, c.logn,
                     b, c.tab.mods);
  BCN_HIP(hipGetLastError());
}

static const Conv* extend_conv(const Context& c, int level) {
  std::vector<int> src, dst;
  for (int i = 0; i < level; ++i) src.push_back(c.idQ(i));
  for (int i = 0; i < c.m; ++i) dst.push_back(c.idB(i));
  return conv_device(c, "ext" + std::to_string(level), make_conv(c, src, dst));
}

void extend_qb(const Context& c, const double* in, double* out, int n, int level, hipStream_t s) {
  if (n == 0) return;
  const Conv* cv = extend_conv(c, level);
  const int npoly = 2 * n;
  const int in_place = in == out ? 1 : 0;
  // in place only the B limbs are written
  ProfScope ps(c, "extend_qb", s, 8.0 * npoly * (double)c.n * (in_place ? level + c.m : 2 * level + c.m));
#define BCN_EXT(NS) hipLaunchKernelGGL(k_extend_qb<NS>, dim3(nblocks((size_t)npoly * c.n)), dim3(TPB), 0, s, in, out, \
                                       npoly, c.logn, in_place, cv, c.tab.mods)
  BCN_DISPATCH_NS(level, BCN_EXT)
#undef BCN_EXT
  BCN_HIP(hipGetLastError());
}

// the scale-and-round conversion of level `level` (Q_level + B -> Q_level), cached on the device
static const Conv* scale_round_conv(const Context& c, int level) {
  std::vector<int> src, dst;
  for (int i = 0; i < level; ++i) { src.push_back(c.idQ(i)); dst.push_back(c.idQ(i)); }
  for (int i = 0; i < c.m; ++i) src.push_back(c.idB(i));
  Conv cv = make_conv(c, src, dst);
  for (int d = 0; d < level; ++d) {
    uint64_t bm = 1;
    const uint64_t q = c.primes[d];
    for (int i = 0; i < c.m; ++i) bm = host::mulmod(bm, c.primes[c.idB(i)] % q, q);
    cv.aux[d] = (double)bm;
  }
  cv.aux2[0] = (double)c.t;
  return conv_device(c, "sr" + std::to_string(level), cv);
}

void scale_round(const Context& c, const double* in, double* out, int n, int level, hipStream_t s, bool only_d2,
                 bool modsw) {
  if (n == 0) return;
  if (modsw && level < 2) throw Error(-2, "modulus switch needs at least two primes");
  const Conv* dcv = scale_round_conv(c, level);
  const int npoly = only_d2 ? n : 3 * n;
  const int pmul = only_d2 ? 3 : 1, padd = only_d2 ? 2 : 0;
  const int ns = level + c.m;
  LimbConsts linv{};
  if (modsw)
    for (int d = 0; d < level - 1; ++d)
      linv.v[d] = (double)host::invmod(c.primes[level - 1] % c.primes[d], c.primes[d]);
  ProfScope ps(c, "scale_round", s, 8.0 * npoly * (double)c.n * (ns + (modsw ? level - 1 : level)));
#define BCN_SR(NS) hipLaunchKernelGGL(k_scale_round<NS>, dim3(nblocks((size_t)npoly * c.n)), dim3(TPB), 0, s, in, out, \
                                      npoly, c.logn, level, pmul, padd, dcv, c.tab.mods, modsw ? 1 : 0, linv)
  BCN_DISPATCH_NS(ns, BCN_SR)
#undef BCN_SR
  BCN_HIP(hipGetLastError());
}

// digit j of level `level` raised to Q_level + P
static const Conv* modup_conv(const Context& c, int level, int j) {
  const Basis dstb = c.basis_QP(level);
  const int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, level);
  std::vector<int> src, dst;
  for (int i = lo; i < hi; ++i) src.push_back(c.idQ(i));
  for (int i = 0; i < dstb.n; ++i) dst.push_back(dstb.id[i]);
  Conv cv = make_conv(c, src, dst);
  for (int d = 0; d < dstb.n; ++d) {
    cv.aux[d] = (d >= lo && d < hi) ? 1.0 : 0.0;
    cv.aux2[d] = (d >= lo && d < hi) ? (double)(d - lo) : 0.0;
  }
  return conv_device(c, "mu" + std::to_string(level) + "_" + std::to_string(j), cv);
}

void decompose_modup(const Context& c, const double* in, size_t in_stride, double* out, int n, int level,
                     hipStream_t s) {
  if (n == 0) return;
  const int dnum = c.dnum(level);
  const Basis dstb = c.basis_QP(level);
  ProfScope ps(c, "modup", s, 8.0 * n * (double)c.n * (level + dnum * dstb.n));
  for (int j = 0; j < dnum; ++j) {
    const int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, level);
    const Conv* dcv = modup_conv(c, level, j);
    const int ns = hi - lo;
#define BCN_MU(NS) hipLaunchKernelGGL(k_modup<NS>, dim3(nblocks((size_t)n * c.n)), dim3(TPB), 0, s, in, in_stride, out, \
                                      n, c.logn, j, dnum, dcv, c.tab.mods, lo)
    BCN_DISPATCH_NS(ns, BCN_MU)
#undef BCN_MU
    BCN_HIP(hipGetLastError());
  }
}

void ks_inner(const Context& c, const double* D, int d_div, const KeySel& ka, int n, int level, double* out,
              hipStream_t s) {
  if (n == 0) return;
  const Basis b = c.basis_QP(level);
  ProfScope ps(c, "ks_inner", s, 8.0 * n * (double)c.n * b.n * (2 + (double)c.dnum(level) * 2));
  hipLaunchKernelGGL(k_ks_inner, dim3(nblocks((size_t)n * b.n * c.n)), dim3(TPB), 0, s, D, ka, n, d_div,
                     level, b.n, c.dnum(level), c.L, c.logn, b, c.tab.mods, out);
  BCN_HIP(hipGetLastError());
}

namespace {
const Conv* moddown_conv(const Context& c, int level) {
  std::vector<int> src, dst;
  for (int i = 0; i < c.K; ++i) src.push_back(c.idP(i));
  for (int i = 0; i < level; ++i) dst.push_back(c.idQ(i));
  Conv cv = make_conv(c, src, dst);
  for (int d = 0; d < level; ++d) {
    const uint64_t q = c.primes[d];
    uint64_t pm = 1;
    for (int i = 0; i < c.K; ++i) pm = host::mulmod(pm, c.primes[c.idP(i)] % q, q);
    cv.aux[d] = (double)host::invmod(pm, q);
    cv.aux2[d] = (d < level - 1) ? (double)host::invmod(c.primes[level - 1] % q, q) : 0.0;
  }
  return conv_device(c, "md" + std::to_string(level), cv);
}
}  // namespace

bool moddown_scale_round_ok(const Context& c, int level) {
  // compiled for 1 or 2 special primes, 2..6 ciphertext primes and 4..7 auxiliary primes
  return c.K >= 1 && c.K <= 2 && level >= 2 && level <= 6 && c.m >= 4 && c.m <= 7;
}

bool moddown_scale_round(const Context& c, const double* u, int n, int level, const double* y, bool modsw,
                         double* out, hipStream_t s) {
  const int ns = level + c.m;
  if (!moddown_scale_round_ok(c, level)) return false;
  if (n == 0) return true;
  const Conv* dcv = moddown_conv(c, level);
  const Conv* scv = scale_round_conv(c, level);
  const size_t work = (size_t)n * 2 * c.n;
  // reads u (level + K limbs) and parts 0, 1 of y (level + m limbs), writes the output
  ProfScope ps(c, "moddown", s, 8.0 * work * ((double)level + c.K + ns + (modsw ? level - 1 : level)));
  const KeySel ks;
  const size_t out_outer = (size_t)2 * (modsw ? level - 1 : level) * c.n;
  const int key = c.K * 10000 + level * 100 + ns;
  switch (key) {
#define BCN_MDS(NK, NQ, NS)                                                                                      \
  case NK * 10000 + NQ * 100 + NS:                                                                               \
    hipLaunchKernelGGL((k_moddown<NK, NQ, NS>), dim3(nblocks(work)), dim3(TPB), 0, s, u, n, c.logn, nullptr, 1,    \
                       (size_t)0, 4, ks, modsw ? 1 : 0, dcv, c.tab.mods, out, 1, out_outer, y, scv);             \
    break;
#define BCN_MDS_M(NK, NQ) BCN_MDS(NK, NQ, NQ + 4) BCN_MDS(NK, NQ, NQ + 5) BCN_MDS(NK, NQ, NQ + 6) BCN_MDS(NK, NQ, NQ + 7)
#define BCN_MDS_Q(NK) BCN_MDS_M(NK, 2) BCN_MDS_M(NK, 3) BCN_MDS_M(NK, 4) BCN_MDS_M(NK, 5) BCN_MDS_M(NK, 6)
    BCN_MDS_Q(1)
    BCN_MDS_Q(2)
#undef BCN_MDS_Q
#undef BCN_MDS_M
#undef BCN_MDS
    default: return false;
  }
  BCN_HIP(hipGetLastError());
  return true;
}

void moddown(const Context& c, const double* u, int n, int level, const double* add, int add_div, size_t add_stride,
             int add_mode, const KeySel& ks, bool modsw, double* out, hipStream_t s, int out_div, size_t out_outer,
             bool ext_qb) {
  if (n == 0) return;
  if (modsw && level < 2) throw Error(-2, "modulus switch needs at least two primes");
  if (ext_qb && (modsw || out_div > 0)) throw Error(-1, "ModDown with the extension to Q+B: contiguous, no switch");
  const Conv* dcv = moddown_conv(c, level);
  const Conv* ecv = ext_qb ? extend_conv(c, level) : nullptr;
  const size_t work = (size_t)n * 2 * c.n;
  ProfScope ps(c, "moddown", s,
               8.0 * work * ((double)level + c.K + (add_mode ? level : 0) + (modsw ? level - 1 : level) + (ext_qb ? c.m : 0)));
  if (ext_qb) {
    out_div = 1;
    out_outer = (size_t)2 * (level + c.m) * c.n;
  }
#define BCN_MD(NK, NQ) hipLaunchKernelGGL((k_moddown<NK, NQ>), dim3(nblocks(work)), dim3(TPB), 0, s, u, n, c.logn, add, \
                                          add_div, add_stride, add_mode, ks, modsw ? 1 : 0, dcv, c.tab.mods, out, \
                                          out_div > 0 ? out_div : 1, \
                                          out_div > 0 ? out_outer : (size_t)2 * (modsw ? level - 1 : level) * c.n, \
                                          nullptr, nullptr, ecv)
#define BCN_MDQ(NK)                                                                                   \
  switch (level) {                                                                                    \
    case 1: BCN_MD(NK, 1); break; case 2: BCN_MD(NK, 2); break; case 3: BCN_MD(NK, 3); break;         \
    case 4: BCN_MD(NK, 4); break; case 5: BCN_MD(NK, 5); break; case 6: BCN_MD(NK, 6); break;         \
    case 7: BCN_MD(NK, 7); break; case 8: BCN_MD(NK, 8); break;                                        \
    default: throw Error(-1, "too many ciphertext primes for moddown");                               \
  }
  switch (c.K) {
    case 1: BCN_MDQ(1); break;
    case 2: BCN_MDQ(2); break;
    case 3: BCN_MDQ(3); break;
    default: throw Error(-1, "too many special primes");
  }
#undef BCN_MDQ
#undef BCN_MD
  BCN_HIP(hipGetLastError());
}

void modswitch(const Context& c, const double* in, double* out, int n, int level, hipStream_t s) {
  if (n == 0) return;
  if (level < 2) throw Error(-2, "modulus switch needs at least two primes");
  LimbConsts linv{};
  for (int d = 0; d < level - 1; ++d) linv.v[d] = (double)host::invmod(c.primes[level - 1] % c.primes[d], c.primes[d]);
  hipLaunchKernelGGL(k_modswitch, dim3(nblocks((size_t)n * 2 * c.n)), dim3(TPB), 0, s, in, out, n, level, c.logn,
                     c.basis_Q(level), c.tab.mods, linv);
  BCN_HIP(hipGetLastError());
}

void automorphism_coeff(const Context& c, const double* in, double* out, int n, const Basis& b, int k, hipStream_t s) {
  if (n == 0) return;
  const int kinv = (int)host::inv_pow2(((uint64_t)k), c.logn + 1);
  hipLaunchKernelGGL(k_automorphism, dim3(nblocks((size_t)n * b.n * c.n)), dim3(TPB), 0, s, in, out, n, b.n, c.logn,
                     kinv, b, c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void lift_plain(const Context& c, const double* m, double* out, int n, int level, hipStream_t s, const Basis* basis) {
  if (n == 0) return;
  const Basis b = basis ? *basis : c.basis_Q(level);
  hipLaunchKernelGGL(k_lift_plain, dim3(nblocks((size_t)n * b.n * c.n)), dim3(TPB), 0, s, m, out, n, b.n, c.logn,
                     (double)c.t, b, c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void slots_to_tdomain(const Context& c, const int64_t* slots, double* out, int n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_slots_to_t, dim3(nblocks((size_t)n * c.n)), dim3(TPB), 0, s, slots, out, n, c.logn,
                     (long long)c.t, c.d_slot_pos);
  BCN_HIP(hipGetLastError());
}

void features_to_tdomain(const Context& c, const float* f, int n_pt, int batch, int stride_b, float scale, int clampv,
                         double* out, hipStream_t s) {
  if (n_pt == 0) return;
  if (clampv < 0 || (uint64_t)clampv >= c.t) throw Error(-1, "feature clamp must lie in [0, t)");
  if (batch > (int)c.n || stride_b < 1) throw Error(-1, "bad feature layout");
  hipLaunchKernelGGL(k_features_to_t, dim3((unsigned)(c.n / 64), (unsigned)((n_pt + 31) / 32)), dim3(TPB), 0, s, f,
                     n_pt, batch, stride_b, scale, clampv, (double)c.t, out, c.logn, c.d_slot_of_word);
  BCN_HIP(hipGetLastError());
}

void tdomain_to_slots(const Context& c, const double* in, int64_t* slots, int n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_t_to_slots, dim3(nblocks((size_t)n * c.n)), dim3(TPB), 0, s, in, slots, n, c.logn,
                     (double)c.t, c.d_slot_pos);
  BCN_HIP(hipGetLastError());
}

static const Conv* dec_conv(const Context& c, int level) {
  std::vector<int> src;
  for (int i = 0; i < level; ++i) src.push_back(c.idQ(i));
  return conv_device(c, "dec" + std::to_string(level), make_conv(c, src, {}));
}

void dec_round(const Context& c, const double* x, double* m, int n, int level, hipStream_t s) {
  if (n == 0) return;
  const Conv* dcv = dec_conv(c, level);
#define BCN_DEC(NS) hipLaunchKernelGGL(k_dec_round<NS>, dim3(nblocks((size_t)n * c.n)), dim3(TPB), 0, s, x, m, n, c.logn, \
                                       (double)c.t, dcv, c.tab.mods)
  BCN_DISPATCH_NS(level, BCN_DEC)
#undef BCN_DEC
  BCN_HIP(hipGetLastError());
}

void pointwise_mul(const Context& c, const double* a, const double* b, double* out, int n, const Basis& bs,
                   bool b_shared, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pointwise, dim3(nblocks((size_t)n * bs.n * c.n)), dim3(TPB), 0, s, a, b, out, n, bs.n, c.logn,
                     b_shared ? 1 : 0, bs, c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void small_to_rns(const Context& c, const int8_t* e, double* out, int n, const Basis& b, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_small_to_rns, dim3(nblocks((size_t)n * b.n * c.n)), dim3(TPB), 0, s, e, out, n, b.n, c.logn, b,
                     c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void add_inplace(const Context& c, double* a, const double* b, int npoly, int level, hipStream_t s) {
  const size_t count = (size_t)npoly * level * c.n;
  if (count == 0) return;
  hipLaunchKernelGGL(k_add_inplace, dim3(nblocks(count)), dim3(TPB), 0, s, a, b, count, level, c.logn, c.basis_Q(level),
                     c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void fill(double* p, size_t count, double v, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(count)), dim3(TPB), 0, s, p, count, v);
  BCN_HIP(hipGetLastError());
}

void copy_rows(const double* src, size_t spitch, double* dst, size_t dpitch, size_t width, size_t rows, hipStream_t s) {
  if (width == 0 || rows == 0) return;
  hipLaunchKernelGGL(k_copy, dim3(nblocks(width * rows)), dim3(TPB), 0, s, src, dst, width, spitch, dpitch, rows);
  BCN_HIP(hipGetLastError());
}

void u64_to_f64(const uint64_t* in, double* out, size_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_u64_to_f64, dim3(nblocks(count)), dim3(TPB), 0, s, in, out, count);
  BCN_HIP(hipGetLastError());
}

void f64_to_u64(const double* in, uint64_t* out, size_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_f64_to_u64, dim3(nblocks(count)), dim3(TPB), 0, s, in, out, count);
  BCN_HIP(hipGetLastError());
}

void combine_keypart(const Context& c, const double* x, const double* e, const double* sp, double* out, const Basis& b,
                     int g_lo, int g_hi, const double* g_val_host, hipStream_t s) {
  LimbConsts g{};
  for (int i = 0; i < b.n; ++i) g.v[i] = g_val_host ? g_val_host[i] : 0.0;
  hipLaunchKernelGGL(k_keypart, dim3(nblocks((size_t)b.n * c.n)), dim3(TPB), 0, s, x, e, sp, out, b.n, c.logn, g_lo,
                     g_hi, g, b, c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void quantise_features(const Context& c, const float* f, int n_pt, int mode, int batch, int stride_b, const int* slot_of,
                       int per, float scale, int clampv, int64_t* slots, hipStream_t s) {
  const size_t work = mode == 0 ? (size_t)n_pt * batch : (size_t)n_pt * per;
  if (work == 0) return;
  hipLaunchKernelGGL(k_quantise, dim3(nblocks(work)), dim3(TPB), 0, s, f, n_pt, mode, batch, stride_b, slot_of, per,
                     scale, clampv, slots, c.logn);
  BCN_HIP(hipGetLastError());
}

// Builds every conversion table the library uses at each level up front, so that
// no later call has to allocate device memory for one.
void preload_conversions(const Context& c) {
  for (int level = 1; level <= c.L; ++level) {
    extend_conv(c, level);
    scale_round_conv(c, level);
    moddown_conv(c, level);
    dec_conv(c, level);
    for (int j = 0; j < c.dnum(level); ++j) modup_conv(c, level, j);
  }
}

}  // namespace bcn
