// Negacyclic NTT / inverse NTT over every limb of a batch of RNS polynomials.
//
// Forward:  out[pos] = a(psi^(2j+1)) mod q with j = bitrev(pos)  (Cooley-Tukey,
//           natural input, the psi twist merged into the twiddles).
// Inverse:  the exact inverse: bit-reversed input, natural output
//           (decimation in time with omega^-1, then one multiply by N^-1 psi^-k).
//
// One workgroup transforms one limb.  Each thread keeps E = 2^LOGE residues in
// registers and applies LOGE butterfly stages per pass; passes exchange data
// through LDS (the whole limb is LDS-resident, bank-swizzled).  The first pass reads
// HBM and the last pass writes HBM, so a limb costs one read and one write of
// N words.  Values grow additively inside the transform (|x| < (LOGN+1) q <
// 2^45), which the lazy FP64 product tolerates; one reduction at the end
// brings them back to [0, q).
#include <algorithm>
#include <cstdlib>
#include <string>

#include "convert.h"

namespace bcn {
namespace {

// LDS word of transform index g: an XOR swizzle of the low five bits by the
// five bits above the register-set size.  It is a bijection on every block of
// 2^(LOGE+5) words and makes all the kernel's lane patterns (consecutive
// indices, or per-lane contiguous sets of 2^LOGE) hit distinct banks.
template <int LOGE>
__device__ __forceinline__ int lds_sw(int g) { return g ^ ((g >> LOGE) & 31); }

template <int LOGN, int LOGE>
struct Shape {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 1 << LOGE;
  static constexpr int T = N / E;
  static constexpr int NP = (LOGN + LOGE - 1) / LOGE;
  static constexpr int C0 = LOGN - LOGE * (NP - 1);
};

// stages in pass P and the first stage of pass P
template <int LOGN, int LOGE, bool INV>
struct Sched {
  using S = Shape<LOGN, LOGE>;
  static constexpr int c(int p) { return INV ? (p < S::NP - 1 ? LOGE : S::C0) : (p == 0 ? S::C0 : LOGE); }
  static constexpr int s0(int p) { return INV ? p * LOGE : (p == 0 ? 0 : S::C0 + (p - 1) * LOGE); }
};

// Twiddles one thread uses in pass P, in the order the butterfly loops consume them:
// forward stages take one per block of butterflies that share it, inverse stages
// one per position inside a block.
template <int LOGN, int LOGE, bool INV, int P>
struct PassTw {
  using S = Shape<LOGN, LOGE>;
  static constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  static constexpr int NT = (S::E >> C) * ((1 << C) - 1);
};

// Index of element j of group g in pass P (transform order).
template <int LOGN, int LOGE, bool INV, int P>
__device__ __forceinline__ int pass_base(int g, int tid) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, T = S::T;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  constexpr int S0 = Sched<LOGN, LOGE, INV>::s0(P);
  constexpr int SMIN = INV ? (1 << S0) : (N >> (S0 + C));
  const int sid = g * T + tid;
  const int b = sid / SMIN, r = sid % SMIN;
  return INV ? b * (SMIN << C) + r : b * (N >> S0) + r;
}

// Read-only load through the constant address space: with a wave-uniform index the
// compiler issues it as a scalar load.
__device__ __forceinline__ double const_load(const double* p, unsigned i) {
  return ((const __attribute__((address_space(4))) double*)p)[i];
}

template <int LOGN, int LOGE, bool INV, int P, int NT>
__device__ __forceinline__ void load_tw(double (&wt)[NT], const double* __restrict__ tw, const int tid) {
  using S = Shape<LOGN, LOGE>;
  constexpr unsigned N = S::N;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  constexpr int S0 = Sched<LOGN, LOGE, INV>::s0(P);
  constexpr int SZ = 1 << C;
  constexpr int G = S::E >> C;
  constexpr unsigned SMIN = INV ? (1u << S0) : (N >> (S0 + C));
  // A pass whose twiddles are the same for all lanes of a wave (forward passes whose
  // blocks span at least 64 lanes, inverse passes whose blocks start at every index)
  // computes the indices from the wave's first lane, so they become scalar loads
  // through the scalar cache instead of vector loads competing with the data stream.
  constexpr bool UNIFORM = INV ? SMIN == 1 : SMIN >= 64;
  const int t = UNIFORM ? __builtin_amdgcn_readfirstlane(tid) : tid;
  // unsigned 32-bit indices: lets the compiler address the table with a scalar base
  // and one 32-bit lane offset
  unsigned base[G];
#pragma unroll
  for (int g = 0; g < G; ++g) base[g] = (unsigned)pass_base<LOGN, LOGE, INV, P>(g, t);
  int k = 0;
#pragma unroll
  for (int l = 0; l < C; ++l) {
    const int s = S0 + l;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!INV) {
        const int sh = C - 1 - l;
#pragma unroll
        for (int kb = 0; kb < (SZ >> (sh + 1)); ++kb) {
          const unsigned gi = base[g] + ((unsigned)kb << (sh + 1)) * SMIN;
          const unsigned w = (1u << s) + fwd_tw_word((int)(gi >> (LOGN - s)), s, LOGN);
          wt[k++] = UNIFORM ? const_load(tw, w) : tw[w];
        }
      } else {
        const unsigned r = base[g] & (SMIN - 1);
#pragma unroll
        for (int jl = 0; jl < (1 << l); ++jl) {
          const unsigned w = (1u << s) + r + jl * SMIN;
          wt[k++] = UNIFORM ? const_load(tw, w) : tw[w];
        }
      }
    }
  }
}

// Wave (64 lanes) that holds transform index e in pass P.
template <int LOGN, int LOGE, bool INV, int P>
constexpr int pass_wave(int e) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, T = S::T;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  constexpr int S0 = Sched<LOGN, LOGE, INV>::s0(P);
  constexpr int SMIN = INV ? (1 << S0) : (N >> (S0 + C));
  const int r = e % SMIN;
  const int b = INV ? e / (SMIN << C) : e / (N >> S0);
  return ((b * SMIN + r) % T) / 64;
}

// True when every wave holds the same indices in passes P and P + 1: the exchange
// between them then stays inside each wave's own LDS words and needs no workgroup
// barrier.
template <int LOGN, int LOGE, bool INV, int P>
constexpr bool exchange_is_wave_local() {
  for (int e = 0; e < (1 << LOGN); ++e)
    if (pass_wave<LOGN, LOGE, INV, P>(e) != pass_wave<LOGN, LOGE, INV, P + 1>(e)) return false;
  return true;
}

// Transform index of register r of thread tid in pass P, for passes that hold one group
// (2^LOGE consecutive butterfly positions per thread).
template <int LOGN, int LOGE, bool INV, int P>
constexpr int pass_index(int tid, int r) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  constexpr int S0 = Sched<LOGN, LOGE, INV>::s0(P);
  constexpr int SMIN = INV ? (1 << S0) : (N >> (S0 + C));
  const int b = tid / SMIN, rr = tid % SMIN;
  return (INV ? b * (SMIN << C) + rr : b * (N >> S0) + rr) + r * SMIN;
}

// True when the exchange between passes P and P + 1 is a 16 x 16 transpose inside every row of
// 16 lanes: register r of lane l in pass P is register (l mod 16) of lane 16 floor(l / 16) + r
// in pass P + 1.  Such an exchange can run on cross-lane moves instead of LDS.
template <int LOGN, int LOGE, bool INV, int P>
constexpr bool exchange_is_row_transpose() {
  using S = Shape<LOGN, LOGE>;
  if (LOGE != 4 || P + 1 >= S::NP) return false;
  if (Sched<LOGN, LOGE, INV>::c(P) != LOGE || Sched<LOGN, LOGE, INV>::c(P + 1) != LOGE) return false;
  for (int tid = 0; tid < S::T; ++tid)
    for (int r = 0; r < 16; ++r)
      if (pass_index<LOGN, LOGE, INV, P + 1>((tid & ~15) | r, tid & 15) != pass_index<LOGN, LOGE, INV, P>(tid, r))
        return false;
  return true;
}

// v of lane (l xor K) inside rows of 16 lanes: DPP quad permutations for K = 1, 2 (a VALU move),
// the swizzle unit's bit-mask mode for K = 4, 8 (no LDS words touched).
template <int K>
__device__ __forceinline__ double lanes_xor(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  if constexpr (K == 1 || K == 2) {
    constexpr int ctrl = K == 1 ? 0xB1 : 0x4E;   // quad_perm [1,0,3,2] / [2,3,0,1]
    lo = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xF, 0xF, true);
    hi = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xF, 0xF, true);
  } else {
    constexpr int pat = 0x1F | (K << 10);          // and 31, or 0, xor K
    lo = __builtin_amdgcn_ds_swizzle(lo, pat);
    hi = __builtin_amdgcn_ds_swizzle(hi, pat);
  }
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// One round of the row transpose: swaps bit K of the lane with bit K of the register index
// (for each pair of registers differing in bit K, the lane whose bit K is 0 sends its upper one
// and the other lane its lower one).
template <int K>
__device__ __forceinline__ void row_transpose_round(double (&x)[16], int lane) {
  const bool up = (lane & K) != 0;
#pragma unroll
  for (int j0 = 0; j0 < 16; ++j0) {
    if (j0 & K) continue;
    const double r = lanes_xor<K>(up ? x[j0] : x[j0 | K]);
    x[j0] = up ? r : x[j0];
    x[j0 | K] = up ? x[j0 | K] : r;
  }
}

// The row transpose of exchange_is_row_transpose in registers: four rounds, round k swapping
// bit k of the lane with bit k of the register index.
__device__ __forceinline__ void row_transpose16(double (&x)[16]) {
  const int lane = (int)(threadIdx.x & 63);
  row_transpose_round<1>(x, lane);
  row_transpose_round<2>(x, lane);
  row_transpose_round<4>(x, lane);
  row_transpose_round<8>(x, lane);
}

// Orders one wave's LDS writes before its later reads.  A wave's LDS operations
// execute in issue order, so only the compiler has to be kept from moving them.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copies n doubles from global memory into LDS with direct global-to-LDS loads (16 bytes per lane,
// a wave fills 1 KiB of consecutive words; no registers in between, so every load of the copy is
// in flight at once), then waits for them and for the whole workgroup.  n must be a multiple of
// 128 times the workgroup's waves; src and lds 16-byte aligned.
__device__ __forceinline__ void stage_to_lds(double* lds, const double* __restrict__ src, int n, int tid,
                                             int nthreads) {
  const int waves = nthreads >> 6;
  const int lane = tid & 63;
  for (int base = (tid >> 6) * 128; base < n; base += waves * 128)
    __builtin_amdgcn_global_load_lds((const void*)(src + base + lane * 2),
                                     (__attribute__((address_space(3))) void*)(lds + base), 16, 0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// One pass of the transform.  FROM_REGS: the first pass starts from the
// registers (already in this pass's layout) instead of reading HBM.  TO_REGS:
// the last pass leaves its results in the registers (lazy form, no final
// reduction or untwist) instead of writing HBM.  PF: every pass loads the next
// pass's twiddles before the exchange barriers, so their latency overlaps the
// exchange (costs registers for one more pass's twiddles).
template <int LOGN, int LOGE, bool INV, int P, bool FROM_REGS = false, bool TO_REGS = false, bool PF = false,
          bool XL = false, bool XREG = false>
__device__ __forceinline__ void run_pass(double (&x)[1 << LOGE], double* lds, const double* __restrict__ src,
                                         double* __restrict__ a, const double* __restrict__ tw,
                                         const double* __restrict__ post, const Mod m, const int tid_in,
                                         const double* wpre = nullptr, int store_gal = 1) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  constexpr int SZ = 1 << C;
  constexpr int G = S::E >> C;
  constexpr int S0 = Sched<LOGN, LOGE, INV>::s0(P);
  constexpr int SMIN = INV ? (1 << S0) : (N >> (S0 + C));
  constexpr int NT = PassTw<LOGN, LOGE, INV, P>::NT;

  // The thread index is hidden from the optimiser at the start of every transform (an
  // empty asm that claims to change it): otherwise the address arithmetic of passes
  // with the same layout in different transforms (the forward transform's last pass and
  // the inverse transform's first, or two transforms in one kernel) is computed once and
  // kept live across the whole kernel, which more than doubles the register use of the
  // fused kernels.
  int tid = tid_in;
  if constexpr (P == 0) asm volatile("" : "+v"(tid));
  int base[G];
#pragma unroll
  for (int g = 0; g < G; ++g) base[g] = pass_base<LOGN, LOGE, INV, P>(g, tid);

  double wt[NT];
  if constexpr (PF && P > 0) {
#pragma unroll
    for (int k = 0; k < NT; ++k) wt[k] = wpre[k];
  } else {
    load_tw<LOGN, LOGE, INV, P>(wt, tw, tid);
  }

  // gather
  if constexpr (P == 0) {
    if constexpr (!FROM_REGS) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int j = 0; j < SZ; ++j) {
          const int gi = base[g] + j * SMIN;
          x[g * SZ + j] = src[INV ? ntt_store(gi, LOGN) : gi];   // inverse input is transform-domain
        }
    }
  } else if constexpr (!XREG) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < SZ; ++j) x[g * SZ + j] = lds[lds_sw<LOGE>(base[g] + j * SMIN)];
  }

  // butterflies
  int k = 0;
#pragma unroll
  for (int l = 0; l < C; ++l) {
    if (!INV) {
      // forward stage: local blocks of 2*half elements, one twiddle per block
      const int sh = C - 1 - l;
      const int half = 1 << sh;
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int kb = 0; kb < (SZ >> (sh + 1)); ++kb) {
          const int j0 = kb << (sh + 1);
          const double w = wt[k++];
#pragma unroll
          for (int jj = 0; jj < half; ++jj) {
            const int j = g * SZ + j0 + jj;
            const double u = x[j];
            const double v = mul_lazy(w, x[j + half], m);
            x[j] = u + v;
            x[j + half] = u - v;
          }
        }
      }
    } else {
      // inverse stage: the twiddle depends only on the position inside a block
      const int half = 1 << l;
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int jl = 0; jl < half; ++jl) {
          const double w = wt[k++];
#pragma unroll
          for (int kb = 0; kb < (SZ >> (l + 1)); ++kb) {
            const int j = g * SZ + (kb << (l + 1)) + jl;
            const double u = x[j];
            const double v = mul_lazy(w, x[j + half], m);
            x[j] = u + v;
            x[j + half] = u - v;
          }
        }
      }
    }
  }

  if constexpr (P == S::NP - 1) {
    if constexpr (!TO_REGS) {
      // scatter to HBM in canonical form
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int j = 0; j < SZ; ++j) {
          const int gi = base[g] + j * SMIN;
          double v = x[g * SZ + j];
          v = INV ? norm(mul_lazy(post[gi], v, m), m) : reduce(v, m);
          // store_gal != 1 (forward only): write sigma(a)^ instead, where sigma(a)^ at index
          // i is a^ at ntt_perm(i, k), i.e. the value of index gi goes to ntt_perm(gi, k^-1)
          a[INV ? gi : ntt_store(store_gal == 1 ? gi : ntt_perm(gi, store_gal, LOGN), LOGN)] = v;
        }
    }
  } else {
    constexpr int NT1 = PassTw<LOGN, LOGE, INV, P + 1>::NT;
    double wn[PF ? NT1 : 1];
    if constexpr (PF) load_tw<LOGN, LOGE, INV, P + 1>(wn, tw, tid);
    if constexpr (XL && exchange_is_row_transpose<LOGN, LOGE, INV, P>()) {
      // no LDS words are written, so no earlier reader needs a barrier
      row_transpose16(x);
      run_pass<LOGN, LOGE, INV, P + 1, FROM_REGS, TO_REGS, PF, XL, true>(x, lds, src, a, tw, post, m, tid, wn,
                                                                          store_gal);
      return;
    }
    // A wave-local exchange inside one transform (P > 0) overwrites only words the same
    // wave read in this pass; the first exchange may overwrite words other waves read in
    // the caller's previous transform, so it keeps the workgroup barrier.
    constexpr bool LOCAL = exchange_is_wave_local<LOGN, LOGE, INV, P>();
    if constexpr (LOCAL && P > 0) {
      wave_sync();
    } else if constexpr (P > 0 || FROM_REGS) {
      __syncthreads();   // previous LDS readers are done
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < SZ; ++j) lds[lds_sw<LOGE>(base[g] + j * SMIN)] = x[g * SZ + j];
    if constexpr (LOCAL) {
      wave_sync();
    } else {
      __syncthreads();
    }
    run_pass<LOGN, LOGE, INV, P + 1, FROM_REGS, TO_REGS, PF, XL>(x, lds, src, a, tw, post, m, tid, wn, store_gal);
  }
}

template <int LOGN, int LOGE, bool INV, bool PF, bool XL = false>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ntt(double* __restrict__ data, Basis basis, Tables tb) {
  constexpr int N = 1 << LOGN;
  extern __shared__ double lds[];
  const int nb = basis.n, npoly = gridDim.x / nb;
  const int w = xcd_order(blockIdx.x, gridDim.x);
  const int limb = w / npoly, poly = w - limb * npoly;
  const int pid = basis.id[limb];
  const Mod m = tb.mods[pid];
  double* a = data + ((size_t)poly * nb + limb) * N;
  const double* tw = INV ? tb.inv + (size_t)pid * N : tb.fwd + (size_t)pid * N;
  const double* post = tb.post + (size_t)pid * N;
  double x[1 << LOGE];
  run_pass<LOGN, LOGE, INV, 0, false, false, PF, XL>(x, lds, a, a, tw, post, m, threadIdx.x);
}

// Register positions of the first pass: element (g, j) of a thread sits at
// transform index base[g] + j*SMIN of pass 0 (the layout run_pass gathers).
template <int LOGN, int LOGE, bool INV>
__device__ __forceinline__ void gather_pass0(double (&x)[1 << LOGE], const double* __restrict__ src, const int tid) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, T = S::T;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(0);
  constexpr int SZ = 1 << C;
  constexpr int G = S::E >> C;
  constexpr int SMIN = INV ? 1 : (N >> C);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int sid = g * T + tid;
    const int base = INV ? sid * SZ : sid;     // pass 0: one block (forward) / contiguous sets (inverse)
#pragma unroll
    for (int j = 0; j < SZ; ++j) {
      const int gi = base + j * SMIN;
      x[g * SZ + j] = src[INV ? ntt_store(gi, LOGN) : gi];
    }
  }
}

// Persistent transform: each workgroup walks limbs blockIdx.x, blockIdx.x +
// gridDim.x, ... and prefetches the next limb into registers before
// transforming the current one, so HBM latency overlaps the LDS passes.
template <int LOGN, int LOGE, bool INV>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ntt_persist(double* __restrict__ data, int total, Basis basis, Tables tb, int zero) {
  constexpr int N = 1 << LOGN;
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  double x[1 << LOGE], xn[1 << LOGE];
  int limb = blockIdx.x;
  if (limb >= total) return;
  gather_pass0<LOGN, LOGE, INV>(x, data + (size_t)limb * N, tid);
  while (limb < total) {
    const int next = limb + gridDim.x;
    // `zero` is 0 at run time: keeps per-pass address arithmetic inside the loop (no hoisting
    // into registers, which would halve occupancy)
    const int z = limb & zero;
    if (next < total) gather_pass0<LOGN, LOGE, INV>(xn, data + (size_t)next * N, tid + z);
    const int pid = basis.id[limb % basis.n];
    const Mod m = tb.mods[pid];
    const double* tw = INV ? tb.inv + (size_t)pid * N : tb.fwd + (size_t)pid * N;
    const double* post = tb.post + (size_t)pid * N;
    double* a = data + (size_t)limb * N;
    run_pass<LOGN, LOGE, INV, 0, true, false>(x, lds + z, nullptr, a, tw, post, m, tid + z);
#pragma unroll
    for (int i = 0; i < (1 << LOGE); ++i) x[i] = xn[i];
    limb = next;
  }
}

// Square in the transform domain, fused: for one limb of one ciphertext
// (a0, a1 in coefficient form over Q then the auxiliary primes) writes, in
// coefficient form, d0 = a0^2, d1 = 2 a0 a1 and d2 = a1^2 (products in the
// transform domain).  The forward transform ends in the register layout the
// inverse transform starts from, so the products and inverse transforms work on
// registers.  At most two register sets are live (so two workgroups share a CU):
// A1^2 is parked in d2's own output words (each thread re-reads only what it wrote)
// while A0^2 and 2 A0 A1 are inverse-transformed, then transformed into d2.
template <int LOGN, int LOGE>
__global__ void __launch_bounds__(1 << (LOGN - LOGE)) __attribute__((amdgpu_waves_per_eu(LOGE <= 4 ? 4 : 2)))
k_square_fused(const double* __restrict__ in, double* __restrict__ out, Basis basis, Tables tb) {
  constexpr int N = 1 << LOGN;
  constexpr int E = 1 << LOGE;
  constexpr int T = N / E;
  extern __shared__ double lds[];
  const int nb = basis.n, nct = gridDim.x / nb;
  const int w = xcd_order(blockIdx.x, gridDim.x);
  const int limb = w / nct, ct = w - limb * nct;
  const int pid = basis.id[limb];
  const Mod m = tb.mods[pid];
  const double* fw = tb.fwd + (size_t)pid * N;
  const double* iw = tb.inv + (size_t)pid * N;
  const double* post = tb.post + (size_t)pid * N;
  const double* a0 = in + ((size_t)(ct * 2) * nb + limb) * N;
  const double* a1 = in + ((size_t)(ct * 2 + 1) * nb + limb) * N;
  double* d0 = out + ((size_t)(ct * 3) * nb + limb) * N;
  double* d1 = d0 + (size_t)nb * N;
  double* d2 = d1 + (size_t)nb * N;
  const int tid = threadIdx.x;
  double x0[E], x1[E];
  run_pass<LOGN, LOGE, false, 0, false, true>(x0, lds, a0, nullptr, fw, post, m, tid);
  __syncthreads();
  run_pass<LOGN, LOGE, false, 0, false, true>(x1, lds, a1, nullptr, fw, post, m, tid);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const double r0 = reduce(x0[i], m);
    const double r1 = reduce(x1[i], m);
    d2[i * T + tid] = mul_mod(r1, r1, m);     // parked: lane-consecutive, read back by this thread
    const double p = mul_mod(r0, r1, m);
    x1[i] = add_mod(p, p, m);
    x0[i] = mul_mod(r0, r0, m);
  }
  run_pass<LOGN, LOGE, true, 0, true, false>(x1, lds, nullptr, d1, iw, post, m, tid);
  run_pass<LOGN, LOGE, true, 0, true, false>(x0, lds, nullptr, d0, iw, post, m, tid);
#pragma unroll
  for (int i = 0; i < E; ++i) x1[i] = d2[i * T + tid];
  // the inverse transform's first exchange is a workgroup barrier that every thread reaches
  // only after consuming its parked words, so its final stores into d2 cannot overtake a
  // slower thread's reads
  run_pass<LOGN, LOGE, true, 0, true, false>(x1, lds, nullptr, d2, iw, post, m, tid);
}

// One persistent launch over transform work of several contexts: ring degrees 4096, 8192
// and 16384 with each context's own prime tables.  The work list holds items, each a batch of
// limbs of one context; every workgroup walks the units blockIdx.x, blockIdx.x + gridDim.x, ...
// of the concatenated list (whole limbs), so one grid sized to the device serves requests of
// uneven ring degree and prime count.  All three degrees run with 512 threads (2^(logn-9)
// residues per thread) and the LDS holds the largest degree of the list.
template <bool INV>
__global__ void __launch_bounds__(512) k_ntt_multi(MultiNttWork w) {
  extern __shared__ double lds[];
  for (int u = blockIdx.x; u < w.total; u += gridDim.x) {
    int k = 0, base = 0;
    while (k + 1 < w.n_items && u >= base + w.it[k].units) {
      base += w.it[k].units;
      ++k;
    }
    const int logn = w.it[k].logn, nl = w.it[k].n_limbs;
    const int local = u - base, limb = local % nl, poly = local / nl;
    const Tables tb = w.it[k].tb;
    const int pid = w.it[k].first_prime + limb;
    const Mod m = tb.mods[pid];
    const size_t N = (size_t)1 << logn;
    double* a = w.it[k].data + ((size_t)poly * nl + limb) * N;
    const double* tw = INV ? tb.inv + (size_t)pid * N : tb.fwd + (size_t)pid * N;
    const double* post = tb.post + (size_t)pid * N;
    if (logn == 12) {
      double x[8];
      run_pass<12, 3, INV, 0>(x, lds, a, a, tw, post, m, threadIdx.x);
    } else if (logn == 13) {
      double x[16];
      run_pass<13, 4, INV, 0>(x, lds, a, a, tw, post, m, threadIdx.x);
    } else {
      double x[32];
      run_pass<14, 5, INV, 0>(x, lds, a, a, tw, post, m, threadIdx.x);
    }
    __syncthreads();   // the next unit reuses the LDS
  }
}

template <int LOGN, int LOGE, bool INV>
void launch(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const size_t lds = (size_t)N * sizeof(double);
  const unsigned blocks = (unsigned)n_polys * b.n;
  if (blocks == 0) return;
  if (c.ntt_xlane && LOGE == 4)
    hipLaunchKernelGGL((k_ntt<LOGN, LOGE, INV, false, true>), dim3(blocks), dim3(N >> LOGE), lds, s, data, b, c.tab);
  else if (c.ntt_prefetch)
    hipLaunchKernelGGL((k_ntt<LOGN, LOGE, INV, true>), dim3(blocks), dim3(N >> LOGE), lds, s, data, b, c.tab);
  else
    hipLaunchKernelGGL((k_ntt<LOGN, LOGE, INV, false>), dim3(blocks), dim3(N >> LOGE), lds, s, data, b, c.tab);
  BCN_HIP(hipGetLastError());
}

// Key switching, fused: for one target limb (prime p of Q_level + P) of one
// source polynomial x (coefficient form over Q_level), accumulates
//   u_k = sum_j NTT(D_j mod p) * key_j[k]   (k = 0, 1)
// over the digits D_j = lift_c([sigma(x)]_{Q_j}) and writes INTT(u_0), INTT(u_1).
// The digits are formed in registers from the source residues (with the
// Galois automorphism sigma folded into the gather; kinv = 1 means none), so
// neither the digits nor the transform-domain products go through HBM.
struct KsDigits {
  const Conv* cv[8];   // digit j: source primes -> Q_level + P (used when the digit has 2 primes)
  int lo[8];           // first Q limb of digit j
  int na[8];           // primes of digit j present at this level
};

template <int LOGN, int LOGE, int NA, bool GAL>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ks_fused(const double* __restrict__ src, size_t src_stride, int level, int L, int dnum, KsDigits dg,
           const double* __restrict__ key, int kinv, double* __restrict__ u, Basis qp, Tables tb, int zero) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, E = S::E, T = S::T;
  constexpr int C0 = S::C0;
  constexpr int SMIN0 = N >> C0, SZ0 = 1 << C0, G0 = E >> C0;
  extern __shared__ double lds[];
  const int nb = qp.n, nct = gridDim.x / nb;
  const int w = xcd_order(blockIdx.x, gridDim.x);
  const int limb = w / nct, ct = w - limb * nct;
  const int pid = qp.id[limb];
  const Mod m = tb.mods[pid];
  const double* fw = tb.fwd + (size_t)pid * N;
  const double* iw = tb.inv + (size_t)pid * N;
  const double* post = tb.post + (size_t)pid * N;
  const double* xs = src + (size_t)ct * src_stride;
  const int KL = L + (nb - level);
  const int klimb = limb < level ? limb : L + (limb - level);
  const int tid = threadIdx.x;
  double acc0[E], acc1[E], x[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc0[i] = acc1[i] = 0.0;
  for (int j = 0; j < dnum; ++j) {
    const int lo = dg.lo[j], na = dg.na[j];
    const bool inside = limb >= lo && limb < lo + na;
    const Mod mq = tb.mods[lo];                      // Q prime ids equal their limb index
#pragma unroll
    for (int g = 0; g < G0; ++g)
#pragma unroll
      for (int jj = 0; jj < SZ0; ++jj) {
        const int pos = g * T + tid + jj * SMIN0;
        int sp = pos;
        bool flip = false;
        if (GAL) {
          const int i2 = (int)(((long long)pos * kinv) & (2 * N - 1));
          flip = i2 >= N;
          sp = flip ? i2 - N : i2;
        }
        double v;
        if (inside) {
          v = xs[(size_t)limb * N + sp];
        } else if (NA == 1 || na == 1) {
          const double xv = xs[(size_t)lo * N + sp];
          const double c = xv > (mq.q - 1.0) * 0.5 ? xv - mq.q : xv;   // |c| < q_j / 2 < p
          v = c < 0.0 ? c + m.q : c;
        } else {
          const Conv& cv = *dg.cv[j];
          const double xa[2] = {xs[(size_t)lo * N + sp], xs[(size_t)(lo + 1) * N + sp]};
          double va[2];
          garner<2>(xa, va, cv, tb.mods);
          double a = mul_lazy(va[1], cv.pm[limb][0], m) + va[0];
          if (above_half<2>(va, 2, cv, tb.mods)) a -= cv.Mmod[limb];
          v = reduce(a, m);
        }
        if (flip) v = v == 0.0 ? 0.0 : m.q - v;
        x[g * SZ0 + jj] = v;
      }
    // `zero` is 0 at run time; indexing through it keeps the per-pass address
    // arithmetic inside the digit loop instead of hoisting it into registers
    run_pass<LOGN, LOGE, false, 0, true, true>(x, lds + (j & zero), nullptr, nullptr, fw, post, m, tid + (j & zero));
    // the forward transform leaves indices tid * E + i in the registers; the keys are
    // stored in transform-domain storage order
    const double* k0 = key + ((size_t)(j * 2) * KL + klimb) * N;
    const double* k1 = key + ((size_t)(j * 2 + 1) * KL + klimb) * N;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int p = ntt_store(tid * E + i, LOGN);
      acc0[i] += mul_lazy(k0[p], x[i], m);
      acc1[i] += mul_lazy(k1[p], x[i], m);
    }
  }
  double* u0 = u + ((size_t)(ct * 2) * nb + limb) * N;
  double* u1 = u + ((size_t)(ct * 2 + 1) * nb + limb) * N;
#pragma unroll
  for (int i = 0; i < E; ++i) x[i] = reduce(acc0[i], m);
  run_pass<LOGN, LOGE, true, 0, true, false>(x, lds, nullptr, u0, iw, post, m, tid);
#pragma unroll
  for (int i = 0; i < E; ++i) x[i] = reduce(acc1[i], m);
  run_pass<LOGN, LOGE, true, 0, true, false>(x, lds, nullptr, u1, iw, post, m, tid);
}

template <int LOGN, int LOGE, bool INV>
void launch_persist(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const int total = n_polys * b.n;
  if (total == 0) return;
  const int grid = std::min(total, c.persist_blocks);
  hipLaunchKernelGGL((k_ntt_persist<LOGN, LOGE, INV>), dim3(grid), dim3(N >> LOGE), (size_t)N * sizeof(double), s, data,
                     total, b, c.tab, 0);
  BCN_HIP(hipGetLastError());
}


template <int LOGN, int LOGE>
void launch_ks(const Context& c, const double* src, size_t stride, int n, int level, const KsDigits& dg,
               const double* key, int kinv, double* u, const Basis& qp, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const unsigned blocks = (unsigned)n * qp.n;
  if (blocks == 0) return;
#define BCN_KSL(NA, GAL)                                                                                 \
  hipLaunchKernelGGL((k_ks_fused<LOGN, LOGE, NA, GAL>), dim3(blocks), dim3(N >> LOGE), (size_t)N * sizeof(double), s, \
                     src, stride, level, c.L, c.dnum(level), dg, key, kinv, u, qp, c.tab, 0)
  if (c.alpha == 1) {
    if (kinv == 1) BCN_KSL(1, false); else BCN_KSL(1, true);
  } else {
    if (kinv == 1) BCN_KSL(2, false); else BCN_KSL(2, true);
  }
#undef BCN_KSL
  BCN_HIP(hipGetLastError());
}

// Key-switching digits straight into the transform domain.  Block (poly, digit j,
// target limb) forms D_j = lift_c([x]_{Q_j}) mod the target prime while gathering
// the forward transform's first pass from the source residues, transforms it and
// stores it in transform-domain order at D[poly][j][limb] (the layout the four-kernel
// path builds with ModUp and a forward transform).  store_gal = k^-1 != 1 stores the
// digits of sigma_k(x) (the transform-domain permutation applied on the store).
template <int LOGN, int LOGE, int NA>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ntt_digits(const double* __restrict__ src, size_t src_stride, int dnum, KsDigits dg, double* __restrict__ D,
             Basis qp, Tables tb, int store_gal) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, E = S::E, T = S::T;
  constexpr int C0 = S::C0;
  constexpr int SMIN0 = N >> C0, SZ0 = 1 << C0, G0 = E >> C0;
  extern __shared__ double lds[];
  const int nb = qp.n;
  // consecutive blocks (one XCD) take the target limbs of one (poly, digit): the
  // digit's source residues are read once from HBM and then hit that XCD's L2
  const int w = xcd_order(blockIdx.x, gridDim.x);
  const int limb = w % nb, pj = w / nb;
  const int j = pj % dnum, poly = pj / dnum;
  const int pid = qp.id[limb];
  const Mod m = tb.mods[pid];
  const double* xs = src + (size_t)poly * src_stride;
  const int lo = dg.lo[j], na = dg.na[j];
  const bool inside = limb >= lo && limb < lo + na;
  const Mod mq = tb.mods[lo];                      // Q prime ids equal their limb index
  const int tid = threadIdx.x;
  double x[E];
#pragma unroll
  for (int g = 0; g < G0; ++g)
#pragma unroll
    for (int jj = 0; jj < SZ0; ++jj) {
      const int sp = g * T + tid + jj * SMIN0;
      double v;
      if (inside) {
        v = xs[(size_t)limb * N + sp];
      } else if (NA == 1 || na == 1) {
        const double xv = xs[(size_t)lo * N + sp];
        const double c = xv > (mq.q - 1.0) * 0.5 ? xv - mq.q : xv;   // |c| < q_j / 2 < p
        v = c < 0.0 ? c + m.q : c;
      } else {
        const Conv& cv = *dg.cv[j];
        const double xa[2] = {xs[(size_t)lo * N + sp], xs[(size_t)(lo + 1) * N + sp]};
        double va[2];
        garner<2>(xa, va, cv, tb.mods);
        double a = mul_lazy(va[1], cv.pm[limb][0], m) + va[0];
        if (above_half<2>(va, 2, cv, tb.mods)) a -= cv.Mmod[limb];
        v = reduce(a, m);
      }
      x[g * SZ0 + jj] = v;
    }
  run_pass<LOGN, LOGE, false, 0, true, false>(x, lds, nullptr, D + ((size_t)pj * nb + limb) * N,
                                              tb.fwd + (size_t)pid * N, tb.post, m, tid, nullptr, store_gal);
}

// Key-switching inner product fused into the inverse transforms.  Block (output o,
// target limb) accumulates u_k = sum_j sigma(D_j^) * key_j[k] (k = 0, 1; sigma the
// transform-domain Galois permutation of output o's key, none for
// relinearisation) while gathering the inverse transform's first pass, then
// inverse-transforms both accumulators into u[o][k][limb] (coefficient form).
// Output o reads the digits of source o / d_div.  SPLIT: a block computes only one of the two
// parts (twice the blocks, each with half the inner product and one inverse transform), for
// launches too small to fill the device, whose time is the latency of one block.
//
// EXT: no inverse transform (the taps of a convolution kept over Q_l P, see ks_extended).
// The block adds P sigma(c0^) on the Q limbs of part 0 (the source's transformed part 0,
// staged in LDS like a digit limb) and stores both parts in the transform domain at
// u + (o / out_div) out_outer + (o % out_div) 2 (level + K) N.
template <int LOGN, int LOGE, bool SPLIT, bool EXT = false>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ks_intt(const double* __restrict__ D, int d_div, KeySel ka, int level, int dnum, int L, Basis qp, Tables tb,
          double* __restrict__ u, KsExt ext) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, E = S::E, T = S::T;
  constexpr int C0 = Sched<LOGN, LOGE, true>::c(0);
  constexpr int SZ0 = 1 << C0, G0 = E >> C0;
  extern __shared__ double lds[];
  const int nb = qp.n, nout = gridDim.x / (nb * (SPLIT ? 2 : 1));
  // limb-major: the blocks of one XCD share one or two target limbs, so that limb's key
  // parts (2 dnum limbs, read by every output) stay in that XCD's L2
  const int wx = xcd_order(blockIdx.x, gridDim.x);
  const int part = SPLIT ? (wx & 1) : 0;
  const int w = SPLIT ? (wx >> 1) : wx;
  const int limb = w / nout, o = w - limb * nout;
  const int pid = qp.id[limb];
  const Mod m = tb.mods[pid];
  const int sel = o % ka.nk;
  const int gal = ka.keys ? ka.galois[sel] : ka.galois1;
  const double* key = ka.keys ? ka.keys[sel] : ka.key1;
  const double* dd = D + (size_t)(o / d_div) * dnum * nb * N + (size_t)limb * N;
  const int klimb = limb < level ? limb : L + (limb - level);
  const int KL = nb - level + L;                   // limbs of a key part (L + K)
  const int tid = threadIdx.x;
  // The inverse transform's first pass holds transform indices (g * T + tid) * SZ0 + jj.
  // Elements are gathered in chunks of CH: all loads of a chunk (CH digit words and 2 CH
  // key words per digit) are issued before any is consumed, so a chunk costs one memory
  // round trip per digit instead of one per element and digit.
  constexpr int CH = 4;
  double x[E], acc1[E];
  if (gal != 1) {
    // Rotations: the Galois permutation scatters the digit reads over the whole limb.  Each
    // digit limb is staged in LDS with coalesced loads and the permuted reads come from LDS;
    // the key words are read in storage order (coalesced) as before.
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = acc1[e] = 0.0;
    for (int j = 0; j < dnum; ++j) {
      const double* dj = dd + (size_t)j * nb * N;
      __syncthreads();                       // the previous digit's reads are done
      stage_to_lds(lds, dj, N, tid, T);
      const double* k0 = key + ((size_t)(j * 2 + part) * KL + klimb) * N;
      const double* k1 = key + ((size_t)(j * 2 + 1) * KL + klimb) * N;
#pragma unroll
      for (int c0 = 0; c0 < E; c0 += CH) {
        int pos[CH];
        double dv[CH], kv0[CH], kv1[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
          const int gi = ((c0 + e) / SZ0 * T + tid) * SZ0 + (c0 + e) % SZ0;
          pos[e] = ntt_store(gi, LOGN);
          dv[e] = lds[ntt_store(ntt_perm(gi, gal, LOGN), LOGN)];
        }
#pragma unroll
        for (int e = 0; e < CH; ++e) {
          kv0[e] = k0[pos[e]];
          if (!SPLIT) kv1[e] = k1[pos[e]];
        }
#pragma unroll
        for (int e = 0; e < CH; ++e) {
          x[c0 + e] += mul_lazy(dv[e], kv0[e], m);
          if (!SPLIT) acc1[c0 + e] += mul_lazy(dv[e], kv1[e], m);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      x[e] = reduce(x[e], m);
      if (!SPLIT) acc1[e] = reduce(acc1[e], m);
    }
    __syncthreads();                         // the transform's exchanges reuse the LDS
  } else {
#pragma unroll
  for (int c0 = 0; c0 < E; c0 += CH) {
    int pos[CH], srcw[CH];
#pragma unroll
    for (int e = 0; e < CH; ++e) {
      const int gi = ((c0 + e) / SZ0 * T + tid) * SZ0 + (c0 + e) % SZ0;
      pos[e] = ntt_store(gi, LOGN);
      srcw[e] = pos[e];
    }
    double a0[CH], a1[CH];
#pragma unroll
    for (int e = 0; e < CH; ++e) a0[e] = a1[e] = 0.0;
    for (int j = 0; j < dnum; ++j) {
      const double* dj = dd + (size_t)j * nb * N;
      const double* k0 = key + ((size_t)(j * 2 + part) * KL + klimb) * N;
      const double* k1 = key + ((size_t)(j * 2 + 1) * KL + klimb) * N;
      double dv[CH], kv0[CH], kv1[CH];
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        dv[e] = dj[srcw[e]];
        kv0[e] = k0[pos[e]];
        if (!SPLIT) kv1[e] = k1[pos[e]];
      }
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        a0[e] += mul_lazy(dv[e], kv0[e], m);
        if (!SPLIT) a1[e] += mul_lazy(dv[e], kv1[e], m);
      }
    }
#pragma unroll
    for (int e = 0; e < CH; ++e) {
      x[c0 + e] = reduce(a0[e], m);
      if (!SPLIT) acc1[c0 + e] = reduce(a1[e], m);
    }
  }
  }
  if constexpr (EXT) {
    if (limb < level && part == 0) {
      // P sigma(c0^): the source's part 0 limb staged in LDS, read through the permutation
      const double* c0 = ext.c0hat + (size_t)(o / d_div) * ext.c0_stride + (size_t)limb * N;
      __syncthreads();
      stage_to_lds(lds, c0, N, tid, T);
      const double pm = ext.pm[limb];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int gi = (e / SZ0 * T + tid) * SZ0 + e % SZ0;
        const double v = lds[gal == 1 ? ntt_store(gi, LOGN) : ntt_store(ntt_perm(gi, gal, LOGN), LOGN)];
        x[e] = reduce(x[e] + mul_lazy(v, pm, m), m);
      }
    }
    double* dst = u + (size_t)(o / ext.out_div) * ext.out_outer + (size_t)(o % ext.out_div) * 2 * nb * N +
                  (size_t)limb * N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = ntt_store((e / SZ0 * T + tid) * SZ0 + e % SZ0, LOGN);
      dst[(size_t)part * nb * N + pos] = x[e];
      if (!SPLIT) dst[(size_t)nb * N + pos] = acc1[e];
    }
    return;
  }
  const double* iw = tb.inv + (size_t)pid * N;
  const double* post = tb.post + (size_t)pid * N;
  run_pass<LOGN, LOGE, true, 0, true, false>(x, lds, nullptr, u + ((size_t)(o * 2 + part) * nb + limb) * N, iw, post,
                                             m, tid);
  if (!SPLIT)
    run_pass<LOGN, LOGE, true, 0, true, false>(acc1, lds, nullptr, u + ((size_t)(o * 2 + 1) * nb + limb) * N, iw,
                                               post, m, tid);
}

template <int LOGN, int LOGE>
void launch_ks_split(const Context& c, int part, const double* src, size_t stride, int n_src, int level,
                     const KsDigits& dg, double* D, const KeySel& ks, int n_out, int d_div, double* u, const Basis& qp,
                     int store_gal, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const size_t lds = (size_t)N * sizeof(double);
  const int dnum = c.dnum(level);
  const unsigned b1 = part == 1 ? (unsigned)n_src * dnum * qp.n : 0u;
  if (b1 > 0) {
    if (c.alpha == 1)
      hipLaunchKernelGGL((k_ntt_digits<LOGN, LOGE, 1>), dim3(b1), dim3(N >> LOGE), lds, s, src, stride, dnum, dg, D, qp,
                         c.tab, store_gal);
    else
      hipLaunchKernelGGL((k_ntt_digits<LOGN, LOGE, 2>), dim3(b1), dim3(N >> LOGE), lds, s, src, stride, dnum, dg, D, qp,
                         c.tab, store_gal);
    BCN_HIP(hipGetLastError());
  }
  const unsigned b2 = part == 2 ? (unsigned)n_out * qp.n : 0u;
  if (b2 > 0 && (int)b2 < c.n_cus) {
    // too few blocks to fill the device: one block per part halves each block's latency
    hipLaunchKernelGGL((k_ks_intt<LOGN, LOGE, true>), dim3(2 * b2), dim3(N >> LOGE), lds, s, D, d_div, ks, level, dnum,
                       c.L, qp, c.tab, u, KsExt());
  } else if (b2 > 0) {
    hipLaunchKernelGGL((k_ks_intt<LOGN, LOGE, false>), dim3(b2), dim3(N >> LOGE), lds, s, D, d_div, ks, level, dnum,
                       c.L, qp, c.tab, u, KsExt());
    BCN_HIP(hipGetLastError());
  }
}

// One round of a rotate-and-sum: block (source i, limb, part) accumulates over every step of
// the key table u = sum_sel sum_j sigma_sel(D_j^) key_sel,j[part] + P c^part + (part 0, Q limbs)
// sum_sel P sigma_sel(c0^): the taps of the round kept over Q_l P and already summed.  Each
// digit limb (and c0^'s limb) is staged once in LDS and read through every step's permutation;
// the key words are read in storage order.  u is stored in the transform domain
// ([n][2][level + K][N]).  The sum has at most 1 + nk (dnum + 1) lazy terms below q, exact for
// nk <= 256.
template <int LOGN, int LOGE>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ks_sum(const double* __restrict__ D, KeySel ka, int level, int dnum, int L, Basis qp, Tables tb,
         const double* __restrict__ chat, size_t c_stride, KsExt ext, int groups, double* __restrict__ u) {
  constexpr int N = 1 << LOGN, E = 1 << LOGE, T = N >> LOGE;
  extern __shared__ double lds[];
  const int nb = qp.n;
  const int n_src = gridDim.x / (nb * 2 * groups);
  // limb-major: the blocks of one XCD share a limb, whose key words they read in step
  const int wx = xcd_order(blockIdx.x, gridDim.x);
  const int part = wx & 1;
  const int w = (wx >> 1) / groups, grp = (wx >> 1) % groups;
  const int limb = w / n_src, i = w - limb * n_src;
  // group grp takes steps [s0, s1) of the table and writes its partial sum to slab grp
  const int s0 = grp * ka.nk / groups, s1 = (grp + 1) * ka.nk / groups;
  u += (size_t)grp * n_src * 2 * nb * N;
  const Mod m = tb.mods[qp.id[limb]];
  const double* dd = D + (size_t)i * dnum * nb * N + (size_t)limb * N;
  const int klimb = limb < level ? limb : L + (limb - level);
  const int KL = nb - level + L;
  const int tid = threadIdx.x;
  int ti[E];                                       // transform index of element e (word e T + tid)
  double acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ti[e] = ntt_index(e * T + tid, LOGN);
    acc[e] = 0.0;
  }
  if (limb < level && grp == 0) {
    const double* cp = chat + (size_t)i * c_stride + ((size_t)part * level + limb) * N;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = mul_lazy(cp[e * T + tid], ext.pm[limb], m);
  }
  for (int j = 0; j < dnum; ++j) {
    const double* dj = dd + (size_t)j * nb * N;
    __syncthreads();
    stage_to_lds(lds, dj, N, tid, T);
    for (int sel = s0; sel < s1; ++sel) {
      const int gal = ka.galois[sel];
      const double* kp = ka.keys[sel] + ((size_t)(j * 2 + part) * KL + klimb) * N;
#pragma unroll
      for (int e = 0; e < E; ++e)
        acc[e] += mul_lazy(lds[ntt_store(ntt_perm(ti[e], gal, LOGN), LOGN)], kp[e * T + tid], m);
    }
  }
  if (part == 0 && limb < level) {
    const double* c0 = chat + (size_t)i * c_stride + (size_t)limb * N;
    __syncthreads();
    stage_to_lds(lds, c0, N, tid, T);
    const double pm = ext.pm[limb];
    for (int sel = s0; sel < s1; ++sel) {
      const int gal = ka.galois[sel];
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] += mul_lazy(lds[ntt_store(ntt_perm(ti[e], gal, LOGN), LOGN)], pm, m);
    }
  }
  double* dst = u + ((size_t)(i * 2 + part) * nb + limb) * N;
#pragma unroll
  for (int e = 0; e < E; ++e) dst[e * T + tid] = reduce(acc[e], m);
}

template <int LOGN, int LOGE>
void launch_ks_sum(const Context& c, int level, const double* D, const KeySel& ks, int n_src, const double* chat,
                   size_t c_stride, const KsExt& ext, int groups, double* u, const Basis& qp, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const unsigned blocks = (unsigned)n_src * qp.n * 2 * groups;
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_ks_sum<LOGN, LOGE>), dim3(blocks), dim3(N >> LOGE), (size_t)N * sizeof(double), s, D, ks,
                     level, c.dnum(level), c.L, qp, c.tab, chat, c_stride, ext, groups, u);
  BCN_HIP(hipGetLastError());
}

// the extended inner product (no inverse transform) of n_out outputs
template <int LOGN, int LOGE>
void launch_ks_ext(const Context& c, int level, const double* D, const KeySel& ks, int n_out, int d_div, double* u,
                   const Basis& qp, const KsExt& ext, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const size_t lds = (size_t)N * sizeof(double);
  const int dnum = c.dnum(level);
  const unsigned b2 = (unsigned)n_out * qp.n;
  if (b2 == 0) return;
  if ((int)b2 < c.n_cus)
    hipLaunchKernelGGL((k_ks_intt<LOGN, LOGE, true, true>), dim3(2 * b2), dim3(N >> LOGE), lds, s, D, d_div, ks, level,
                       dnum, c.L, qp, c.tab, u, ext);
  else
    hipLaunchKernelGGL((k_ks_intt<LOGN, LOGE, false, true>), dim3(b2), dim3(N >> LOGE), lds, s, D, d_div, ks, level,
                       dnum, c.L, qp, c.tab, u, ext);
  BCN_HIP(hipGetLastError());
}

template <int LOGN, int LOGE>
void set_attr() {
  const int lds = (1 << LOGN) * (int)sizeof(double);
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt_persist<LOGN, LOGE, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt_persist<LOGN, LOGE, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, false, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, true, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_square_fused<LOGN, LOGE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_fused<LOGN, LOGE, 1, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_fused<LOGN, LOGE, 2, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_fused<LOGN, LOGE, 1, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_fused<LOGN, LOGE, 2, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt_digits<LOGN, LOGE, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt_digits<LOGN, LOGE, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_intt<LOGN, LOGE, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_intt<LOGN, LOGE, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_sum<LOGN, LOGE>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_intt<LOGN, LOGE, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ks_intt<LOGN, LOGE, true, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds));
}

template <int LOGN, int LOGE>
void launch_square(const Context& c, const double* in, double* out, int n, const Basis& b, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const unsigned blocks = (unsigned)n * b.n;
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_square_fused<LOGN, LOGE>), dim3(blocks), dim3(N >> LOGE), (size_t)N * sizeof(double), s, in,
                     out, b, c.tab);
  BCN_HIP(hipGetLastError());
}

template <bool INV>
void dispatch(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  // algorithmic traffic: each limb read once and written once; algorithmic VALU work: 8 FP64
  // operations per butterfly (exact lazy product 6, add, subtract) and 4 per word at the end
  const double limbs = (double)n_polys * b.n;
  ProfScope ps(c, INV ? "ntt_inverse" : "ntt_forward", s, 16.0 * c.n * limbs,
               limbs * (8.0 * (c.n / 2) * c.logn + 4.0 * c.n));
  const int key = c.logn * 16 + c.ntt_loge;
  if (c.ntt_persist) {
    switch (key) {
#define BCN_NTTP_CASE(LN, LE) \
  case LN * 16 + LE: launch_persist<LN, LE, INV>(c, data, n_polys, b, s); return;
      BCN_NTTP_CASE(10, 3) BCN_NTTP_CASE(10, 4)
      BCN_NTTP_CASE(11, 3) BCN_NTTP_CASE(11, 4)
      BCN_NTTP_CASE(12, 4) BCN_NTTP_CASE(12, 5)
      BCN_NTTP_CASE(13, 4) BCN_NTTP_CASE(13, 5)
      BCN_NTTP_CASE(14, 4) BCN_NTTP_CASE(14, 5)
#undef BCN_NTTP_CASE
      default: throw Error(-1, "unsupported ring degree / transform shape");
    }
  }
  switch (key) {
#define BCN_NTT_CASE(LN, LE) \
  case LN * 16 + LE: launch<LN, LE, INV>(c, data, n_polys, b, s); break;
    BCN_NTT_CASE(10, 3) BCN_NTT_CASE(10, 4)
    BCN_NTT_CASE(11, 3) BCN_NTT_CASE(11, 4)
    BCN_NTT_CASE(12, 4) BCN_NTT_CASE(12, 5)
    BCN_NTT_CASE(13, 4) BCN_NTT_CASE(13, 5)
    BCN_NTT_CASE(14, 4) BCN_NTT_CASE(14, 5)
#undef BCN_NTT_CASE
    default: throw Error(-1, "unsupported ring degree / transform shape");
  }
}

}  // namespace

std::vector<int> Context::ntt_loge_options() const {
  switch (logn) {
    case 10: return {3, 4};
    case 11: return {3, 4};
    case 12: return {4, 5};
    case 13: return {4, 5};
    case 14: return {4, 5};
    default: return {};
  }
}

void ntt_multi(const std::vector<MultiNttItem>& items, bool inverse, hipStream_t s) {
  if (items.empty()) return;
  if ((int)items.size() > kMaxMultiItems) throw Error(-1, "too many items in one transform launch");
  MultiNttWork w{};
  int maxlog = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    if (items[i].logn < 12 || items[i].logn > 14) throw Error(-1, "multi-context transform: N must be 4096..16384");
    w.it[i] = items[i];
    w.total += items[i].units;
    maxlog = std::max(maxlog, items[i].logn);
  }
  w.n_items = (int)items.size();
  if (w.total == 0) return;
  static bool attr = false;
  if (!attr) {
    BCN_HIP(hipFuncSetAttribute((const void*)k_ntt_multi<false>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
    BCN_HIP(hipFuncSetAttribute((const void*)k_ntt_multi<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
    attr = true;
  }
  int dev = 0;
  BCN_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  BCN_HIP(hipGetDeviceProperties(&prop, dev));
  const size_t lds = ((size_t)1 << maxlog) * sizeof(double);
  const int per_cu = std::max(1, (int)(prop.maxSharedMemoryPerMultiProcessor / lds));
  const int grid = std::min(w.total, prop.multiProcessorCount * per_cu);
  if (inverse)
    hipLaunchKernelGGL(k_ntt_multi<true>, dim3(grid), dim3(512), lds, s, w);
  else
    hipLaunchKernelGGL(k_ntt_multi<false>, dim3(grid), dim3(512), lds, s, w);
  BCN_HIP(hipGetLastError());
}

void ntt_setup(const Context& c) {
  switch (c.logn) {
    case 10: set_attr<10, 3>(); set_attr<10, 4>(); break;
    case 11: set_attr<11, 3>(); set_attr<11, 4>(); break;
    case 12: set_attr<12, 4>(); set_attr<12, 5>(); break;
    case 13: set_attr<13, 4>(); set_attr<13, 5>(); break;
    case 14: set_attr<14, 4>(); set_attr<14, 5>(); break;
    default: throw Error(-1, "unsupported ring degree");
  }
}

void square_transform_fused(const Context& c, const double* in, double* out, int n, const Basis& b, hipStream_t s) {
  // algorithmic traffic: two limbs in, three limbs out per (ciphertext, limb); work: five
  // transforms, three products, two normalisations
  const double units = (double)n * b.n;
  ProfScope ps(c, "square_fused", s, 8.0 * c.n * units * 5,
               units * (5.0 * (8.0 * (c.n / 2) * c.logn + 4.0 * c.n) + 3.0 * 8.0 * c.n + 2.0 * 4.0 * c.n));
  const int key = c.logn * 16 + c.square_loge;
  switch (key) {
#define BCN_SQ_CASE(LN, LE) \
  case LN * 16 + LE: launch_square<LN, LE>(c, in, out, n, b, s); break;
    BCN_SQ_CASE(10, 3) BCN_SQ_CASE(10, 4)
    BCN_SQ_CASE(11, 3) BCN_SQ_CASE(11, 4)
    BCN_SQ_CASE(12, 4) BCN_SQ_CASE(12, 5)
    BCN_SQ_CASE(13, 4) BCN_SQ_CASE(13, 5)
    BCN_SQ_CASE(14, 4) BCN_SQ_CASE(14, 5)
#undef BCN_SQ_CASE
    default: throw Error(-1, "unsupported ring degree / transform shape");
  }
}

namespace {
KsDigits ks_digits(const Context& c, int level, const Basis& qp) {
  if (c.alpha > 2) throw Error(-1, "fused key switching supports digits of at most two primes");
  const int dnum = c.dnum(level);
  if (dnum > 8) throw Error(-1, "too many digits");
  KsDigits dg{};
  for (int j = 0; j < dnum; ++j) {
    const int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, level);
    dg.lo[j] = lo;
    dg.na[j] = hi - lo;
    dg.cv[j] = nullptr;
    if (hi - lo == 2) {
      std::vector<int> src_ids, dst;
      for (int i = lo; i < hi; ++i) src_ids.push_back(c.idQ(i));
      for (int i = 0; i < qp.n; ++i) dst.push_back(qp.id[i]);
      dg.cv[j] = conv_device(c, "ksd" + std::to_string(level) + "_" + std::to_string(j), make_conv(c, src_ids, dst));
    }
  }
  return dg;
}
}  // namespace

namespace {
// the first kernel of ks_split alone: digits of the sources into D
void ks_split_digits_only(const Context& c, const double* src, size_t src_stride, int n_src, int level, double* D,
                          hipStream_t s) {
  KeySel none;
  ks_split(c, src, src_stride, n_src, level, none, 0, 1, D, nullptr, s);
}
}  // namespace

void ks_split(const Context& c, const double* src, size_t src_stride, int n_src, int level, const KeySel& ks,
              int n_out, int d_div, double* D, double* u, hipStream_t s, int src_galois) {
  const Basis qp = c.basis_QP(level);
  const KsDigits dg = ks_digits(c, level, qp);
  const int dnum = c.dnum(level);
  const double tr = 8.0 * (c.n / 2) * c.logn + 4.0 * c.n;        // FP64 ops of one limb transform
  const int key = c.logn * 16 + c.ks_loge;
  const int store_gal = src_galois == 1 ? 1 : (int)host::inv_pow2((uint64_t)src_galois, c.logn + 1);
  for (int part = 1; part <= (n_out > 0 ? 2 : 1); ++part) {
    // digits: source limbs once, digits out, dnum * (level + K) forward transforms per source;
    // inner product: digits and two key parts in, two parts out, two inverse transforms per output limb
    const double u1 = (double)n_src * dnum * qp.n, u2 = (double)n_out * qp.n;
    ProfScope ps(c, part == 1 ? "ntt_digits" : "ks_intt", s,
                 part == 1 ? 8.0 * c.n * ((double)n_src * level + u1) : 8.0 * c.n * u2 * (dnum + 2.0),
                 part == 1 ? u1 * tr : u2 * (2.0 * tr + dnum * 2.0 * 7.0 * c.n));
    switch (key) {
#define BCN_KSS_CASE(LN, LE)                                                                                 \
  case LN * 16 + LE:                                                                                         \
    launch_ks_split<LN, LE>(c, part, src, src_stride, n_src, level, dg, D, ks, n_out, d_div, u, qp, store_gal, s); break;
      BCN_KSS_CASE(10, 3) BCN_KSS_CASE(10, 4)
      BCN_KSS_CASE(11, 3) BCN_KSS_CASE(11, 4)
      BCN_KSS_CASE(12, 4) BCN_KSS_CASE(12, 5)
      BCN_KSS_CASE(13, 4) BCN_KSS_CASE(13, 5)
      BCN_KSS_CASE(14, 4) BCN_KSS_CASE(14, 5)
#undef BCN_KSS_CASE
      default: throw Error(-1, "unsupported ring degree / transform shape");
    }
  }
}

void ks_extended(const Context& c, const double* src, size_t src_stride, int n_src, int level, const KeySel& ks,
                 int n_out, int d_div, double* D, double* u, const KsExt& ext, hipStream_t s) {
  // the digits as for a complete key switch, then the inner products with no inverse transform
  ks_split_digits_only(c, src, src_stride, n_src, level, D, s);
  const Basis qp = c.basis_QP(level);
  const int dnum = c.dnum(level);
  const double u2 = (double)n_out * qp.n;
  // algorithmic bytes: each distinct limb once (every source's digits and transformed part 0, every
  // key's two parts, the outputs); the re-reads of digits and keys by other outputs hit the caches
  const double nk = ks.keys ? ks.nk : 1.0;
  ProfScope ps(c, "ks_ext", s,
               8.0 * c.n * ((double)n_src * (dnum * qp.n + level) + nk * dnum * 2.0 * qp.n + 2.0 * u2),
               u2 * dnum * 2.0 * 7.0 * c.n);
  const int key = c.logn * 16 + c.ks_loge;
  switch (key) {
#define BCN_KSE_CASE(LN, LE) \
  case LN * 16 + LE: launch_ks_ext<LN, LE>(c, level, D, ks, n_out, d_div, u, qp, ext, s); break;
    BCN_KSE_CASE(10, 3) BCN_KSE_CASE(10, 4)
    BCN_KSE_CASE(11, 3) BCN_KSE_CASE(11, 4)
    BCN_KSE_CASE(12, 4) BCN_KSE_CASE(12, 5)
    BCN_KSE_CASE(13, 4) BCN_KSE_CASE(13, 5)
    BCN_KSE_CASE(14, 4) BCN_KSE_CASE(14, 5)
#undef BCN_KSE_CASE
    default: throw Error(-1, "unsupported ring degree / transform shape");
  }
}

void ks_sum_round(const Context& c, const double* src, size_t src_stride, int n, int level, const KeySel& ks,
                  const double* chat, size_t c_stride, const KsExt& ext, double* D, double* u, hipStream_t s) {
  if (!ks.keys || ks.nk < 1 || ks.nk > 256) throw Error(-1, "a rotate-and-sum round takes 1..256 keys");
  ks_split_digits_only(c, src, src_stride, n, level, D, s);
  const Basis qp = c.basis_QP(level);
  const int dnum = c.dnum(level);
  const double units = (double)n * qp.n * 2;
  // the steps are split into groups so that the launch has about two blocks per CU; the groups'
  // partial sums are added by sum_slabs
  double per_cu = 2.0;
  if (const char* e = std::getenv("BCN_KS_SUM_PER_CU")) per_cu = std::max(0.25, std::atof(e));
  const int groups = std::max(1, std::min(ks.nk, (int)((per_cu * c.n_cus) / units)));
  double* part_u = groups > 1 ? c.arena->take((size_t)groups * n * 2 * qp.n * c.n) : u;
  // algorithmic bytes: each distinct limb once (the sources' digits and transformed parts, the steps'
  // key parts, the partial sums out); products: every step's digits and P sigma(c0^) terms
  ProfScope ps(c, "ks_sum", s,
               8.0 * c.n * ((double)n * (dnum * qp.n + 2.0 * level) + (double)ks.nk * dnum * 2.0 * qp.n +
                            (double)groups * n * 2.0 * qp.n),
               units * ks.nk * (dnum + 1.0) * 7.0 * c.n);
  const int key = c.logn * 16 + c.ks_loge;
  switch (key) {
#define BCN_KSM_CASE(LN, LE) \
  case LN * 16 + LE: launch_ks_sum<LN, LE>(c, level, D, ks, n, chat, c_stride, ext, groups, part_u, qp, s); break;
    BCN_KSM_CASE(10, 3) BCN_KSM_CASE(10, 4)
    BCN_KSM_CASE(11, 3) BCN_KSM_CASE(11, 4)
    BCN_KSM_CASE(12, 4) BCN_KSM_CASE(12, 5)
    BCN_KSM_CASE(13, 4) BCN_KSM_CASE(13, 5)
    BCN_KSM_CASE(14, 4) BCN_KSM_CASE(14, 5)
#undef BCN_KSM_CASE
    default: throw Error(-1, "unsupported ring degree / transform shape");
  }
  if (groups > 1) sum_slabs(c, part_u, groups, (size_t)n * 2 * qp.n * c.n, n * 2, qp, u, s);
}

void ks_fused(const Context& c, const double* src, size_t src_stride, int n, int level, const double* key, int galois,
              double* u, hipStream_t s) {
  const Basis qp = c.basis_QP(level);
  const KsDigits dg = ks_digits(c, level, qp);
  const int dnum = c.dnum(level);
  const int kinv = galois == 1 ? 1 : (int)host::inv_pow2((uint64_t)galois, c.logn + 1);
  // algorithmic traffic: digit sources (level limbs per target limb), two key limbs per digit, two outputs
  const double units = (double)n * qp.n;
  ProfScope ps(c, "ks_fused", s, 8.0 * c.n * units * (level + 2.0 * dnum + 2),
               units * ((dnum + 2.0) * (8.0 * (c.n / 2) * c.logn + 4.0 * c.n) + dnum * 2.0 * 7.0 * c.n));
  // two accumulators and the working set stay in registers (sixteen residues per
  // thread; spill-free up to N = 8192)
  switch (c.logn) {
    case 10: launch_ks<10, 4>(c, src, src_stride, n, level, dg, key, kinv, u, qp, s); break;
    case 11: launch_ks<11, 4>(c, src, src_stride, n, level, dg, key, kinv, u, qp, s); break;
    case 12: launch_ks<12, 4>(c, src, src_stride, n, level, dg, key, kinv, u, qp, s); break;
    case 13: launch_ks<13, 4>(c, src, src_stride, n, level, dg, key, kinv, u, qp, s); break;
    default: throw Error(-1, "fused key switching supports N <= 8192");
  }
}

void ntt_forward(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  dispatch<false>(c, data, n_polys, b, s);
}

void ntt_inverse(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  dispatch<true>(c, data, n_polys, b, s);
}

// Builds the two-prime digit tables of the fused key-switching paths at every level.
void preload_ks_digits(const Context& c) {
  if (c.alpha > 2) return;
  for (int level = 1; level <= c.L; ++level) ks_digits(c, level, c.basis_QP(level));
}

}  // namespace bcn
