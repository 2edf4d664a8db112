// Negacyclic NTT / inverse NTT over every limb of a batch of RNS polynomials.
//
// Forward:  out[pos] = a(psi^(2j+1)) mod q with j = bitrev(pos)  (Cooley-Tukey,
//           natural input, the psi twist merged into the twiddles).
// Inverse:  the exact inverse: bit-reversed input, natural output
//           (decimation in time with omega^-1, then one multiply by N^-1 psi^-k).
//
// One workgroup transforms one limb.  Each thread keeps E = 2^LOGE residues in
// registers and applies LOGE butterfly stages per pass; passes exchange data
// through LDS (the whole limb, padded, is LDS-resident).  The first pass reads
// HBM and the last pass writes HBM, so a limb costs one read and one write of
// N words.  Values grow additively inside the transform (|x| < (LOGN+1) q <
// 2^45), which the lazy FP64 product tolerates; one reduction at the end
// brings them back to [0, q).
#include "internal.h"

namespace bcn {
namespace {

__device__ __forceinline__ int lds_pad(int g) { return g + (g >> 5); }

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

template <int LOGN, int LOGE, bool INV, int P>
__device__ __forceinline__ void run_pass(double (&x)[1 << LOGE], double* lds, double* __restrict__ a,
                                         const double* __restrict__ tw, const double* __restrict__ post,
                                         const Mod m, const int tid) {
  using S = Shape<LOGN, LOGE>;
  constexpr int N = S::N, T = S::T;
  constexpr int C = Sched<LOGN, LOGE, INV>::c(P);
  constexpr int S0 = Sched<LOGN, LOGE, INV>::s0(P);
  constexpr int SZ = 1 << C;
  constexpr int G = S::E >> C;
  constexpr int SMIN = INV ? (1 << S0) : (N >> (S0 + C));

  int base[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int sid = g * T + tid;
    const int b = sid / SMIN, r = sid % SMIN;
    base[g] = INV ? b * (SMIN << C) + r : b * (N >> S0) + r;
  }

  // gather
  if constexpr (P == 0) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < SZ; ++j) x[g * SZ + j] = a[base[g] + j * SMIN];
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < SZ; ++j) x[g * SZ + j] = lds[lds_pad(base[g] + j * SMIN)];
  }

  // butterflies
#pragma unroll
  for (int l = 0; l < C; ++l) {
    const int s = S0 + l;
    const int sh = INV ? l : (C - 1 - l);
    const int half = 1 << sh;
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int jj = 0; jj < SZ / 2; ++jj) {
        const int j = ((jj >> sh) << (sh + 1)) | (jj & (half - 1));
        const int gi = base[g] + j * SMIN;
        double w;
        if (INV)
          w = tw[(gi & ((1 << s) - 1)) * (N >> (s + 1))];
        else
          w = tw[(1 << s) + (gi >> (LOGN - s))];
        const double u = x[g * SZ + j];
        const double v = mul_lazy(w, x[g * SZ + j + half], m);
        x[g * SZ + j] = u + v;
        x[g * SZ + j + half] = u - v;
      }
    }
  }

  if constexpr (P == S::NP - 1) {
    // scatter to HBM in canonical form
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < SZ; ++j) {
        const int gi = base[g] + j * SMIN;
        double v = x[g * SZ + j];
        v = INV ? norm(mul_lazy(post[gi], v, m), m) : reduce(v, m);
        a[gi] = v;
      }
  } else {
    if constexpr (P > 0) __syncthreads();   // everyone has finished reading this pass's LDS data
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < SZ; ++j) lds[lds_pad(base[g] + j * SMIN)] = x[g * SZ + j];
    __syncthreads();
    run_pass<LOGN, LOGE, INV, P + 1>(x, lds, a, tw, post, m, tid);
  }
}

template <int LOGN, int LOGE, bool INV>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_ntt(double* __restrict__ data, Basis basis, Tables tb) {
  constexpr int N = 1 << LOGN;
  extern __shared__ double lds[];
  const int limb = blockIdx.x % basis.n;
  const int pid = basis.id[limb];
  const Mod m = tb.mods[pid];
  double* a = data + (size_t)blockIdx.x * N;
  const double* tw = INV ? tb.inv + (size_t)pid * (N / 2) : tb.fwd + (size_t)pid * N;
  const double* post = tb.post + (size_t)pid * N;
  double x[1 << LOGE];
  run_pass<LOGN, LOGE, INV, 0>(x, lds, a, tw, post, m, threadIdx.x);
}

template <int LOGN, int LOGE, bool INV>
void launch(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const size_t lds = (size_t)(N + N / 32) * sizeof(double);
  const unsigned blocks = (unsigned)n_polys * b.n;
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_ntt<LOGN, LOGE, INV>), dim3(blocks), dim3(N >> LOGE), lds, s, data, b, c.tab);
  BCN_HIP(hipGetLastError());
}

template <int LOGN, int LOGE>
void set_attr() {
  const int lds = (int)((1 << LOGN) + (1 << LOGN) / 32) * (int)sizeof(double);
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  BCN_HIP(hipFuncSetAttribute((const void*)k_ntt<LOGN, LOGE, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
}

template <bool INV>
void dispatch(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  switch (c.logn) {
    case 10: launch<10, 3, INV>(c, data, n_polys, b, s); break;
    case 11: launch<11, 3, INV>(c, data, n_polys, b, s); break;
    case 12: launch<12, 4, INV>(c, data, n_polys, b, s); break;
    case 13: launch<13, 4, INV>(c, data, n_polys, b, s); break;
    case 14: launch<14, 5, INV>(c, data, n_polys, b, s); break;
    default: throw Error(-1, "unsupported ring degree");
  }
}

}  // namespace

void ntt_setup(const Context& c) {
  switch (c.logn) {
    case 10: set_attr<10, 3>(); break;
    case 11: set_attr<11, 3>(); break;
    case 12: set_attr<12, 4>(); break;
    case 13: set_attr<13, 4>(); break;
    case 14: set_attr<14, 5>(); break;
    default: throw Error(-1, "unsupported ring degree");
  }
}

void ntt_forward(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  dispatch<false>(c, data, n_polys, b, s);
}

void ntt_inverse(const Context& c, double* data, int n_polys, const Basis& b, hipStream_t s) {
  dispatch<true>(c, data, n_polys, b, s);
}

}  // namespace bcn
