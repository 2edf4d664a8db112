// CKKS, the paper's scheme (section "Experiments", appendix "CKKS Scheme"), on the
// same RNS rings, transforms, keys and key switching as the BFV path.  A ciphertext
// holds N/2 fixed-point slot values; slot i sits at the evaluation point
// zeta^(5^i mod 2N), zeta = exp(i pi / N).  Encoding takes the real polynomial m with
// m(zeta^(5^i)) = z_i and rounds scale * m to integers; the product of two
// ciphertexts is the exact tensor mod Q (no rounding), relinearised by key switching
// and then rescaled (the exact nearest division by the last prime).
//
// Encoder: with 5^i mod 2N = 4 j(i) + 1, m(zeta^(4j+1)) = sum_k p_k zeta^k omega^(jk) for
// p_k = m_k + i m_(k+N/2) and omega = zeta^4 a primitive (N/2)-th root of unity, so
// encoding is one complex inverse DFT of length N/2 (one workgroup per plaintext, the
// vector in LDS) followed by the twist zeta^-k.
#include <cmath>
#include <complex>
#include <cstring>

#include "convert.h"
#include "scheme.h"

namespace bcn {

namespace {
constexpr int kEncThreads = 512;

// tables (doubles): omega^-k for k < N/4 (complex), zeta^-k / (N/2) for k < N/2 (complex),
// then j(i) for i < N/2 (as doubles)
size_t om_off(const Context&) { return 0; }
size_t tw_off(const Context& c) { return (size_t)c.n / 2; }          // N/4 complex = N/2 doubles
size_t jm_off(const Context& c) { return tw_off(c) + (size_t)c.n; }  // N/2 complex = N doubles

__device__ __forceinline__ double to_residue(double v, const Mod m) {
  // v an integer-valued double with |v| < 2^53; exact remainder by an FMA
  const double f = floor(v * m.qinv);
  double r = fma(-f, m.q, v);
  if (r < 0.0) r += m.q;
  if (r >= m.q) r -= m.q;
  return r;
}

__global__ void __launch_bounds__(kEncThreads)
k_ckks_encode(const double* __restrict__ z, int logn, int level, double scale, const double* __restrict__ tab,
              const Mod* __restrict__ mods, Basis b, double* __restrict__ out) {
  extern __shared__ double lds[];                 // [N/2] complex
  const int N = 1 << logn, h = N >> 1, logh = logn - 1;
  const double* om = tab;                         // omega^-k, k < N/4
  const double* tw = tab + (size_t)h;             // zeta^-k / (N/2), k < N/2
  const double* jm = tab + (size_t)h + N;         // j(i)
  const double* zp = z + (size_t)blockIdx.x * h;
  for (int i = threadIdx.x; i < h; i += blockDim.x) {
    const int j = (int)jm[i];
    const int br = (int)(__brev((unsigned)j) >> (32 - logh));
    lds[2 * br] = zp[i];
    lds[2 * br + 1] = 0.0;
  }
  __syncthreads();
  // iterative radix-2 inverse DFT (bit-reversed input, natural output)
  for (int st = 1; st <= logh; ++st) {
    const int half = 1 << (st - 1);
    for (int bf = threadIdx.x; bf < (h >> 1); bf += blockDim.x) {
      const int p = bf & (half - 1);
      const int i0 = ((bf >> (st - 1)) << st) + p, i1 = i0 + half;
      const int wi = p << (logh - st);
      const double wr = om[2 * wi], wim = om[2 * wi + 1];
      const double ar = lds[2 * i1], ai = lds[2 * i1 + 1];
      const double tr = wr * ar - wim * ai, ti = wr * ai + wim * ar;
      const double ur = lds[2 * i0], ui = lds[2 * i0 + 1];
      lds[2 * i0] = ur + tr;
      lds[2 * i0 + 1] = ui + ti;
      lds[2 * i1] = ur - tr;
      lds[2 * i1 + 1] = ui - ti;
    }
    __syncthreads();
  }
  double* o = out + (size_t)blockIdx.x * level * N;
  for (int k = threadIdx.x; k < h; k += blockDim.x) {
    const double ar = lds[2 * k], ai = lds[2 * k + 1];
    const double wr = tw[2 * k], wim = tw[2 * k + 1];
    const double mr = ar * wr - ai * wim, mi = ar * wim + ai * wr;
    const double c0 = rint(scale * mr), c1 = rint(scale * mi);
    for (int l = 0; l < level; ++l) {
      const Mod m = mods[b.id[l]];
      o[(size_t)l * N + k] = to_residue(c0, m);
      o[(size_t)l * N + k + h] = to_residue(c1, m);
    }
  }
}

__global__ void k_add_c0(double* __restrict__ ct, int n, int level, int logn, const double* __restrict__ pt, Basis b,
                         const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n * level * N) return;
  const size_t ci = idx / (level * N), lk = idx % (level * N);
  const Mod m = mods[b.id[lk >> logn]];
  double* p = ct + ci * 2 * level * N + lk;
  *p = add_mod(*p, pt[idx], m);
}

// centred value of [x]_{Q_level} as a double (exact when below 2^53 in magnitude)
template <int NS>
__global__ void k_crt_double(const double* __restrict__ x, double* __restrict__ out, int n, int logn,
                             const Conv* __restrict__ cvp, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << logn;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n * N) return;
  const Conv& cv = *cvp;
  const size_t ci = idx >> logn, k = idx & (N - 1);
  double r[NS], v[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) r[i] = x[(ci * NS + i) * N + k];
  garner<NS>(r, v, cv, mods);
  const bool neg = above_half<NS>(v, NS, cv, mods);
  // Q - x has the mixed-radix digits q_k - 1 - v_k, plus one
  double acc = 0.0;
#pragma unroll
  for (int kk = NS - 1; kk >= 0; --kk) {
    const double q = mods[cv.src[kk]].q;
    acc = acc * q + (neg ? q - 1.0 - v[kk] : v[kk]);
  }
  out[idx] = neg ? -(acc + 1.0) : acc;
}

unsigned nb256(size_t work) { return (unsigned)((work + 255) / 256); }

// host DFT helper for decoding: in place, length n (a power of two), sign -1 or +1
void fft_host(std::vector<std::complex<double>>& a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const long double ang = sign * 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)len;
        const std::complex<double> w((double)std::cos(ang), (double)std::sin(ang));
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}
}  // namespace

void ckks_setup(Context& c) {
  const size_t N = c.n, h = N / 2;
  std::vector<double> t(jm_off(c) + h);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (size_t k = 0; k < h / 2; ++k) {               // omega^-k, omega = exp(2 pi i / (N/2))
    const long double a = -2.0L * pi * (long double)k / (long double)h;
    t[om_off(c) + 2 * k] = (double)std::cos(a);
    t[om_off(c) + 2 * k + 1] = (double)std::sin(a);
  }
  for (size_t k = 0; k < h; ++k) {                   // zeta^-k / (N/2), zeta = exp(i pi / N)
    const long double a = -pi * (long double)k / (long double)N;
    t[tw_off(c) + 2 * k] = (double)(std::cos(a) / (long double)h);
    t[tw_off(c) + 2 * k + 1] = (double)(std::sin(a) / (long double)h);
  }
  uint64_t e = 1;
  for (size_t i = 0; i < h; ++i) {                   // 5^i mod 2N = 4 j(i) + 1
    t[jm_off(c) + i] = (double)((e - 1) / 4);
    e = e * 5 % (2 * N);
  }
  BCN_HIP(hipMalloc(&c.ckks_tab, t.size() * sizeof(double)));
  BCN_HIP(hipMemcpy(c.ckks_tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
}

void ckks_encode(const Context& c, const double* z, int n, int level, double scale, bool ntt_domain, double* out,
                 hipStream_t s) {
  if (n == 0) return;
  if (!(scale > 0.0) || scale >= 4503599627370496.0) throw Error(-1, "CKKS scale must be in (0, 2^52)");
  const size_t lds = (size_t)c.n * sizeof(double);   // N/2 complex
  const Basis b = c.basis_Q(level);
  ProfScope ps(c, "ckks_encode", s, 8.0 * n * ((double)c.n / 2 + (double)level * c.n));
  hipLaunchKernelGGL(k_ckks_encode, dim3(n), dim3(kEncThreads), lds, s, z, c.logn, level, scale, c.ckks_tab,
                     c.tab.mods, b, out);
  BCN_HIP(hipGetLastError());
  if (ntt_domain) ntt_forward(c, out, n, b, s);
}

void ckks_add_plain(const Context& c, double* ct, int n, int level, const double* pt, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_add_c0, dim3(nb256((size_t)n * level * c.n)), dim3(256), 0, s, ct, n, level, c.logn, pt,
                     c.basis_Q(level), c.tab.mods);
  BCN_HIP(hipGetLastError());
}

void ckks_encrypt(Context& c, const SecretKey& sk, const double* z_host, double scale, const uint64_t* a_host,
                  const int8_t* e_host, int n, int level, double* ct, hipStream_t s) {
  if (level < 1 || level > c.L) throw Error(-2, "bad level");
  Arena& ar = *c.arena;
  const size_t N = c.n, pw = (size_t)level * N;
  const Basis q = c.basis_Q(level);
  double* zd = ar.take((size_t)n * N / 2);
  BCN_HIP(hipMemcpyAsync(zd, z_host, (size_t)n * N / 2 * sizeof(double), hipMemcpyHostToDevice, s));
  double* M = ar.take((size_t)n * pw);
  ckks_encode(c, zd, n, level, scale, false, M, s);
  uint64_t* au = reinterpret_cast<uint64_t*>(ar.take((size_t)n * pw));
  BCN_HIP(hipMemcpyAsync(au, a_host, (size_t)n * pw * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  double* A = ar.take((size_t)n * pw);
  u64_to_f64(au, A, (size_t)n * pw, s);
  double* AS = ar.take((size_t)n * pw);
  BCN_HIP(hipMemcpyAsync(AS, A, (size_t)n * pw * sizeof(double), hipMemcpyDeviceToDevice, s));
  ntt_forward(c, AS, n, q, s);
  pointwise_mul(c, AS, sk.s_hat, AS, n, q, true, s);
  ntt_inverse(c, AS, n, q, s);
  int8_t* ed = reinterpret_cast<int8_t*>(ar.take(((size_t)n * N + 7) / 8));
  BCN_HIP(hipMemcpyAsync(ed, e_host, (size_t)n * N, hipMemcpyHostToDevice, s));
  double* E = ar.take((size_t)n * pw);
  small_to_rns(c, ed, E, n, q, s);
  for (int i = 0; i < n; ++i)
    combine_keypart(c, AS + i * pw, E + i * pw, nullptr, ct + (size_t)i * 2 * pw, q, 0, 0, nullptr, s);
  BCN_HIP(hipMemcpy2DAsync(ct + pw, 2 * pw * sizeof(double), A, pw * sizeof(double), pw * sizeof(double), n,
                           hipMemcpyDeviceToDevice, s));
  ckks_add_plain(c, ct, n, level, M, s);
  BCN_HIP(hipStreamSynchronize(s));
}

void ckks_decrypt(Context& c, const SecretKey& sk, const double* ct, int n, int level, double scale, double* z_host,
                  hipStream_t s) {
  if (level < 1 || level > c.L) throw Error(-2, "bad level");
  Arena& ar = *c.arena;
  const size_t N = c.n, pw = (size_t)level * N, h = N / 2;
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
  double* V = ar.take((size_t)n * N);
  std::vector<int> src;
  for (int i = 0; i < level; ++i) src.push_back(c.idQ(i));
  const Conv* cv = conv_device(c, "dec" + std::to_string(level), make_conv(c, src, {}));
  switch (level) {
#define BCN_CRT(NS) \
  case NS: hipLaunchKernelGGL(k_crt_double<NS>, dim3(nb256((size_t)n * N)), dim3(256), 0, s, X, V, n, c.logn, cv, c.tab.mods); break;
    BCN_CRT(1) BCN_CRT(2) BCN_CRT(3) BCN_CRT(4) BCN_CRT(5) BCN_CRT(6) BCN_CRT(7) BCN_CRT(8)
#undef BCN_CRT
    default: throw Error(-1, "unsupported level");
  }
  BCN_HIP(hipGetLastError());
  std::vector<double> m((size_t)n * N);
  BCN_HIP(hipMemcpyAsync(m.data(), V, m.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  BCN_HIP(hipStreamSynchronize(s));
  // decode: p_k = (m_k + i m_(k+N/2)) zeta^k, forward DFT of length N/2, slot i at j(i)
  const long double pi = 3.14159265358979323846264338327950288L;
  std::vector<std::complex<double>> p(h);
  for (int ci = 0; ci < n; ++ci) {
    const double* mc = m.data() + (size_t)ci * N;
    for (size_t k = 0; k < h; ++k) {
      const long double a = pi * (long double)k / (long double)N;
      p[k] = std::complex<double>(mc[k], mc[k + h]) * std::complex<double>((double)std::cos(a), (double)std::sin(a));
    }
    fft_host(p, +1);
    uint64_t e = 1;
    for (size_t i = 0; i < h; ++i) {
      z_host[(size_t)ci * h + i] = p[(e - 1) / 4].real() / scale;
      e = e * 5 % (2 * N);
    }
  }
}

void ckks_square_relin_rescale(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level,
                               hipStream_t s) {
  if (!ek.relin) throw Error(-3, "missing relinearisation key");
  if (level < 2) throw Error(-2, "rescaling needs two primes");
  if (n == 0) return;
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const Basis qb = c.basis_Q(level), qp = c.basis_QP(level);
  const int nbp = qp.n, dn = c.dnum(level);
  // the tensor (c0^2, 2 c0 c1, c1^2) mod each q_i, exact
  double* Y = ar.take((size_t)n * 3 * level * N);
  if (c.fuse_square) {
    square_transform_fused(c, in, Y, n, qb, s);
  } else {
    double* X = ar.take((size_t)n * 2 * level * N);
    copy_rows(in, 0, X, 0, (size_t)n * 2 * level * N, 1, s);
    ntt_forward(c, X, 2 * n, qb, s);
    tensor_square(c, X, Y, n, qb, s);
    ntt_inverse(c, Y, 3 * n, qb, s);
  }
  const double* d2 = Y + (size_t)2 * level * N;
  const size_t stride = (size_t)3 * level * N;
  double* U = ar.take((size_t)n * 2 * nbp * N);
  KeySel ks;
  ks.key1 = ek.relin;
  if (c.ks_mode == 1) {
    ks_fused(c, d2, stride, n, level, ek.relin, 1, U, s);
  } else if (c.ks_mode == 2) {
    double* D = ar.take((size_t)n * dn * nbp * N);
    ks_split(c, d2, stride, n, level, ks, n, 1, D, U, s);
  } else {
    double* D = ar.take((size_t)n * dn * nbp * N);
    decompose_modup(c, d2, stride, D, n, level, s);
    ntt_forward(c, D, n * dn, qp, s);
    ks_inner(c, D, 1, ks, n, level, U, s);
    ntt_inverse(c, U, 2 * n, qp, s);
  }
  // (d0, d1) + round(u / P), then divided by q_level with nearest rounding (the rescale)
  moddown(c, U, n, level, Y, 1, stride, 1, ks, true, out, s);
}

}  // namespace bcn
