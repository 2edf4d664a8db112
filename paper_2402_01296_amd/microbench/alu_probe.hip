// Device facts and ALU throughput behind the residue-arithmetic choice:
// FP64 FMA rate, 64-bit integer multiply rates, FP64-exact modular products
// (the library's mul_lazy) vs 64-bit integer Shoup modular products, and the
// bandwidth of a plain copy kernel.
//
// Build and run:  hipcc --offload-arch=gfx950 -O3 -ffp-contract=off alu_probe.hip -o alu_probe && ./alu_probe
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "../csrc/modarith.h"

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
      return 1;                                                                      \
    }                                                                                \
  } while (0)

constexpr int ILP = 8;

__global__ void k_fma(double* out, int iters, double a, double b) {
  double x[ILP];
  for (int i = 0; i < ILP; ++i) x[i] = threadIdx.x + i;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < ILP; ++i) x[i] = fma(x[i], a, b);
  double s = 0;
  for (int i = 0; i < ILP; ++i) s += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_mul64(uint64_t* out, int iters, uint64_t a, uint64_t b) {
  uint64_t x[ILP];
  for (int i = 0; i < ILP; ++i) x[i] = threadIdx.x + i;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < ILP; ++i) x[i] = x[i] * a + b;
  uint64_t s = 0;
  for (int i = 0; i < ILP; ++i) s += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_mulhi64(uint64_t* out, int iters, uint64_t a, uint64_t b) {
  uint64_t x[ILP];
  for (int i = 0; i < ILP; ++i) x[i] = threadIdx.x + i;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < ILP; ++i) x[i] = __umul64hi(x[i], a) + b;
  uint64_t s = 0;
  for (int i = 0; i < ILP; ++i) s += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// x <- x * w mod q, FP64-exact lazy product (values stay in (-q, q))
__global__ void k_modmul_fp64(double* out, int iters, double w, double q) {
  const bcn::Mod m{q, 1.0 / q};
  double x[ILP];
  for (int i = 0; i < ILP; ++i) x[i] = threadIdx.x + i + 1;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < ILP; ++i) x[i] = bcn::mul_lazy(w, x[i], m);
  double s = 0;
  for (int i = 0; i < ILP; ++i) s += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// x <- x * w mod q with Shoup's precomputed w' = floor(w 2^64 / q), 64-bit integers
__global__ void k_modmul_shoup(uint64_t* out, int iters, uint64_t w, uint64_t wp, uint64_t q) {
  uint64_t x[ILP];
  for (int i = 0; i < ILP; ++i) x[i] = threadIdx.x + i + 1;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < ILP; ++i) {
      const uint64_t t = __umul64hi(x[i], wp);
      uint64_t r = x[i] * w - t * q;
      x[i] = r >= q ? r - q : r;
    }
  uint64_t s = 0;
  for (int i = 0; i < ILP; ++i) s += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_copy(const double4* __restrict__ in, double4* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

int main() {
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  int optin = 0;
  CK(hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, 0));
  std::printf("arch=%s CUs=%d clock_kHz=%d L2=%d LDS_per_block=%zu LDS_optin=%d HBM_GiB=%.1f\n", p.gcnArchName,
              p.multiProcessorCount, p.clockRate, p.l2CacheSize, p.sharedMemPerBlock, optin,
              p.totalGlobalMem / 1073741824.0);
  const int blocks = 256 * 8, threads = 256, iters = 4096;
  const double ops = (double)blocks * threads * iters * ILP;
  double* dout;
  uint64_t* uout;
  CK(hipMalloc(&dout, (size_t)blocks * threads * 8));
  CK(hipMalloc(&uout, (size_t)blocks * threads * 8));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  float ms = 0;
  const uint64_t q = 68719230977ull, w = 12345678901ull;
  const uint64_t wp = (uint64_t)(((unsigned __int128)w << 64) / q);
  for (int rep = 0; rep < 2; ++rep) {
#define TIME(label, launch)                                                         \
  CK(hipEventRecord(e0));                                                           \
  launch;                                                                           \
  CK(hipEventRecord(e1));                                                           \
  CK(hipEventSynchronize(e1));                                                      \
  CK(hipEventElapsedTime(&ms, e0, e1));                                             \
  if (rep == 1) std::printf("%-34s %8.3f ms  %7.2f T/s\n", label, ms, ops / ms / 1e9);
    TIME("fp64 fma", (k_fma<<<blocks, threads>>>(dout, iters, 1.0000001, 0.5)))
    TIME("u64 mul-lo + add", (k_mul64<<<blocks, threads>>>(uout, iters, 0x123456789ull, 7)))
    TIME("u64 mul-hi + add", (k_mulhi64<<<blocks, threads>>>(uout, iters, 0x123456789abcdull, 7)))
    TIME("modmul fp64-exact (36-bit q)", (k_modmul_fp64<<<blocks, threads>>>(dout, iters, (double)w, (double)q)))
    TIME("modmul u64 Shoup (36-bit q)", (k_modmul_shoup<<<blocks, threads>>>(uout, iters, w, wp, q)))
#undef TIME
  }
  const size_t nbytes = (size_t)2 << 30, n4 = nbytes / 32;
  double4 *a, *b;
  CK(hipMalloc(&a, nbytes));
  CK(hipMalloc(&b, nbytes));
  CK(hipMemset(a, 0, nbytes));
  for (int rep = 0; rep < 3; ++rep) {
    CK(hipEventRecord(e0));
    k_copy<<<256 * 16, 256>>>(a, b, n4);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    if (rep == 2) std::printf("copy 2 GiB                         %8.3f ms  %7.1f GB/s (read + write)\n", ms,
                              2.0 * nbytes / ms / 1e6);
  }
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(dout));
  CK(hipFree(uout));
  return 0;
}
