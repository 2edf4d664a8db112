// Square + relinearisation without any device allocation: its scratch lives in
// a fixed array of device memory that the library holds per GPU until the
// process ends.
#include <map>
#include <mutex>

#include "scheme.h"

namespace bcn {

namespace {
constexpr size_t kFixedScratchBytes = (size_t)64 << 20;   // 64 MiB per device
// In host code `scratch` names a host-side stand-in, not device memory: only the
// address from hipGetSymbolAddress (per device) may be handed to kernels or copies.
__device__ __align__(256) double scratch[kFixedScratchBytes / sizeof(double)];

std::mutex g_mu;
std::map<int, double*> g_scratch_ptr;   // device -> device address of `scratch`

// Binds the context's arena to the fixed array for one call and forbids allocation.
struct FixedScratch {
  Context& c;
  explicit FixedScratch(Context& cx) : c(cx) {
    c.arena->bind_external(c.fixed_scratch, c.fixed_scratch_doubles);
    c.no_alloc = true;
  }
  ~FixedScratch() {
    c.no_alloc = false;
    c.arena->unbind_external();
  }
};
}  // namespace

// Once per device, with that device current (context creation sets it): the
// device address of this device's copy of `scratch`.
void fixed_scratch_setup(Context& c) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch_ptr.find(c.device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    BCN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(-5, "no device address for the fixed scratch array");
    it = g_scratch_ptr.emplace(c.device, static_cast<double*>(p)).first;
  }
  c.fixed_scratch = it->second;
  c.fixed_scratch_doubles = kFixedScratchBytes / sizeof(double);
}

void square_relin_noalloc(Context& c, const EvalKeys& ek, const double* in, double* out, int n, int level, bool modsw,
                          hipStream_t s) {
  if (!c.fixed_scratch) throw Error(-6, "fixed scratch array not set up on this device");
  const size_t need = square_relin_scratch_doubles(c, n, level);
  if (need > c.fixed_scratch_doubles)
    throw Error(-1, "square_relin_noalloc: " + std::to_string(n) + " ciphertexts at level " + std::to_string(level) +
                        " need " + std::to_string(need * sizeof(double)) + " bytes of scratch; the fixed buffer holds " +
                        std::to_string(kFixedScratchBytes) + " (use fewer ciphertexts per call)");
  FixedScratch bind(c);
  square_relin(c, ek, in, out, n, level, modsw, s);
}

}  // namespace bcn
