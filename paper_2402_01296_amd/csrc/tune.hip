// Autotuner: times the candidate transform shapes and MAC tile sizes on the
// device with hipEvents and keeps the fastest.
#include <algorithm>
#include <cstdio>
#include <string>

#include "layers.h"

namespace bcn {

namespace {
float time_ms(hipStream_t s, int reps, const std::function<void()>& f) {
  hipEvent_t a, b;
  BCN_HIP(hipEventCreate(&a));
  BCN_HIP(hipEventCreate(&b));
  f();  // warm-up
  BCN_HIP(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i) f();
  BCN_HIP(hipEventRecord(b, s));
  BCN_HIP(hipEventSynchronize(b));
  float ms = 0;
  BCN_HIP(hipEventElapsedTime(&ms, a, b));
  BCN_HIP(hipEventDestroy(a));
  BCN_HIP(hipEventDestroy(b));
  return ms / reps;
}

// Mean time of f with the caches cold, as in a step whose inputs were written long before:
// before every repetition a fill of `flush` (larger than the L2s and the last-level cache)
// evicts them.
float time_ms_cold(hipStream_t s, int reps, double* flush, size_t flush_doubles, const std::function<void()>& f) {
  hipEvent_t a, b;
  BCN_HIP(hipEventCreate(&a));
  BCN_HIP(hipEventCreate(&b));
  f();  // warm-up
  float total = 0;
  for (int i = 0; i < reps; ++i) {
    fill(flush, flush_doubles, (double)i, s);
    BCN_HIP(hipEventRecord(a, s));
    f();
    BCN_HIP(hipEventRecord(b, s));
    BCN_HIP(hipEventSynchronize(b));
    float ms = 0;
    BCN_HIP(hipEventElapsedTime(&ms, a, b));
    total += ms;
  }
  BCN_HIP(hipEventDestroy(a));
  BCN_HIP(hipEventDestroy(b));
  return total / reps;
}
}  // namespace

std::string autotune_ntt(Context& c, hipStream_t s) {
  // a batch shaped like the square's transforms: many polynomials over Q_L + aux
  const Basis b = c.basis_QB(c.L);
  const int polys = std::max(16, 2048 / b.n);
  double* buf = c.arena->take((size_t)polys * b.n * c.n);
  BCN_HIP(hipMemsetAsync(buf, 0, (size_t)polys * b.n * c.n * sizeof(double), s));
  std::string report;
  // a candidate replaces the current (default) choice only when it is clearly faster, so that
  // near-ties do not flip the shape from one process to the next
  constexpr float kMargin = 0.97f;
  if (!c.pinned_loge) {
    const int dflt = c.ntt_loge;
    int best = dflt;
    float best_ms = 1e30f, dflt_ms = 1e30f;
    for (int loge : c.ntt_loge_options()) {
      c.ntt_loge = loge;
      const float ms = time_ms(s, 5, [&] {
        ntt_forward(c, buf, polys, b, s);
        ntt_inverse(c, buf, polys, b, s);
      });
      char line[128];
      std::snprintf(line, sizeof line, "ntt logn=%d loge=%d: %.3f ms for %d limbs fwd+inv\n", c.logn, loge, ms,
                    polys * b.n);
      report += line;
      if (loge == dflt) dflt_ms = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = loge;
      }
    }
    c.ntt_loge = best_ms < kMargin * dflt_ms ? best : dflt;
  }
  report += "ntt chosen loge=" + std::to_string(c.ntt_loge) + "\n";
  if (!c.pinned_prefetch) {
    float t[2];
    for (int pf = 0; pf < 2; ++pf) {
      c.ntt_prefetch = pf != 0;
      t[pf] = time_ms(s, 5, [&] {
        ntt_forward(c, buf, polys, b, s);
        ntt_inverse(c, buf, polys, b, s);
      });
    }
    c.ntt_prefetch = t[1] < kMargin * t[0];
    char line[160];
    std::snprintf(line, sizeof line, "ntt twiddles per pass %.3f ms, prefetched across the exchange %.3f ms\n", t[0],
                  t[1]);
    report += line;
  }
  report += std::string("ntt chosen prefetch=") + (c.ntt_prefetch ? "1" : "0") + "\n";
  if (!c.pinned_xlane && c.ntt_loge == 4) {
    float t[2];
    for (int xl = 0; xl < 2; ++xl) {
      c.ntt_xlane = xl != 0;
      t[xl] = time_ms(s, 5, [&] {
        ntt_forward(c, buf, polys, b, s);
        ntt_inverse(c, buf, polys, b, s);
      });
    }
    c.ntt_xlane = t[1] < kMargin * t[0];
    char line[160];
    std::snprintf(line, sizeof line, "ntt row-transpose exchanges through LDS %.3f ms, cross-lane %.3f ms\n", t[0], t[1]);
    report += line;
  }
  report += std::string("ntt chosen xlane=") + (c.ntt_xlane ? "1" : "0") + "\n";
  {
    float t[2];
    for (int pers = 0; pers < 2; ++pers) {
      c.ntt_persist = pers != 0;
      t[pers] = time_ms(s, 5, [&] {
        ntt_forward(c, buf, polys, b, s);
        ntt_inverse(c, buf, polys, b, s);
      });
    }
    c.ntt_persist = t[1] < kMargin * t[0];
    char line[160];
    std::snprintf(line, sizeof line, "ntt per-limb %.3f ms, persistent prefetching %.3f ms\n", t[0], t[1]);
    report += line;
    report += std::string("ntt chosen persistent=") + (c.ntt_persist ? "1" : "0") + "\n";
  }
  // square's transform segment: fused kernel (each transform shape) vs forward + tensor + inverse
  // (at N = 16384 the fused kernel needs all of a CU's LDS and spills a little; measured anyway)
  if (c.logn <= 14) {
    const int n = std::max(8, polys / 2);
    double* in = buf;
    double* out = c.arena->take((size_t)n * 3 * b.n * c.n);
    double* tmp = c.arena->take((size_t)n * 2 * b.n * c.n);
    const float unfused = time_ms(s, 5, [&] {
      BCN_HIP(hipMemcpyAsync(tmp, in, (size_t)n * 2 * b.n * c.n * sizeof(double), hipMemcpyDeviceToDevice, s));
      ntt_forward(c, tmp, 2 * n, b, s);
      tensor_square(c, tmp, out, n, b, s);
      ntt_inverse(c, out, 3 * n, b, s);
    });
    const float copy = time_ms(s, 5, [&] {
      BCN_HIP(hipMemcpyAsync(tmp, in, (size_t)n * 2 * b.n * c.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    });
    const int dflt = c.square_loge;
    int best = dflt;
    float best_ms = 1e30f, dflt_ms = 1e30f;
    for (int loge : c.ntt_loge_options()) {
      if (c.pinned_square_loge && loge != dflt) continue;
      c.square_loge = loge;
      const float ms = time_ms(s, 5, [&] { square_transform_fused(c, in, out, n, b, s); });
      char line[160];
      std::snprintf(line, sizeof line, "square transforms (%d ciphertexts, %d limbs): fused loge=%d %.3f ms\n", n,
                    b.n, loge, ms);
      report += line;
      if (loge == dflt) dflt_ms = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = loge;
      }
    }
    c.square_loge = best_ms < kMargin * dflt_ms ? best : dflt;
    const float fused = c.square_loge == best ? best_ms : dflt_ms;
    char line[160];
    std::snprintf(line, sizeof line, "square transforms unfused %.3f ms\n", unfused - copy);
    report += line;
    c.fuse_square = fused < unfused - copy;
    report += "square chosen loge=" + std::to_string(c.square_loge) + "\n";
  } else {
    c.fuse_square = false;
  }
  report += std::string("square chosen fused=") + (c.fuse_square ? "1" : "0") + "\n";
  // key switching: four kernels (ModUp, forward transforms, inner product, inverse
  // transforms), one fused kernel, or two kernels (digits + forward transform, inner
  // product + inverse transforms), on a batch shaped like the first relinearisation
  if (!c.pinned_ks) {
    const int level = c.L;
    const Basis qp = c.basis_QP(level);
    const int dn = c.dnum(level);
    const int n = std::max(8, 8192 / (qp.n * (dn + 2)));
    double* src = c.arena->take((size_t)n * level * c.n);
    double* key = c.arena->take((size_t)dn * 2 * (c.L + c.K) * c.n);
    double* D = c.arena->take((size_t)n * dn * qp.n * c.n);
    double* U = c.arena->take((size_t)n * 2 * qp.n * c.n);
    BCN_HIP(hipMemsetAsync(src, 0, (size_t)n * level * c.n * sizeof(double), s));
    BCN_HIP(hipMemsetAsync(key, 0, (size_t)dn * 2 * (c.L + c.K) * c.n * sizeof(double), s));
    KeySel ks;
    ks.key1 = key;
    float t[3] = {1e30f, 1e30f, 1e30f};
    t[0] = time_ms(s, 5, [&] {
      decompose_modup(c, src, (size_t)level * c.n, D, n, level, s);
      ntt_forward(c, D, n * dn, qp, s);
      ks_inner(c, D, 1, ks, n, level, U, s);
      ntt_inverse(c, U, 2 * n, qp, s);
    });
    if (c.logn <= 13 && c.alpha <= 2)
      t[1] = time_ms(s, 5, [&] { ks_fused(c, src, (size_t)level * c.n, n, level, key, 1, U, s); });
    if (c.alpha <= 2) {
      // the two-kernel path's own transform shape (its kernels hold more registers than a
      // plain transform, so the best shape can differ)
      const int dflt_loge = c.ks_loge;
      float best_l = 1e30f, dflt_l = 1e30f;
      int best_loge = dflt_loge;
      for (int loge : c.ntt_loge_options()) {
        c.ks_loge = loge;
        const float ms = time_ms(s, 5, [&] { ks_split(c, src, (size_t)level * c.n, n, level, ks, n, 1, D, U, s); });
        if (loge == dflt_loge) dflt_l = ms;
        if (ms < best_l) best_l = ms, best_loge = loge;
      }
      c.ks_loge = best_l < kMargin * dflt_l ? best_loge : dflt_loge;
      t[2] = c.ks_loge == best_loge ? best_l : dflt_l;
    }
    char line[200];
    std::snprintf(line, sizeof line,
                  "key switch (%d polynomials, %d digits): four kernels %.3f ms, fused %.3f ms, two kernels %.3f ms\n", n,
                  dn, t[0], t[1] < 1e29f ? t[1] : -1.0f, t[2] < 1e29f ? t[2] : -1.0f);
    report += line;
    const int dflt = c.ks_mode;
    int best = dflt;
    for (int k = 0; k < 3; ++k)
      if (t[k] < t[best]) best = k;
    c.ks_mode = t[best] < kMargin * t[dflt] ? best : dflt;
    // hoisted rotations: each source's digits serve several Galois keys, and the
    // transform-domain permutation scatters the inner product's digit reads
    if (c.alpha <= 2) {
      const int ns = 8, nsrc = std::max(2, n / ns);
      double* U2 = c.arena->take((size_t)nsrc * ns * 2 * qp.n * c.n);
      KeySel kr;
      kr.key1 = key;
      kr.galois1 = 3;
      const float r0 = time_ms(s, 3, [&] {
        decompose_modup(c, src, (size_t)level * c.n, D, nsrc, level, s);
        ntt_forward(c, D, nsrc * dn, qp, s);
        ks_inner(c, D, ns, kr, nsrc * ns, level, U2, s);
        ntt_inverse(c, U2, 2 * nsrc * ns, qp, s);
      });
      const float r2 = time_ms(s, 3, [&] { ks_split(c, src, (size_t)level * c.n, nsrc, level, kr, nsrc * ns, ns, D, U2, s); });
      std::snprintf(line, sizeof line, "hoisted rotations (%d sources x %d keys): four kernels %.3f ms, two kernels %.3f ms\n",
                    nsrc, ns, r0, r2);
      report += line;
      const int d = c.ks_mode_rot;
      const float td = d == 2 ? r2 : r0, tb = std::min(r0, r2);
      c.ks_mode_rot = tb < kMargin * td ? (r2 < r0 ? 2 : 0) : d;
    }
  }
  report += "key switch chosen mode=" + std::to_string(c.ks_mode) + " rotations=" + std::to_string(c.ks_mode_rot) +
            " loge=" + std::to_string(c.ks_loge) + "\n";
  return report;
}

std::string autotune_layer_mac(Context& c, Layer& L, hipStream_t s) {
  if (L.mac_weights.empty()) return "";
  // a HW convolution's MAC runs over the taps kept over Q_level then P
  const bool ext = L.packing != BCN_PACK_BATCH && L.kind == BCN_CONV2D && !L.diag;
  const Basis qp = c.basis_QP(L.level);
  const Basis* basis = ext ? &qp : nullptr;
  // three-part (unrelinearised) inputs: the MAC runs over three parts
  const int parts = L.in_parts;
  const size_t ctw = (size_t)parts * (ext ? qp.n : L.level) * c.n;
  // a slot-batched square layer's MAC writes the square's Q+B input: timed with the extension,
  // either fused into the MAC or as the separate kernel
  const bool qb = L.packing == BCN_PACK_BATCH && L.square && parts == 2;
  const size_t ctq = (size_t)2 * (L.level + c.m) * c.n;
  const int n_in_mac = L.mac.n_in;
  double* in = c.arena->take((size_t)n_in_mac * ctw);
  double* out = c.arena->take((size_t)L.mac.n_out * (qb ? ctq : ctw));
  BCN_HIP(hipMemsetAsync(in, 0, (size_t)n_in_mac * ctw * sizeof(double), s));
  // the MAC streams inputs another kernel wrote long before, so candidates are timed cold
  constexpr size_t kFlush = (size_t)1 << 26;   // 512 MiB, twice the last-level cache
  double* flush = c.arena->take(kFlush);
  std::string report;
  float best_ms = 1e30f;
  int best_tile = L.mac.tile;
  bool best_ext = false;
  for (int tile : {1, 2, 4, 8, 16, 32, 64}) {
    if (tile / 2 >= L.mac.n_out && tile > 8) break;
    if (tile < 8 && L.mac.n_out > 64) continue;   // narrow tiles only pay off for narrow layers
    MacPlan p = make_mac_plan(c, L.mac_weights, L.mac.n_out, n_in_mac, L.mac_order, tile);
    for (int fused = 0; fused <= (qb ? 1 : 0); ++fused) {
      if (fused && !mac_qb_supported(p, L.level)) continue;
      float ms = 0;
      try {
        ms = time_ms_cold(s, 5, flush, kFlush, [&] {
          if (!qb) {
            mac(c, p, in, out, L.level, s, 1, 0, 0, nullptr, 0, 0, basis, parts);
          } else if (fused) {
            mac_qb(c, p, in, out, L.level, s, 1, 0, 0, nullptr, ctq, ctq / 2);
          } else {
            mac(c, p, in, out, L.level, s, 1, 0, 0, nullptr, ctq, ctq / 2);
            extend_qb(c, out, out, L.mac.n_out, L.level, s);
          }
        });
      } catch (...) {
        free_mac_plan(p);
        throw;
      }
      char line[160];
      std::snprintf(line, sizeof line, "mac %dx%d tile=%d%s: %.3f ms\n", L.mac.n_out, n_in_mac, tile,
                    qb ? (fused ? " extension fused" : " + extension") : "", ms);
      report += line;
      if (ms < best_ms) {
        best_ms = ms;
        best_tile = tile;
        best_ext = fused != 0;
      }
    }
    free_mac_plan(p);
  }
  L.mac_ext = best_ext;
  if (best_tile != L.mac.tile) {
    BCN_HIP(hipStreamSynchronize(s));
    free_mac_plan(L.mac);
    L.mac = make_mac_plan(c, L.mac_weights, L.mac.n_out, n_in_mac, L.mac_order, best_tile);
  }
  report += "mac chosen tile=" + std::to_string(best_tile) + (qb ? (best_ext ? " extension fused" : " + extension") : "") +
            "\n";
  return report;
}

}  // namespace bcn
