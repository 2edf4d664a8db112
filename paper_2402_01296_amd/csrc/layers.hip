// Layer lowering: HW- and batch-packed convolution / dense layers with the
// mask, feature injection, square + relinearisation, modulus switch and
// global sum epilogues (appendix "Implementation Details"; features enter as
// in section "The unidirectional connections").
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "../../include/bcn.h"
#include "layers.h"

namespace bcn {

Layer::~Layer() {
  free_mac_plan(mac);
  if (mask_hat_qp) (void)hipFree(mask_hat_qp);
  if (ptv_hat) (void)hipFree(ptv_hat);
  if (slot_of) (void)hipFree(slot_of);
}

namespace {
// BCN_MAC_TILE pins a slot-batched layer's MAC tile (a power of two in 1..64) until an autotune;
// BCN_MAC_EXT=0 keeps the extension to Q+B out of the MAC
int env_mac_tile(int dflt) {
  const char* e = std::getenv("BCN_MAC_TILE");
  if (!e) return dflt;
  const int t = std::atoi(e);
  if (t < 1 || t > 64 || (t & (t - 1))) throw Error(-1, "BCN_MAC_TILE must be a power of two in 1..64");
  return t;
}

int next_pow2(int x) {
  int s = 1;
  while (s < x) s *= 2;
  return s;
}
}  // namespace

Layer* layer_create(Context& c, const bcn_layer_desc& d, int level) {
  if (level < 1 || level > c.L) throw Error(-2, "bad level");
  if (d.kind == BCN_POOL) {
    // local sum pooling = a valid HW convolution whose weights are 1 on the channel itself
    if (d.packing != BCN_PACK_HW) throw Error(-1, "pooling needs HW packing");
    if (d.in_c < 1 || d.k < 1) throw Error(-1, "bad pooling shape");
    std::vector<int32_t> w((size_t)d.in_c * d.in_c * d.k * d.k, 0);
    for (int ch = 0; ch < d.in_c; ++ch)
      for (int t = 0; t < d.k * d.k; ++t) w[((size_t)ch * d.in_c + ch) * d.k * d.k + t] = 1;
    bcn_layer_desc dc = d;
    dc.kind = BCN_CONV2D;
    dc.out_c = d.in_c;
    dc.pad = 0;
    dc.weights = w.data();
    dc.has_features = 0;
    dc.square = 0;
    dc.modswitch = 0;
    dc.sum = 0;
    return layer_create(c, dc, level);
  }
  if (!d.weights) throw Error(-1, "layer weights missing");
  if (d.in_c < 1 || d.in_h < 1 || d.in_w < 1 || d.out_c < 1) throw Error(-1, "bad layer shape");
  auto L = std::make_unique<Layer>();
  L->kind = d.kind;
  L->packing = d.packing;
  if (d.in_parts != 0 && d.in_parts != 2 && d.in_parts != 3) throw Error(-1, "in_parts must be 2 or 3");
  L->in_parts = d.in_parts == 3 ? 3 : 2;
  L->defer = d.defer_relin != 0;
  if (L->in_parts == 3 && (d.packing != BCN_PACK_BATCH || d.kind != BCN_DENSE))
    throw Error(-1, "three-part inputs need a slot-batched (scalar) dense layer");
  if (L->defer && !d.square) throw Error(-1, "defer_relin needs a square");
  if (L->defer && d.packing != BCN_PACK_BATCH && (d.kind != BCN_CONV2D || d.sum))
    throw Error(-1, "a HW layer defers relinearisation only as a convolution without a global sum");
  if (const char* e = std::getenv("BCN_MAC_EXT")) L->mac_ext = std::atoi(e) != 0;
  L->level = level;
  L->square = d.square != 0;
  L->modsw = d.square && d.modswitch && level >= 2;
  L->level_out = L->modsw ? level - 1 : level;
  L->features = d.has_features != 0;
  L->fscale = d.feature_scale;
  L->fclamp = d.feature_clamp;
  const int N = c.n;
  if (d.kind == BCN_CONV2D) {
    if (d.k < 1 || d.stride < 1 || d.pad < 0) throw Error(-1, "bad convolution geometry");
    L->oh = (d.in_h + 2 * d.pad - d.k) / d.stride + 1;
    L->ow = (d.in_w + 2 * d.pad - d.k) / d.stride + 1;
    if (L->oh < 1 || L->ow < 1) throw Error(-1, "convolution output is empty");
  }
  if (d.packing == BCN_PACK_BATCH) {
    if (d.batch < 1 || d.batch > N) throw Error(-1, "batch must be 1..N");
    L->batch = d.batch;
    if (d.kind == BCN_CONV2D) {
      L->n_in = d.in_c * d.in_h * d.in_w;
      L->n_out = d.out_c * L->oh * L->ow;
      std::vector<int32_t> W((size_t)L->n_out * L->n_in, 0);
      for (int o = 0; o < d.out_c; ++o)
        for (int i = 0; i < L->oh; ++i)
          for (int j = 0; j < L->ow; ++j) {
            const int row = (o * L->oh + i) * L->ow + j;
            for (int ci = 0; ci < d.in_c; ++ci)
              for (int di = 0; di < d.k; ++di)
                for (int dj = 0; dj < d.k; ++dj) {
                  const int y = d.stride * i + di - d.pad, x = d.stride * j + dj - d.pad;
                  if (y < 0 || y >= d.in_h || x < 0 || x >= d.in_w) continue;
                  W[(size_t)row * L->n_in + (ci * d.in_h + y) * d.in_w + x] =
                      d.weights[((o * d.in_c + ci) * d.k + di) * d.k + dj];
                }
          }
      // tiles group all channels of neighbouring output positions, which share input pixels
      std::vector<int> order;
      for (int i = 0; i < L->oh; ++i)
        for (int j = 0; j < L->ow; ++j)
          for (int o = 0; o < d.out_c; ++o) order.push_back((o * L->oh + i) * L->ow + j);
      L->mac = make_mac_plan(c, W, L->n_out, L->n_in, order, env_mac_tile(16));
      L->mac_weights = W;
      L->mac_order = order;
    } else {
      L->n_in = d.in_c * d.in_h * d.in_w;
      L->n_out = d.out_c;
      std::vector<int32_t> W(d.weights, d.weights + (size_t)L->n_out * L->n_in);
      L->mac = make_mac_plan(c, W, L->n_out, L->n_in, {}, env_mac_tile(0));
      L->mac_weights = W;
    }
    L->stride_b = L->n_out;
    if (d.sum) {
      // a global sum moved after a scalar dense layer (sum and dense are linear): rotate-and-sum
      // of each output over d.sum slots
      if (d.kind != BCN_DENSE || d.has_features || d.square)
        throw Error(-1, "a batch-packed layer's sum must follow a plain dense layer");
      if (d.sum < 2 || (d.sum & (d.sum - 1)) || d.sum > N / 2)
        throw Error(-1, "sum span must be a power of two in 2..N/2");
      L->span = d.sum;
      for (const auto& rs : rotate_sum_rounds(L->span)) L->all_steps.insert(L->all_steps.end(), rs.begin(), rs.end());
      std::sort(L->all_steps.begin(), L->all_steps.end());
    }
    return L.release();
  }
  if (d.packing != BCN_PACK_HW) throw Error(-1, "unknown packing");
  if (d.row < 1 || d.pos_stride < 1) throw Error(-1, "HW packing needs row and pos_stride");
  const int half = N / 2;
  L->n_in = d.in_c;
  L->n_out = d.out_c;
  auto slot = [&](int ps, int y, int x) { return ps * (d.row * y + x); };
  // BHW packing: image b's block starts at bases[b]; HW packing: one image at slot 0
  std::vector<int> bases(1, 0);
  int extent = half;              // slots one image may use
  if (d.block > 0) {
    if (d.block > half || half % d.block) throw Error(-1, "BHW block must divide N/2");
    const int per_row = half / d.block;
    if (d.batch < 1 || d.batch > 2 * per_row) throw Error(-1, "BHW: 1..N/block images per ciphertext");
    bases.clear();
    for (int b = 0; b < d.batch; ++b) bases.push_back((b % per_row) * d.block + (b / per_row) * half);
    extent = d.block;
  }
  if (slot(d.pos_stride, d.in_h - 1, d.in_w - 1) >= extent) throw Error(-1, "input positions beyond the image block");
  if (d.kind == BCN_CONV2D) {
    if (d.pad != 0) throw Error(-1, "HW convolution is valid (pad 0)");
    const int k2 = d.k * d.k;
    // taps: index 0 = offset 0 (the input itself), then the nonzero offsets in (di, dj) order
    std::vector<int> tap_of(k2);
    for (int di = 0; di < d.k; ++di)
      for (int dj = 0; dj < d.k; ++dj) {
        const int off = slot(d.pos_stride, di, dj);
        if (off >= extent) throw Error(-1, "rotation offset beyond the image block");
        if (off == 0) {
          tap_of[di * d.k + dj] = 0;
        } else {
          L->steps.push_back(off);
          tap_of[di * d.k + dj] = (int)L->steps.size();
        }
      }
    if ((int)L->steps.size() != k2 - 1) throw Error(-1, "duplicate convolution offsets");
    L->k2 = k2;
    std::vector<int32_t> W((size_t)d.out_c * d.in_c * k2, 0);
    for (int o = 0; o < d.out_c; ++o)
      for (int ci = 0; ci < d.in_c; ++ci)
        for (int t = 0; t < k2; ++t)
          W[(size_t)o * d.in_c * k2 + ci * k2 + tap_of[t]] = d.weights[(o * d.in_c + ci) * k2 + t];
    L->mac = make_mac_plan(c, W, d.out_c, d.in_c * k2);
    L->mac_weights = W;
    // valid output slots and their mask
    const int ops = d.pos_stride * d.stride;
    std::vector<int> so;
    for (int i = 0; i < L->oh; ++i)
      for (int j = 0; j < L->ow; ++j) so.push_back(slot(ops, i, j));
    const int maxs = *std::max_element(so.begin(), so.end());
    if (maxs >= extent) throw Error(-1, "output positions beyond the image block");
    std::vector<int64_t> mask(N, 0);
    for (int b : bases)
      for (int v : so) mask[b + v] = 1;
    BCN_HIP(hipMalloc(&L->mask_hat_qp, (size_t)(level + c.K) * N * sizeof(double)));
    c.arena->reset();
    encode_plain_ntt(c, mask.data(), 1, level, L->mask_hat_qp, nullptr, true);
    // feature slots of one output map: images in order, positions in (i, j) order
    std::vector<int> fo;
    for (int b : bases)
      for (int v : so) fo.push_back(b + v);
    L->per = (int)fo.size();
    BCN_HIP(hipMalloc(&L->slot_of, fo.size() * sizeof(int)));
    BCN_HIP(hipMemcpy(L->slot_of, fo.data(), fo.size() * sizeof(int), hipMemcpyHostToDevice));
    if (d.sum) {
      L->span = next_pow2(maxs + 1);
      if (L->span > extent) throw Error(-1, "sum span beyond the image block");
      for (const auto& rs : rotate_sum_rounds(L->span)) L->all_steps.insert(L->all_steps.end(), rs.begin(), rs.end());
    }
  } else if (d.method == BCN_DENSE_DIAGONAL) {
    // diagonal method: n1 + n2 - 1 rotations of each input channel (steps 1 - n2 .. n1 - 1), each
    // multiplied by one weight vector; outputs at slots 0..n2-1 of one ciphertext
    if (d.block > 0) throw Error(-1, "the diagonal method packs one image");
    if (d.pos_stride != 1 || (d.in_h > 1 && d.in_w != d.row)) throw Error(-1, "diagonal method needs contiguous inputs");
    const int n1 = d.in_h * d.in_w, n2 = d.out_c;
    if (n1 + n2 > half) throw Error(-1, "diagonal method: n1 + n2 must not exceed N/2");
    std::vector<int> rs;
    for (int i = 1; i < n1 + n2; ++i) rs.push_back(i - n2);
    const int k2 = (int)rs.size();
    std::vector<int> tap_r(k2);        // tap 0 = offset 0, then the nonzero steps in order
    tap_r[0] = 0;
    for (int r : rs)
      if (r != 0) {
        L->steps.push_back(r);
        tap_r[L->steps.size()] = r;
      }
    L->k2 = k2;
    L->diag = true;
    L->n_out = 1;
    std::vector<int64_t> vec((size_t)d.in_c * k2 * N, 0);
    for (int ci = 0; ci < d.in_c; ++ci)
      for (int t = 0; t < k2; ++t) {
        const int r = tap_r[t];
        for (int j = 0; j < n2; ++j)
          if (j + r >= 0 && j + r < n1)
            vec[((size_t)ci * k2 + t) * N + j] = d.weights[(size_t)j * d.in_c * n1 + ci * n1 + j + r];
      }
    BCN_HIP(hipMalloc(&L->ptv_hat, (size_t)d.in_c * k2 * level * N * sizeof(double)));
    c.arena->reset();
    encode_plain_ntt(c, vec.data(), d.in_c * k2, level, L->ptv_hat, nullptr);
    if (d.has_features) throw Error(-1, "features are supported on convolutions");
  } else {
    // dense over spatially laid out channels: weight vectors, then rotate-and-sum
    const int per = d.in_h * d.in_w;
    std::vector<int> si;
    for (int y = 0; y < d.in_h; ++y)
      for (int x = 0; x < d.in_w; ++x) si.push_back(slot(d.pos_stride, y, x));
    const int maxs = *std::max_element(si.begin(), si.end());
    if (maxs >= extent) throw Error(-1, "input positions beyond the image block");
    std::vector<int64_t> vec((size_t)d.out_c * d.in_c * N, 0);
    for (int o = 0; o < d.out_c; ++o)
      for (int ci = 0; ci < d.in_c; ++ci)
        for (int p = 0; p < per; ++p)
          for (int b : bases)
            vec[((size_t)o * d.in_c + ci) * N + b + si[p]] = d.weights[(size_t)o * d.in_c * per + ci * per + p];
    BCN_HIP(hipMalloc(&L->ptv_hat, (size_t)d.out_c * d.in_c * level * N * sizeof(double)));
    c.arena->reset();
    encode_plain_ntt(c, vec.data(), d.out_c * d.in_c, level, L->ptv_hat, nullptr);
    L->span = next_pow2(maxs + 1);
    if (L->span < 2) L->span = 2;
    if (L->span > extent) throw Error(-1, "sum span beyond the image block");
    for (const auto& rs : rotate_sum_rounds(L->span)) L->all_steps.insert(L->all_steps.end(), rs.begin(), rs.end());
    if (d.has_features) throw Error(-1, "features are supported on convolutions");
  }
  for (int st : L->steps) L->all_steps.push_back(st);
  std::sort(L->all_steps.begin(), L->all_steps.end());
  L->all_steps.erase(std::unique(L->all_steps.begin(), L->all_steps.end()), L->all_steps.end());
  return L.release();
}

namespace {

// fn(first, count, stream) over ciphertexts [0, n): in two halves, the second on the context's
// side stream (forked after the work already queued on s, joined back into s), when n is large
// enough for two launches of each kernel to fill the device.
template <class F>
void run_halves(Context& c, int n, hipStream_t s, F&& fn) {
  constexpr int kMinSplit = 32;
  if (!c.split_chain || c.prof || n < kMinSplit) {
    fn(0, n, s);
    return;
  }
  const int h = n / 2;
  BCN_HIP(hipEventRecord(c.fork_ev, s));
  BCN_HIP(hipStreamWaitEvent(c.side, c.fork_ev, 0));
  fn(0, h, s);
  fn(h, n - h, c.side);
  BCN_HIP(hipEventRecord(c.join_ev, c.side));
  BCN_HIP(hipStreamWaitEvent(s, c.join_ev, 0));
}

}  // namespace

void layer_eval(Context& c, EvalKeys& ek, const Layer& L, const double* in, double* out, const float* features,
                hipStream_t s, int R) {
  // R independent requests: in [R][n_in][in_parts][level][N] -> out [R][n_out][out_parts][level_out][N]; every step
  // below runs once over all R requests' ciphertexts (one launch per kernel).
  Arena& ar = *c.arena;
  const size_t N = c.n;
  const int level = L.level;
  const size_t ctw = (size_t)2 * level * N;
  const int nin = R * L.n_in, nout = R * L.n_out;
  if (L.features && !features) throw Error(-1, "layer expects features");
  const bool direct = !L.square && !L.features && L.span == 0 && L.packing == BCN_PACK_BATCH;
  // a slot-batched square layer's MAC writes straight into the Q limbs of the square's
  // Q+B input, so the extension to Q+B only adds the B limbs
  const bool qb = L.packing == BCN_PACK_BATCH && L.square;
  const size_t ctq = (size_t)2 * (level + c.m) * N;
  double* A = direct ? out : ar.take((size_t)nout * (qb ? ctq : ctw));
  bool b_filled = false;        // the MAC wrote the B limbs of the square's Q+B input
  // three-part MAC outputs of a square layer: relinearised, features added and extended to Q+B
  // per ciphertext, inside the square's per-ciphertext chain
  const double* M3 = nullptr;
  double* A2q = nullptr;
  const double* fm3 = nullptr;
  if (L.packing == BCN_PACK_BATCH) {
    // slot batching: the features are quantised straight into the transform domain of R_t,
    // encoded (inverse transform mod t) and added by the MAC's own stores
    double* fm = nullptr;
    if (L.features) {
      fm = ar.take((size_t)nout * N);
      features_to_tdomain(c, features, nout, L.batch, L.stride_b, L.fscale, L.fclamp, fm, s);
      Basis bt{};
      bt.n = 1;
      bt.id[0] = c.id_t;
      ntt_inverse(c, fm, nout, bt, s);
    }
    if (L.in_parts == 3) {
      // unrelinearised inputs: the weighted sums run over the three parts and each output is
      // relinearised once (then the features, then the square's extension to Q+B)
      const size_t ct3 = (size_t)3 * level * N;
      double* M = ar.take((size_t)nout * ct3);
      mac(c, L.mac, in, M, level, s, R, (size_t)L.n_in * ct3, (size_t)L.n_out * ct3, nullptr, 0, 0, nullptr, 3);
      if (qb) {
        M3 = M;
        if (fm) A2q = ar.take((size_t)nout * ctw);
        fm3 = fm;
        b_filled = true;
      } else {
        relinearize3(c, ek, M, A, nout, level, s);
        if (fm) add_delta(c, A, nout, level, fm, s);
      }
    } else if (qb) {
      b_filled = L.mac_ext &&
                 mac_qb(c, L.mac, in, A, level, s, R, (size_t)L.n_in * ctw, (size_t)L.n_out * ctq, fm, ctq, ctq / 2);
      if (!b_filled) mac(c, L.mac, in, A, level, s, R, (size_t)L.n_in * ctw, (size_t)L.n_out * ctq, fm, ctq, ctq / 2);
    } else {
      mac(c, L.mac, in, A, level, s, R, (size_t)L.n_in * ctw, (size_t)L.n_out * ctw, fm);
    }
  } else if (L.diag) {
    // taps [R*n_in][k2] as for a convolution, then all taps times their weight vectors, summed
    double* taps = ar.take((size_t)nin * L.k2 * ctw);
    copy_rows(in, ctw, taps, L.k2 * ctw, ctw, nin, s);
    rotate_hoisted(c, ek, in, nin, level, L.steps, taps + ctw, s, (int)L.steps.size(), L.k2 * ctw);
    ntt_forward(c, taps, 2 * nin * L.k2, c.basis_Q(level), s);
    ptvec_mac_ntt(c, taps, L.n_in * L.k2, A, 1, level, L.ptv_hat, s, R);
    ntt_inverse(c, A, 2 * nout, c.basis_Q(level), s);
  } else if (L.kind == BCN_CONV2D) {
    // taps [R*n_in][k2] over Q_level P in the transform domain (tap 0 = P * the input, taps 1.. =
    // hoisted rotations before their ModDown), weighted sum, mask, then one ModDown per output
    const Basis qp = c.basis_QP(level);
    const size_t ctx = (size_t)2 * qp.n * N;
    double* H = ar.take((size_t)nin * ctw);
    copy_rows(in, 0, H, 0, (size_t)nin * ctw, 1, s);
    ntt_forward(c, H, 2 * nin, c.basis_Q(level), s);
    double* X = ar.take((size_t)nin * L.k2 * ctx);
    taps_extended(c, ek, in, H, nin, level, L.steps, X, s);
    double* U = ar.take((size_t)nout * ctx);
    mac(c, L.mac, X, U, level, s, R, (size_t)L.n_in * L.k2 * ctx, (size_t)L.n_out * ctx, nullptr, 0, 0, &qp, 2,
        L.mask_hat_qp);
    ntt_inverse(c, U, 2 * nout, qp, s);
    moddown(c, U, nout, level, nullptr, 1, 0, 0, KeySel(), false, A, s);
  } else {
    double* H = ar.take((size_t)nin * ctw);
    copy_rows(in, 0, H, 0, (size_t)nin * ctw, 1, s);
    ntt_forward(c, H, 2 * nin, c.basis_Q(level), s);
    ptvec_mac_ntt(c, H, L.n_in, A, L.n_out, level, L.ptv_hat, s, R);
    ntt_inverse(c, A, 2 * nout, c.basis_Q(level), s);
  }
  if (L.features && L.packing != BCN_PACK_BATCH) {
    // HW packing: features enter after the conv's mask
    double* m = ar.take((size_t)nout * N);
    int64_t* sl = reinterpret_cast<int64_t*>(ar.take((size_t)nout * N));
    fill(reinterpret_cast<double*>(sl), (size_t)nout * N, 0.0, s);   // all-zero bits = int64 zeros
    quantise_features(c, features, nout, 1, 0, 0, L.slot_of, L.per, L.fscale, L.fclamp, sl, s);
    encode_device(c, sl, m, nout, s);
    add_delta(c, A, nout, level, m, s);
  }
  if (direct) return;
  const bool hw_dense = L.packing == BCN_PACK_HW && L.kind == BCN_DENSE && !L.diag;
  if (hw_dense) {
    // rotate-and-sum before the (optional) square
    rotate_sum(c, ek, A, nout, level, L.span, s);
    if (L.square) {
      square_relin(c, ek, A, out, nout, level, L.modsw, s);
    } else {
      copy_rows(A, 0, out, 0, (size_t)nout * ctw, 1, s);
    }
    return;
  }
  if (qb) {
    const size_t ct3 = (size_t)3 * level * N;
    const size_t out_ct = (size_t)(L.defer ? 3 : 2) * L.level_out * N;
    run_halves(c, nout, s, [&](int o0, int cnt, hipStream_t st) {
      double* a = A + (size_t)o0 * ctq;
      if (M3 && !fm3) {
        // relinearisation's ModDown writes the square's Q+B input itself
        relinearize3(c, ek, M3 + (size_t)o0 * ct3, a, cnt, level, st, true);
      } else if (M3) {
        double* a2 = A2q + (size_t)o0 * ctw;
        relinearize3(c, ek, M3 + (size_t)o0 * ct3, a2, cnt, level, st);
        add_delta(c, a2, cnt, level, fm3 + (size_t)o0 * N, st);
        extend_qb(c, a2, a, cnt, level, st);
      }
      if (L.defer)
        square_defer(c, a, out + (size_t)o0 * out_ct, cnt, level, L.modsw, st, b_filled);
      else
        square_relin_qb(c, ek, a, out + (size_t)o0 * out_ct, cnt, level, L.modsw, st, b_filled);
    });
  } else if (L.square && L.defer) {
    double* X = ar.take((size_t)nout * ctq);
    extend_qb(c, A, X, nout, level, s);
    square_defer(c, X, out, nout, level, L.modsw, s, true);
  } else if (L.square) {
    square_relin(c, ek, A, out, nout, level, L.modsw, s);
  } else {
    copy_rows(A, 0, out, 0, (size_t)nout * ctw, 1, s);
  }
  if (L.span > 0) rotate_sum(c, ek, out, nout, L.level_out, L.span, s);
}

}  // namespace bcn
