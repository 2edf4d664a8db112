#pragma once

#include "../../include/bcn.h"
#include <functional>
#include <string>

#include "scheme.h"

namespace bcn {

struct Layer {
  int kind = 0, packing = 0, level = 0, level_out = 0;
  int n_in = 0, n_out = 0;
  int oh = 0, ow = 0, k2 = 0;
  bool diag = false;             // HW dense by the diagonal method (taps as in a convolution)
  bool square = false, modsw = false, features = false;
  float fscale = 8.0f;
  int fclamp = 127;
  int batch = 0, stride_b = 0;
  MacPlan mac;
  int in_parts = 2;              // 3: inputs are unrelinearised products (relinearised after the MAC)
  bool defer = false;            // the square's output stays unrelinearised (3 parts)
  bool mac_ext = true;           // slot-batched square layer: the MAC writes the B limbs too (when supported)
  std::vector<int32_t> mac_weights;  // host copy of the MAC matrix (for retuning)
  std::vector<int> mac_order;
  std::vector<int> steps;        // HW conv: nonzero tap offsets, tap index = position + 1
  std::vector<int> all_steps;    // every Galois step the layer needs
  double* mask_hat_qp = nullptr; // [level + K][N]: the conv mask over Q_level then P
  double* ptv_hat = nullptr;     // [n_out][n_in][level][N]
  int* slot_of = nullptr;        // [per] output slot of each output position (HW)
  int per = 0;
  int span = 0;                  // rotate-and-sum span (0 = none)
  ~Layer();
};

Layer* layer_create(Context& c, const bcn_layer_desc& d, int level);
std::string autotune_ntt(Context& c, hipStream_t s);
std::string autotune_layer_mac(Context& c, Layer& L, hipStream_t s);
void layer_eval(Context& c, EvalKeys& ek, const Layer& L, const double* in, double* out, const float* features,
                hipStream_t s, int requests = 1);

}  // namespace bcn
