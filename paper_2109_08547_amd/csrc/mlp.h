// Internal: the screening MLP (mlp.hip) used by the learned screen (screen.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/elph.h"

struct elph_mlp_s {
  std::string err;
  bool hip_dead = false;
  hipStream_t stream = nullptr;
  int nin = 0, in_pad = 0, width = 0, depth = 0;
  int64_t nparams = 0;
  std::vector<int64_t> w_off, b_off;     // offsets of W_l and b_l in the flat vector
  std::vector<int> fan_in, fan_out;      // per layer (depth hidden layers + output)
  float* d_params = nullptr;             // master FP32 parameters (flat)
  float* d_grad = nullptr;               // FP32 gradient (flat)
  float* d_m = nullptr;                  // Adam moments
  float* d_v = nullptr;
  int64_t step = 0;
  std::vector<unsigned short*> d_W;      // BF16 W_l [in_pad or width][width]  (hidden layers)
  std::vector<unsigned short*> d_Wt;     // BF16 W_l^T [width][in_pad or width]
  unsigned short* d_wout = nullptr;      // BF16 output weights [width]
  // activations for a batch of up to cap rows
  int64_t cap = 0;
  unsigned short* d_x = nullptr;         // [cap][in_pad]
  std::vector<unsigned short*> d_h;      // [depth][cap][width] BF16 activations
  std::vector<float*> d_z;               // [depth][cap][width] FP32 pre-activations
  unsigned short* d_dz[2] = {nullptr, nullptr};  // [cap][width] BF16 backward signals
  float* d_y = nullptr;                  // [cap]
  float* d_part = nullptr;               // reduction partials
  int64_t part_len = 0;
  float* h_pin = nullptr;                // pinned host words
  std::vector<void*> allocs;
};

namespace elph {

// Forward pass of n rows whose BF16 padded inputs are already in m->d_x
// (n <= m->cap); keep = store the FP32 pre-activations for a backward pass.
// y [n] FP32 on the MLP stream.
elph_status mlp_forward_rows(elph_mlp m, int64_t n, bool keep, float* y);
// Make room for batches of n rows.
elph_status mlp_reserve(elph_mlp m, int64_t n);

}  // namespace elph
