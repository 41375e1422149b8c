// Learned initial guess of the interface PCG: a small multilayer perceptron
// trained on the solver's own trajectories (the C ABI is in sgw.h).
//
// A plain perceptron with two hidden layers: n_in -> H (ReLU) -> H (ReLU) ->
// n_out, applied to the rows of a batch.  The solver's guess uses n_in = 4,
// n_out = 1, one row per (PCE mode, interface node) (see sgw.h).  FP32
// master parameters (updated by Adam), BF16 copies of the weight matrices
// for the matrix products, which run on MFMA with FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "sgw.h"

struct sgw_mlp {
  int ng = 0, nin = 0, H = 0;   // outputs, inputs, hidden width
  long long np = 0;             // number of parameters
  long long off[6] = {0, 0, 0, 0, 0, 0};  // W1 b1 W2 b2 W3 b3 in the parameter vector
  sgw_allocator al{};
  bool has_al = false;
  std::vector<void*> mem;
  std::string err;
  float* w = nullptr;           // FP32 master parameters [np]
  unsigned short* wb = nullptr; // BF16 copy, same layout (biases unused)
  float *g = nullptr, *m = nullptr, *v = nullptr;  // gradient, Adam moments
  long long adam_t = 0;
  // work space for batches of up to cap rows
  int cap = 0;
  float *xb = nullptr, *tb = nullptr, *y = nullptr, *d2 = nullptr, *d1 = nullptr, *dy = nullptr,
        *loss = nullptr;
  unsigned short *h1 = nullptr, *h2 = nullptr;  // hidden activations, BF16
  float* part = nullptr;        // partial sums of the gradient reductions
  int* perm = nullptr;          // sample permutation of an epoch
  int perm_cap = 0;
  float* hloss = nullptr;       // pinned
};

namespace sgw {
// y[nb][ng] = network(x[nb][nin]) on stream st (device arrays); returns 0
// or a negative SGW_* code.
int mlp_forward(sgw_mlp* m, const float* x, float* y, int nb, hipStream_t st);
}  // namespace sgw
