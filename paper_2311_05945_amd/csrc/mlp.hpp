// Warm-start network object of the HIP library (per-vertex MLP 16-64-64-64-3).
#pragma once
#include <string>

#include "../../include/zema.h"
#include "common.hpp"

namespace zema {
constexpr int kMlpParams = 9603;    // W1 64x16, b1, W2 64x64, b2, W3 64x64, b3, W4 3x64, b4
constexpr int kTilesPerBlock = 4;   // 16-vertex tiles per training wavefront
// allocation-free gradient: at most this many block partials, each block taking
// ceil(tiles / kNoAllocBlocks) (at least kTilesPerBlock) 16-row tiles
constexpr int kNoAllocBlocks = 256;
}  // namespace zema

struct zema_mlp {
  hipStream_t st = nullptr;
  std::string err;
  zema::DBuf<float> theta, mom, vel, grad, gpart;  // FP32 master weights, Adam moments
  zema::DBuf<double> lpart, loss;
  long long step = 0;
  int dev = 0;  // device current at creation (holds theta and the Adam state)
};

namespace zema {
void mlp_forward(const zema_mlp* M, hipStream_t st, const float* feat, long n, float* out);
// loss of the batch; grad (and, with adam, one Adam step) left on the device
double mlp_grad(zema_mlp* M, const float* feat, const float* target, const int* idx, long nrows, long n, bool adam,
                float lr);
// loss and gradient (into grad, device) with every partial in the library's static
// per-device scratch array; no device memory is allocated
double mlp_grad_noalloc(zema_mlp* M, const float* feat, const float* target, long n, float* grad);
}  // namespace zema
