// Refinement network: a 288 -> 128 -> 128 -> 1 perceptron that proposes the
// split / no-split decision of a quadtree box from samples of the source on
// the box (the adaptive refinement of section 3.1; the plain tail criterion
// still checks every leaf).  BF16 operands on the matrix cores, FP32 sums,
// FP32 master parameters and Adam moments.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bx {

constexpr int MLP_IN = 288, MLP_HID = 128;
// flat parameter layout: W1[128][288], b1[128], W2[128][128], b2[128], w3[128], b3
constexpr int MLP_OW1 = 0, MLP_OB1 = MLP_OW1 + MLP_HID * MLP_IN, MLP_OW2 = MLP_OB1 + MLP_HID,
              MLP_OB2 = MLP_OW2 + MLP_HID * MLP_HID, MLP_OW3 = MLP_OB2 + MLP_HID, MLP_OB3 = MLP_OW3 + MLP_HID,
              MLP_NPARAM = MLP_OB3 + 1;

struct MlpDev {
  float *theta;      // FP32 parameters [MLP_NPARAM]
  float *grad;       // gradient of the last bx_mlp_grad [MLP_NPARAM]
  float *m, *v;      // Adam moments [MLP_NPARAM]
  float *loss;       // mean loss of the last bx_mlp_grad [1]
  uint16_t *w1b;     // BF16 W1 [128][288]
  uint16_t *w2b;     // BF16 W2 [128][128]
  uint16_t *w2tb;    // BF16 W2 transposed [128][128]
};

void launch_mlp_features(const double *samples, const int8_t *level, long long n, uint16_t *x, hipStream_t s);
void launch_mlp_refresh(const MlpDev &m, hipStream_t s);   // BF16 copies from theta
void launch_mlp_forward(const MlpDev &m, const uint16_t *x, long long n, float *logit, hipStream_t s);
void launch_mlp_grad(const MlpDev &m, const uint16_t *x, const float *y, long long n, hipStream_t s);
void launch_mlp_adam(const MlpDev &m, float lr, float beta1, float beta2, float eps, float c1, float c2,
                     hipStream_t s);

}  // namespace bx
