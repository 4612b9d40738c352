// Kernels of the refinement network (see mlp.h).
//
// v_mfma_f32_16x16x32_bf16 operand layout (lane l, i = l % 16, q = l / 16):
// A[i][8q + e] and B[8q + e][i] are element e of the lane's 8-element
// operands; the accumulator holds D[4q + r][i] in register r.  A block of
// 256 threads takes 64 boxes, 16 per wave.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "mlp.h"

namespace bx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest BF16, ties to even (finite inputs)
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline f32x4 mfma(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// features of a box from samples s[16][16] and level l (one wave per box):
// s / max|s|, l / 16, clip((log10 max|s| + 10) / 10, -1, 2),
// max(log10 max|s|, -320) / 320, zeros to 288
__global__ void __launch_bounds__(256) mlp_features_kernel(const double *__restrict__ s,
                                                           const int8_t *__restrict__ level, long long n,
                                                           uint16_t *__restrict__ x) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * 4;
  for (long long b = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); b < n; b += nw) {
    const double *sb = s + b * 256;
    double v[4], a = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = sb[lane + 64 * j];
      a = fmax(a, fabs(v[j]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o));
    uint16_t *xb = x + b * MLP_IN;
#pragma unroll
    for (int j = 0; j < 4; ++j) xb[lane + 64 * j] = a > 0.0 ? to_bf16((float)(v[j] / a)) : (uint16_t)0;
    if (lane < 32) {
      double e = 0.0;
      if (lane == 0) e = level[b] / 16.0;
      if (lane == 1) e = a > 0.0 ? fmin(2.0, fmax(-1.0, (log10(a) + 10.0) / 10.0)) : -1.0;
      if (lane == 2) e = a > 0.0 ? fmax(log10(a), -320.0) / 320.0 : -1.0;
      xb[256 + lane] = to_bf16((float)e);
    }
  }
}

constexpr int HP = MLP_HID + 8;   // row pitch (elements) of the row-major activations in LDS
constexpr int TP = 64 + 8;        // row pitch of the transposed (feature-major) copies
constexpr int LDS_FWD = 64 * HP;
constexpr int LDS_TRAIN = 2 * 64 * HP + 3 * MLP_HID * TP + MLP_IN * TP;

// Forward pass of 64 boxes per block; with TRAIN also the backward pass of
// the mean binary cross-entropy, the weight gradients of these boxes added
// to m.grad (FP32 atomics) and their loss to m.loss.
template <bool TRAIN>
__global__ void __launch_bounds__(256) mlp_kernel(MlpDev m, const uint16_t *__restrict__ x,
                                                  const float *__restrict__ y, long long n, float inv_n,
                                                  float *__restrict__ logit) {
  __shared__ __attribute__((aligned(16))) uint16_t smem[TRAIN ? LDS_TRAIN : LDS_FWD];
  uint16_t *sH1 = smem;                          // [64][HP]   bf16(h1)
  uint16_t *sD2 = smem + 64 * HP;                // [64][HP]   bf16(dL/dz2)
  uint16_t *sH1T = smem + 2 * 64 * HP;           // [128][TP]  transposed copies
  uint16_t *sD2T = sH1T + MLP_HID * TP;
  uint16_t *sD1T = sD2T + MLP_HID * TP;
  uint16_t *sXT = sD1T + MLP_HID * TP;           // [288][TP]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, q = lane >> 4;
  const long long rb = (long long)blockIdx.x * 64 + w * 16;   // first box of this wave
  const long long row = rb + i < n ? rb + i : n - 1;         // A-operand row (clamped)

  // layer 1: z1 = x W1^T + b1 (9 K steps of 32, 8 column tiles)
  f32x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint4 *xr = (const uint4 *)(x + row * MLP_IN);
  for (int ks = 0; ks < MLP_IN / 32; ++ks) {
    const uint4 a = xr[ks * 4 + q];
    if constexpr (TRAIN) {
      const uint16_t *ae = (const uint16_t *)&a;
#pragma unroll
      for (int e = 0; e < 8; ++e) sXT[(ks * 32 + 8 * q + e) * TP + w * 16 + i] = ae[e];
    }
    uint4 b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) b[t] = ((const uint4 *)(m.w1b + (t * 16 + i) * MLP_IN))[ks * 4 + q];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(a, b[t], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int col = t * 16 + i;
    const float bias = m.theta[MLP_OB1 + col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint16_t h = to_bf16(fmaxf(acc[t][r] + bias, 0.f));
      sH1[(w * 16 + 4 * q + r) * HP + col] = h;
      if constexpr (TRAIN) sH1T[col * TP + w * 16 + 4 * q + r] = h;
    }
  }
  __syncthreads();

  // layer 2: z2 = h1 W2^T + b2; h2 = relu(z2) stays in registers
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < MLP_HID / 32; ++ks) {
    const uint4 a = *(const uint4 *)(sH1 + (w * 16 + i) * HP + ks * 32 + 8 * q);
    uint4 b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) b[t] = ((const uint4 *)(m.w2b + (t * 16 + i) * MLP_HID))[ks * 4 + q];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(a, b[t], acc[t]);
  }
  float w3[8];
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int col = t * 16 + i;
    const float bias = m.theta[MLP_OB2 + col];
    w3[t] = m.theta[MLP_OW3 + col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[t][r] += bias;                          // z2
      part[r] += fmaxf(acc[t][r], 0.f) * w3[t];
    }
  }
  // layer 3: the logit of box 4q + r is the sum over the 16 lanes of group q
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) part[r] += __shfl_xor(part[r], o);
  const float b3 = m.theta[MLP_OB3];
  if constexpr (!TRAIN) {
    if (i == 0)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (rb + 4 * q + r < n) logit[rb + 4 * q + r] = part[r] + b3;
    return;
  }

  // backward: dL/dlogit = (sigmoid - y) / N per box, 0 for boxes past n
  float dz3[4], lsum = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const long long bi = rb + 4 * q + r;
    const float z = part[r] + b3;
    if (bi < n) {
      const float yy = y[bi];
      dz3[r] = (1.f / (1.f + expf(-z)) - yy) * inv_n;
      lsum += fmaxf(z, 0.f) - z * yy + log1pf(expf(-fabsf(z)));
    } else {
      dz3[r] = 0.f;
    }
  }
  // per-wave sums over the 4 row groups (lanes i, i + 16, i + 32, i + 48)
  auto qsum = [](float v) {
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
  };
  const float db3 = qsum(dz3[0] + dz3[1] + dz3[2] + dz3[3]);
  lsum = qsum(lsum);
  if (lane == 0) {
    atomicAdd(m.grad + MLP_OB3, db3);
    atomicAdd(m.loss, lsum * inv_n);
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int col = t * 16 + i;
    float gw3 = 0.f, gb2 = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float z2 = acc[t][r];
      gw3 += fmaxf(z2, 0.f) * dz3[r];
      const float d2 = z2 > 0.f ? dz3[r] * w3[t] : 0.f;
      gb2 += d2;
      const uint16_t hb = to_bf16(d2);
      sD2[(w * 16 + 4 * q + r) * HP + col] = hb;
      sD2T[col * TP + w * 16 + 4 * q + r] = hb;
    }
    gw3 = qsum(gw3);
    gb2 = qsum(gb2);
    if (q == 0) {
      atomicAdd(m.grad + MLP_OW3 + col, gw3);
      atomicAdd(m.grad + MLP_OB2 + col, gb2);
    }
  }
  __syncthreads();

  // dL/dz1 = bf16(dL/dz2) W2, masked where h1 = 0
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < MLP_HID / 32; ++ks) {
    const uint4 a = *(const uint4 *)(sD2 + (w * 16 + i) * HP + ks * 32 + 8 * q);
    uint4 b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) b[t] = ((const uint4 *)(m.w2tb + (t * 16 + i) * MLP_HID))[ks * 4 + q];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = mfma(a, b[t], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int col = t * 16 + i;
    float gb1 = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = w * 16 + 4 * q + r;
      const float d1 = (sH1[rr * HP + col] & 0x7fff) ? acc[t][r] : 0.f;
      gb1 += d1;
      sD1T[col * TP + rr] = to_bf16(d1);
    }
    gb1 = qsum(gb1);
    if (q == 0) atomicAdd(m.grad + MLP_OB1 + col, gb1);
  }
  __syncthreads();

  // weight gradients over the block's 64 boxes (K = 64: two MFMA steps):
  // dW2[o][j] = sum_b dz2[b][o] h1[b][j], dW1[o][j] = sum_b dz1[b][o] x[b][j]
  for (int tile = w; tile < 8 * 8; tile += 4) {
    const int o0 = (tile >> 3) * 16, j0 = (tile & 7) * 16;
    f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const uint4 a = *(const uint4 *)(sD2T + (o0 + i) * TP + kk * 32 + 8 * q);
      const uint4 b = *(const uint4 *)(sH1T + (j0 + i) * TP + kk * 32 + 8 * q);
      c = mfma(a, b, c);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) atomicAdd(m.grad + MLP_OW2 + (o0 + 4 * q + r) * MLP_HID + j0 + i, c[r]);
  }
  for (int tile = w; tile < 8 * (MLP_IN / 16); tile += 4) {
    const int o0 = (tile % 8) * 16, j0 = (tile / 8) * 16;
    f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const uint4 a = *(const uint4 *)(sD1T + (o0 + i) * TP + kk * 32 + 8 * q);
      const uint4 b = *(const uint4 *)(sXT + (j0 + i) * TP + kk * 32 + 8 * q);
      c = mfma(a, b, c);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) atomicAdd(m.grad + MLP_OW1 + (o0 + 4 * q + r) * MLP_IN + j0 + i, c[r]);
  }
}

__global__ void __launch_bounds__(256) mlp_zero_kernel(MlpDev m) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < MLP_NPARAM; k += gridDim.x * 256) m.grad[k] = 0.f;
  if (blockIdx.x == 0 && threadIdx.x == 0) m.loss[0] = 0.f;
}

// BF16 copies of W1 and W2 (and W2 transposed) from parameter k
__device__ inline void refresh_one(const MlpDev &m, int k, float wv) {
  if (k < MLP_OB1) {
    m.w1b[k - MLP_OW1] = to_bf16(wv);
  } else if (k >= MLP_OW2 && k < MLP_OB2) {
    const int e = k - MLP_OW2, o = e / MLP_HID, j = e % MLP_HID;
    const uint16_t h = to_bf16(wv);
    m.w2b[e] = h;
    m.w2tb[j * MLP_HID + o] = h;
  }
}

__global__ void __launch_bounds__(256) mlp_refresh_kernel(MlpDev m) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < MLP_NPARAM; k += gridDim.x * 256) refresh_one(m, k, m.theta[k]);
}

// one Adam step; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
__global__ void __launch_bounds__(256) mlp_adam_kernel(MlpDev m, float lr, float beta1, float beta2, float eps,
                                                       float c1, float c2) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < MLP_NPARAM; k += gridDim.x * 256) {
    const float g = m.grad[k];
    const float mk = beta1 * m.m[k] + (1.f - beta1) * g;
    const float vk = beta2 * m.v[k] + (1.f - beta2) * g * g;
    const float wv = m.theta[k] - lr * (mk * c1) / (sqrtf(vk * c2) + eps);
    m.m[k] = mk;
    m.v[k] = vk;
    m.theta[k] = wv;
    refresh_one(m, k, wv);
  }
}

}  // namespace

void launch_mlp_features(const double *samples, const int8_t *level, long long n, uint16_t *x, hipStream_t s) {
  if (n <= 0) return;
  const long long nb = (n + 3) / 4;
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)(nb < 65536 ? nb : 65536)), dim3(256), 0, s, samples,
                     level, n, x);
}

void launch_mlp_refresh(const MlpDev &m, hipStream_t s) {
  hipLaunchKernelGGL(mlp_refresh_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, m);
}

void launch_mlp_forward(const MlpDev &m, const uint16_t *x, long long n, float *logit, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_kernel<false>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, m, x,
                     (const float *)nullptr, n, 0.f, logit);
}

void launch_mlp_grad(const MlpDev &m, const uint16_t *x, const float *y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(mlp_zero_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, m);
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_kernel<true>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, m, x, y, n,
                     (float)(1.0 / (double)n), (float *)nullptr);
}

void launch_mlp_adam(const MlpDev &m, float lr, float beta1, float beta2, float eps, float c1, float c2,
                     hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, m, lr, beta1, beta2, eps,
                     c1, c2);
}

}  // namespace bx
