// Device kernels of the box code (gfx950).
//
// Expansions are stored per box as KP complex coefficients (re, im
// interleaved), scaled by powers of the box width h: multipole a~_k = a_k / h^k,
// local b~_l = b_l h^l.  With this scaling every translation operator is the
// same at every level; only a_0 log h terms and the 1/h of gradients carry the
// level, and they are applied here in FP64.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace bx {
namespace {

constexpr double kInv2Pi = 0.15915494309189533577;

__device__ inline double box_h(double width, int level) { return ldexp(width, -level); }

// ------------------------------------------------------------------ P2M
// a~ = h^2 * P2M * f (leaf samples), one block per (leaf, rhs).
__global__ void __launch_bounds__(64) p2m_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                 double *__restrict__ M) {
  __shared__ double fs[256];
  const int leaf = blockIdx.x, rhs = blockIdx.y;
  const double *fl = f + ((size_t)rhs * g.n_leaves + leaf) * t.P;
  for (int j = threadIdx.x; j < t.P; j += blockDim.x) fs[j] = fl[j];
  __syncthreads();
  const double h = box_h(g.width, g.leaf_level[leaf]), h2 = h * h;
  double *Mb = M + ((size_t)rhs * g.n_boxes + g.box_of_leaf[leaf]) * t.KP * 2;
  for (int k = threadIdx.x; k < t.KP; k += blockDim.x) {
    double re = 0.0, im = 0.0;
    if (k < t.nt) {
      const double *ar = t.p2m + (size_t)k * t.P, *ai = t.p2m + (size_t)(t.KP + k) * t.P;
      for (int j = 0; j < t.P; ++j) {
        re = fma(ar[j], fs[j], re);
        im = fma(ai[j], fs[j], im);
      }
    }
    Mb[2 * k] = re * h2;
    Mb[2 * k + 1] = im * h2;
  }
}

// ------------------------------------------------------------------ M2M
// parent from its four children, one block per (box at this level, rhs).
__global__ void __launch_bounds__(64) m2m_kernel(DevTables t, DevTree g, int box0, double *__restrict__ M) {
  __shared__ double cs[4 * 64 * 2];
  const int box = box0 + blockIdx.x, rhs = blockIdx.y;
  const int c0 = g.child0[box];
  if (c0 < 0) return;
  double *Mr = M + (size_t)rhs * g.n_boxes * t.KP * 2;
  for (int i = threadIdx.x; i < 4 * t.KP * 2; i += blockDim.x) {
    int c = i / (t.KP * 2), r = i % (t.KP * 2);
    cs[i] = Mr[(size_t)(c0 + c) * t.KP * 2 + r];
  }
  __syncthreads();
  for (int l = threadIdx.x; l < t.KP; l += blockDim.x) {
    double re = 0.0, im = 0.0;
    if (l < t.nt)
      for (int c = 0; c < 4; ++c) {
        const double *op = t.m2m + ((size_t)c * t.nt + l) * t.nt * 2;
        const double *a = cs + c * t.KP * 2;
        for (int k = 0; k <= l; ++k) {
          double orr = op[2 * k], oi = op[2 * k + 1], ar = a[2 * k], ai = a[2 * k + 1];
          re += orr * ar - oi * ai;
          im += orr * ai + oi * ar;
        }
      }
    Mr[(size_t)box * t.KP * 2 + 2 * l] = re;
    Mr[(size_t)box * t.KP * 2 + 2 * l + 1] = im;
  }
}

// ------------------------------------------------------------------ M2L
// b~_l = sum_s (d/2)^-l sum_k H[l][k] y_k(s) + [l=0] sum_s a_0 (log h + log|d|),
// y_k = a~_k (-d/2)^-k.  Writes (initialises) the local expansion of every box.
__global__ void __launch_bounds__(64) m2l_kernel(DevTables t, DevTree g, const double *__restrict__ M,
                                                 double *__restrict__ L) {
  __shared__ double ys[64 * 2];
  const int box = blockIdx.x, rhs = blockIdx.y, l = threadIdx.x;
  const double *Mr = M + (size_t)rhs * g.n_boxes * t.KP * 2;
  const double logh = log(box_h(g.width, g.lvl[box]));
  double accr = 0.0, acci = 0.0, a0 = 0.0;
  for (int e = g.v_ptr[box]; e < g.v_ptr[box + 1]; ++e) {
    const int s = g.v_src[e], o = g.v_cfg[e];
    if (l < t.KP) {
      double ar = Mr[(size_t)s * t.KP * 2 + 2 * l], ai = Mr[(size_t)s * t.KP * 2 + 2 * l + 1];
      double pr = t.pw_src[((size_t)o * t.KP + l) * 2], pi = t.pw_src[((size_t)o * t.KP + l) * 2 + 1];
      ys[2 * l] = l < t.nt ? ar * pr - ai * pi : 0.0;
      ys[2 * l + 1] = l < t.nt ? ar * pi + ai * pr : 0.0;
      if (l == 0) a0 += ar * (logh + t.logd[o]);
    }
    __syncthreads();
    if (l < t.nt) {
      double zr = 0.0, zi = 0.0;
      const double *Hl = t.H + (size_t)l * t.KP;
      for (int k = 0; k < t.nt; ++k) {
        zr = fma(Hl[k], ys[2 * k], zr);
        zi = fma(Hl[k], ys[2 * k + 1], zi);
      }
      double qr = t.pw_tgt[((size_t)o * t.KP + l) * 2], qi = t.pw_tgt[((size_t)o * t.KP + l) * 2 + 1];
      accr += zr * qr - zi * qi;
      acci += zr * qi + zi * qr;
    }
    __syncthreads();
  }
  if (l < t.KP) {
    double *Lb = L + ((size_t)rhs * g.n_boxes + box) * t.KP * 2;
    Lb[2 * l] = accr + (l == 0 ? a0 : 0.0);
    Lb[2 * l + 1] = acci;
  }
}

// ------------------------------------------------------------------ P2L
// X list: b~ += h^2 * P2L_c * f_s, b~_0 += h^2 log h * 4 (W . f_s).
__global__ void __launch_bounds__(64) p2l_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                 double *__restrict__ L) {
  __shared__ double fs[256];
  const int box = blockIdx.x, rhs = blockIdx.y;
  const int e0 = g.x_ptr[box], e1 = g.x_ptr[box + 1];
  if (e0 == e1) return;
  const double h = box_h(g.width, g.lvl[box]), h2 = h * h;
  double re[2] = {0.0, 0.0}, im[2] = {0.0, 0.0}, mass = 0.0;
  for (int e = e0; e < e1; ++e) {
    const int s = g.x_src[e], c = g.x_cfg[e];
    const double *fl = f + ((size_t)rhs * g.n_leaves + s) * t.P;
    for (int j = threadIdx.x; j < t.P; j += blockDim.x) fs[j] = fl[j];
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      int l = threadIdx.x + q * blockDim.x;
      if (l < t.nt) {
        const double *ar = t.p2l + ((size_t)c * 2 * t.KP + l) * t.P;
        const double *ai = t.p2l + ((size_t)c * 2 * t.KP + t.KP + l) * t.P;
        for (int j = 0; j < t.P; ++j) {
          re[q] = fma(ar[j], fs[j], re[q]);
          im[q] = fma(ai[j], fs[j], im[q]);
        }
      }
    }
    if (threadIdx.x == 0)
      for (int j = 0; j < t.P; ++j) mass = fma(t.wq[j], fs[j], mass);
    __syncthreads();
  }
  double *Lb = L + ((size_t)rhs * g.n_boxes + box) * t.KP * 2;
  for (int q = 0; q < 2; ++q) {
    int l = threadIdx.x + q * blockDim.x;
    if (l < t.nt) {
      Lb[2 * l] += h2 * re[q] + (l == 0 ? 4.0 * h2 * log(h) * mass : 0.0);
      Lb[2 * l + 1] += h2 * im[q];
    }
  }
}

// ------------------------------------------------------------------ L2L
__global__ void __launch_bounds__(64) l2l_kernel(DevTables t, DevTree g, int box0, double *__restrict__ L) {
  __shared__ double ps[64 * 2];
  const int box = box0 + blockIdx.x, rhs = blockIdx.y;
  const int par = g.parent[box];
  const int c = box - g.child0[par];
  double *Lr = L + (size_t)rhs * g.n_boxes * t.KP * 2;
  for (int i = threadIdx.x; i < t.KP * 2; i += blockDim.x) ps[i] = Lr[(size_t)par * t.KP * 2 + i];
  __syncthreads();
  for (int m = threadIdx.x; m < t.nt; m += blockDim.x) {
    const double *op = t.l2l + ((size_t)c * t.nt + m) * t.nt * 2;
    double re = 0.0, im = 0.0;
    for (int l = m; l < t.nt; ++l) {
      double orr = op[2 * l], oi = op[2 * l + 1], br = ps[2 * l], bi = ps[2 * l + 1];
      re += orr * br - oi * bi;
      im += orr * bi + oi * br;
    }
    Lr[(size_t)box * t.KP * 2 + 2 * m] += re;
    Lr[(size_t)box * t.KP * 2 + 2 * m + 1] += im;
  }
}

// --------------------------------------------------------- L2T and W list
// V = L2T_V b~ + sum_W (M2T_V a~ + a_0 log(h/2) / 2pi),
// grad V = L2T_D b~ / h + sum_W M2T_D a~ / (h/2).  Writes V and G.
__global__ void __launch_bounds__(256) leaf_far_kernel(DevTables t, DevTree g, const double *__restrict__ M,
                                                       const double *__restrict__ L, double *__restrict__ V,
                                                       double *__restrict__ G) {
  __shared__ double vec[2 * 64];   // [re_0..re_KP-1, im_0..im_KP-1]
  const int leaf = blockIdx.x, rhs = blockIdx.y;
  const int box = g.box_of_leaf[leaf];
  const double h = box_h(g.width, g.leaf_level[leaf]), hs = 0.5 * h;
  const int P = t.P, K2 = 2 * t.KP;
  double acc[3] = {0.0, 0.0, 0.0};
  const double *Lb = L + ((size_t)rhs * g.n_boxes + box) * t.KP * 2;
  for (int i = threadIdx.x; i < t.KP; i += blockDim.x) {
    vec[i] = Lb[2 * i];
    vec[t.KP + i] = Lb[2 * i + 1];
  }
  __syncthreads();
  for (int q = 0; q < 3; ++q) {
    int r = threadIdx.x + q * blockDim.x;
    if (r < 3 * P) {
      const double *row = t.l2t + (size_t)r * K2;
      double s = 0.0;
      for (int k = 0; k < K2; ++k) s = fma(row[k], vec[k], s);
      acc[q] = r < P ? s : s / h;
    }
  }
  __syncthreads();
  const double *Mr = M + (size_t)rhs * g.n_boxes * t.KP * 2;
  for (int e = g.w_ptr[leaf]; e < g.w_ptr[leaf + 1]; ++e) {
    const int s = g.w_src[e], c = g.w_cfg[e];
    for (int i = threadIdx.x; i < t.KP; i += blockDim.x) {
      vec[i] = Mr[(size_t)s * t.KP * 2 + 2 * i];
      vec[t.KP + i] = Mr[(size_t)s * t.KP * 2 + 2 * i + 1];
    }
    __syncthreads();
    for (int q = 0; q < 3; ++q) {
      int r = threadIdx.x + q * blockDim.x;
      if (r < 3 * P) {
        const double *row = t.m2t + ((size_t)c * 3 * P + r) * K2;
        double sum = 0.0;
        for (int k = 0; k < K2; ++k) sum = fma(row[k], vec[k], sum);
        acc[q] += r < P ? sum + vec[0] * log(hs) * kInv2Pi : sum / hs;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < 3; ++q) {
    int r = threadIdx.x + q * blockDim.x;
    if (r < P) V[((size_t)rhs * g.n_leaves + leaf) * P + r] = acc[q];
    else if (r < 3 * P) G[((size_t)rhs * g.n_leaves + leaf) * 2 * P + (r - P)] = acc[q];
  }
}

// ------------------------------------------------------------ near tables
// V += h^2 T f + (h^2 log h / 2pi) (W . f), grad V += h D f over the U list.
__global__ void __launch_bounds__(256) near_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                   double *__restrict__ V, double *__restrict__ G) {
  __shared__ double fs[256];
  const int leaf = blockIdx.x, rhs = blockIdx.y;
  const int P = t.P;
  const double h = box_h(g.width, g.leaf_level[leaf]);
  double acc[3] = {0.0, 0.0, 0.0}, mass = 0.0;
  for (int e = g.u_ptr[leaf]; e < g.u_ptr[leaf + 1]; ++e) {
    const int s = g.u_src[e], c = g.u_cfg[e];
    const double *fl = f + ((size_t)rhs * g.n_leaves + s) * P;
    for (int j = threadIdx.x; j < P; j += blockDim.x) fs[j] = fl[j];
    __syncthreads();
    const double *Tc = t.near_ + (size_t)c * t.MR * P;
    for (int q = 0; q < 3; ++q) {
      int r = threadIdx.x + q * blockDim.x;
      if (r < 3 * P) {
        double sum = 0.0;
        for (int j = 0; j < P; ++j) sum = fma(Tc[(size_t)r * P + j], fs[j], sum);
        acc[q] += sum;
      }
    }
    for (int j = 0; j < P; ++j) mass = fma(Tc[(size_t)3 * P * P + j], fs[j], mass);
    __syncthreads();
  }
  const double h2 = h * h, lg = h2 * log(h) * kInv2Pi * mass;
  for (int q = 0; q < 3; ++q) {
    int r = threadIdx.x + q * blockDim.x;
    if (r < P) V[((size_t)rhs * g.n_leaves + leaf) * P + r] += h2 * acc[q] + lg;
    else if (r < 3 * P) G[((size_t)rhs * g.n_leaves + leaf) * 2 * P + (r - P)] += h * acc[q];
  }
}

}  // namespace

void launch_p2m(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *M, hipStream_t s) {
  hipLaunchKernelGGL(p2m_kernel, dim3(g.n_leaves, nrhs), dim3(64), 0, s, t, g, f, M);
}
void launch_m2m(const DevTables &t, const DevTree &g, int level, int box0, int box1, int nrhs, double *M,
                hipStream_t s) {
  (void)level;
  if (box1 > box0) hipLaunchKernelGGL(m2m_kernel, dim3(box1 - box0, nrhs), dim3(64), 0, s, t, g, box0, M);
}
void launch_m2l(const DevTables &t, const DevTree &g, int nrhs, const double *M, double *L, hipStream_t s) {
  hipLaunchKernelGGL(m2l_kernel, dim3(g.n_boxes, nrhs), dim3(64), 0, s, t, g, M, L);
}
void launch_p2l(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *L, hipStream_t s) {
  hipLaunchKernelGGL(p2l_kernel, dim3(g.n_boxes, nrhs), dim3(64), 0, s, t, g, f, L);
}
void launch_l2l(const DevTables &t, const DevTree &g, int box0, int box1, int nrhs, double *L, hipStream_t s) {
  if (box1 > box0) hipLaunchKernelGGL(l2l_kernel, dim3(box1 - box0, nrhs), dim3(64), 0, s, t, g, box0, L);
}
void launch_leaf_far(const DevTables &t, const DevTree &g, int nrhs, const double *M, const double *L, double *V,
                     double *G, hipStream_t s) {
  hipLaunchKernelGGL(leaf_far_kernel, dim3(g.n_leaves, nrhs), dim3(256), 0, s, t, g, M, L, V, G);
}
void launch_near(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *V, double *G,
                 hipStream_t s) {
  hipLaunchKernelGGL(near_kernel, dim3(g.n_leaves, nrhs), dim3(256), 0, s, t, g, f, V, G);
}

}  // namespace bx
