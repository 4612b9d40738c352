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

// ------------------------------------------------------------------ P2L
// X list: b~ += h^2 * P2L_c * f_s, b~_0 += h^2 log h * 4 (W . f_s).
__global__ void __launch_bounds__(64) p2l_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                 double *__restrict__ L) {
  __shared__ double fs[256];
  const int box = g.x_boxes[blockIdx.x], rhs = blockIdx.y;
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


typedef double dbl4 __attribute__((ext_vector_type(4)));

// FP64 MFMA 16x16x4 on gfx950.  Operand layouts (one value per lane):
//   A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and accumulator
//   register r of lane l holds D[4 r + l / 16][l % 16].
__device__ inline dbl4 mfma4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ P2M
// a~ = h^2 * P2M * f, as a GEMM over 16-leaf tiles: rows Re a_k (k < KP) then
// Im a_k, K = P, one wave per tile.
template <int KPT>
__global__ void __launch_bounds__(256) p2m_mfma_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                       double *__restrict__ M) {
  constexpr int MT = 2 * KPT / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int leaf0 = (blockIdx.x * 4 + wave) * 16;
  if (leaf0 >= g.n_leaves) return;
  const int rhs = blockIdx.y, leaf = leaf0 + col, KS = t.P / 4;
  const bool ok = leaf < g.n_leaves;
  const double *fp = f + ((size_t)rhs * g.n_leaves + (ok ? leaf : 0)) * t.P + kq * KS;
  dbl4 acc[MT];
  for (int m = 0; m < MT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  for (int ks = 0; ks < KS; ++ks) {
    const double b = ok ? fp[ks] : 0.0;
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = mfma4(t.p2m_frag[((size_t)m * KS + ks) * 64 + lane], b, acc[m]);
  }
  if (!ok) return;
  const double h = box_h(g.width, g.leaf_level[leaf]), h2 = h * h;
  double *Mb = M + ((size_t)rhs * g.n_boxes + g.box_of_leaf[leaf]) * KPT * 2;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m * 16 + 4 * r + kq;          // Re rows then Im rows
      Mb[2 * (row % KPT) + row / KPT] = h2 * acc[m][r];
    }
}

// ------------------------------------------------------------------ M2L
// b~_l = sum_s (d/2)^-l [H y(s)]_l + [l = 0] sum_s a_0 (log h + log|d|),
// y_k = a~_k (-d/2)^-k, for the V list of each box.  H (KP x KP, real, the same
// for every offset) stays in registers as MFMA A fragments; the B columns are
// (source, Re/Im) pairs, 8 sources per 16 columns.  One wave per target box;
// writes (initialises) every box's local expansion.
template <int KPT>
__global__ void __launch_bounds__(256) m2l_mfma_kernel(DevTables t, DevTree g, const double *__restrict__ M,
                                                       double *__restrict__ L) {
  constexpr int MT = KPT / 16, KS = KPT / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4, part = col & 1;
  const int box = blockIdx.x * 4 + wave;
  if (box >= g.n_boxes) return;
  const int rhs = blockIdx.y;
  const double *Mr = M + (size_t)rhs * g.n_boxes * KPT * 2;
  double hA[MT][KS];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) hA[m][ks] = t.H[(size_t)(m * 16 + col) * KPT + kq * KS + ks];
  double acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[m][r] = 0.0;
  double a0 = 0.0;
  const double logh = log(box_h(g.width, g.lvl[box]));
  const int e0 = g.v_ptr[box], e1 = g.v_ptr[box + 1];
  for (int e = e0; e < e1; e += 8) {
    const int pe = e + (col >> 1);
    const bool ok = pe < e1;
    const int s = ok ? g.v_src[pe] : 0, o = ok ? g.v_cfg[pe] : 0;
    const double2 *ap = (const double2 *)(Mr + (size_t)s * KPT * 2) + kq * KS;
    const double2 *wp = (const double2 *)(t.pw_src + (size_t)o * KPT * 2) + kq * KS;
    double bv[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const double2 a = ap[ks], w = wp[ks];
      const double y = part ? a.x * w.y + a.y * w.x : a.x * w.x - a.y * w.y;
      bv[ks] = ok ? y : 0.0;
    }
    if (ok && part == 0 && kq == 0) a0 += Mr[(size_t)s * KPT * 2] * (logh + t.logd[o]);
    dbl4 c[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) c[m] = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int m = 0; m < MT; ++m) c[m] = mfma4(hA[m][ks], bv[ks], c[m]);
    const double2 *qp = (const double2 *)(t.pw_tgt + (size_t)o * KPT * 2);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double z = c[m][r], zo = __shfl_xor(z, 1);
        const double zr = part ? zo : z, zi = part ? z : zo;
        const double2 q = qp[m * 16 + 4 * r + kq];
        const double v = part ? zr * q.y + zi * q.x : zr * q.x - zi * q.y;
        acc[m][r] += ok ? v : 0.0;
      }
  }
  // sum over the 8 sources of each column group (lanes with equal kq and part)
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = acc[m][r];
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      acc[m][r] = v;
    }
  a0 += __shfl_xor(a0, 2);
  a0 += __shfl_xor(a0, 4);
  a0 += __shfl_xor(a0, 8);
  if (col < 2) {
    double *Lb = L + ((size_t)rhs * g.n_boxes + box) * KPT * 2;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int l = m * 16 + 4 * r + kq;
        Lb[2 * l + part] = acc[m][r] + (l == 0 && part == 0 ? a0 : 0.0);
      }
  }
}

// --------------------------------------------------- fused leaf evaluation
// For each 64-leaf tile, one stacked-K FP64 MFMA GEMM over its slots:
//   near tables  (K = P,    B = f of the source leaf),
//   L2T          (K = 2KP,  B = local expansion of the target / h^2),
//   W list       (K = 2KP,  B = multipole of the source box / h^2),
// rows V (P), dV/dx1 (P), dV/dx2 (P), mass (1).  Then
//   V = h^2 acc_V + (h^2 log h / 2pi) acc_mass,  grad V = h acc_D,
// which carries the per-level scaling of the unit-box tables, the a_0 log h
// of the W multipoles and the 1/h of the gradients (the tables hold the rest).
// Block = 4 waves = 64 leaves (16 per wave); the A fragments of each chunk of
// 4 k-steps are loaded once per block into LDS (double buffered, the next
// chunk prefetched into registers while the current one is multiplied).
// grid.y splits the rows into groups of MTG tiles.
constexpr int LEAF_TILE = 64;

// logical block index that gives each XCD (blocks are dealt round-robin to
// the 8 XCDs) a contiguous range of tiles; -1 for padding blocks
__device__ inline int xcd_block(int b, int nb_logical) {
  const int per = (nb_logical + 7) / 8;
  const int l = (b % 8) * per + b / 8;
  return l < nb_logical ? l : -1;
}

template <int MTG>
__global__ void __launch_bounds__(256, 2) leaf_mfma_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                           const double *__restrict__ M,
                                                           const double *__restrict__ L, double *__restrict__ V,
                                                           double *__restrict__ G, int mass_mt) {
  constexpr int NTS = MTG + 1;                 // staged row tiles: the group plus a mass tile
  constexpr int CH = NTS * 4 * 64;             // doubles per staged chunk
  constexpr int PER = (CH + 255) / 256;        // doubles each thread stages
  __shared__ double sA[2][CH];
  const int tile = xcd_block(blockIdx.x, g.n_tiles);
  if (tile < 0) return;                        // whole block: no barrier is skipped
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int rhs = blockIdx.z, mt0 = blockIdx.y * MTG, P = t.P, K2 = 2 * t.KP;
  const int MT = t.MR / 16;
  const int tgt = g.tile_tgt[tile * LEAF_TILE + wave * 16 + col];
  const double h = tgt >= 0 ? box_h(g.width, g.leaf_level[tgt]) : 1.0, inv_h2 = 1.0 / (h * h);
  const bool vrows = mt0 * 16 < P;
  const bool extra_mass = vrows && (mass_mt < mt0 || mass_mt >= mt0 + MTG);
  const int s0 = g.tile_ptr[tile], s1 = g.tile_ptr[tile + 1];
  const double *fr = f + (size_t)rhs * g.n_leaves * P;
  const double *Lr = L + (size_t)rhs * g.n_boxes * K2, *Mr = M + (size_t)rhs * g.n_boxes * K2;

  // staged tile i of a chunk: group tile mt0 + i (i < MTG), else the mass tile
  auto stage_load = [&](int sl, int ks0, double *reg) {
    const int K = g.slot_type[sl] == 0 ? P : K2, KS = K / 4;
    const double *A = t.leaf_frag + g.slot_aoff[sl];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * 256;
      double v = 0.0;
      if (idx < CH) {
        const int i = idx / 256, j = (idx / 64) & 3, ln = idx & 63;
        const int mt = i < MTG ? mt0 + i : mass_mt;
        if (mt < MT && (i < MTG || extra_mass)) v = A[((size_t)mt * KS + ks0 + j) * 64 + ln];
      }
      reg[q] = v;
    }
  };
  auto stage_store = [&](int buf, const double *reg) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * 256;
      if (idx < CH) sA[buf][idx] = reg[q];
    }
  };

  dbl4 acc[NTS];
#pragma unroll
  for (int m = 0; m < NTS; ++m) acc[m] = dbl4{0, 0, 0, 0};
  double reg[PER];
  int sl = s0, ks0 = 0, buf = 0;
  if (sl < s1) stage_load(sl, 0, reg);
  while (sl < s1) {
    const int type = g.slot_type[sl], src = g.slot_src[sl * LEAF_TILE + wave * 16 + col];
    const int K = type == 0 ? P : K2, KS = K / 4;
    stage_store(buf, reg);
    __syncthreads();
    // prefetch the next chunk (this slot's next 4 k-steps, or the next slot's first)
    int nsl = sl, nks = ks0 + 4;
    if (nks >= KS) { ++nsl; nks = 0; }
    if (nsl < s1) stage_load(nsl, nks, reg);
    const double *bp = type == 0 ? fr + (size_t)(src >= 0 ? src : 0) * P
                                 : (type == 1 ? Lr : Mr) + (size_t)(src >= 0 ? src : 0) * K2;
    const double sc = src < 0 ? 0.0 : (type == 0 ? 1.0 : inv_h2);
    double bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = sc * bp[kq * KS + ks0 + j];
    const double *S = sA[buf];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = 0; m < NTS; ++m)
        if (m < MTG || extra_mass) acc[m] = mfma4(S[(m * 4 + j) * 64 + lane], bv[j], acc[m]);
    sl = nsl;
    ks0 = nks;
    buf ^= 1;
  }
  double mass = 0.0;
  if (vrows) {
    double mv = acc[MTG][0];
#pragma unroll
    for (int m = 0; m < MTG; ++m)
      if (mt0 + m == mass_mt) mv = acc[m][0];
    mass = __shfl(mv, col);                              // row 0 of the mass tile lives in lanes 0..15
  }
  if (tgt < 0) return;
  const double lg = h * h * log(h) * kInv2Pi * mass;
  double *Vt = V + ((size_t)rhs * g.n_leaves + tgt) * P;
  double *Gt = G + ((size_t)rhs * g.n_leaves + tgt) * 2 * P;
#pragma unroll
  for (int m = 0; m < MTG; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = (mt0 + m) * 16 + 4 * r + kq;
      if (row < P) Vt[row] = h * h * acc[m][r] + lg;
      else if (row < 3 * P) Gt[row - P] = h * acc[m][r];
    }
}

}  // namespace

void launch_p2m(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *M, hipStream_t s) {
  dim3 grid((g.n_leaves + 63) / 64, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(p2m_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, f, M);
  else if (t.KP == 32) hipLaunchKernelGGL(p2m_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, f, M);
  else hipLaunchKernelGGL(p2m_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, f, M);
}
void launch_m2m(const DevTables &t, const DevTree &g, int level, int box0, int box1, int nrhs, double *M,
                hipStream_t s) {
  (void)level;
  if (box1 > box0) hipLaunchKernelGGL(m2m_kernel, dim3(box1 - box0, nrhs), dim3(64), 0, s, t, g, box0, M);
}
void launch_m2l(const DevTables &t, const DevTree &g, int nrhs, const double *M, double *L, hipStream_t s) {
  dim3 grid((g.n_boxes + 3) / 4, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(m2l_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, M, L);
  else if (t.KP == 32) hipLaunchKernelGGL(m2l_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, M, L);
  else hipLaunchKernelGGL(m2l_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, M, L);
}
void launch_p2l(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *L, hipStream_t s) {
  if (g.n_x_boxes > 0) hipLaunchKernelGGL(p2l_kernel, dim3(g.n_x_boxes, nrhs), dim3(64), 0, s, t, g, f, L);
}
void launch_l2l(const DevTables &t, const DevTree &g, int box0, int box1, int nrhs, double *L, hipStream_t s) {
  if (box1 > box0) hipLaunchKernelGGL(l2l_kernel, dim3(box1 - box0, nrhs), dim3(64), 0, s, t, g, box0, L);
}
void launch_leaf(const DevTables &t, const DevTree &g, const double *f, int nrhs, const double *M,
                 const double *L, double *V, double *G, hipStream_t s) {
  const int mass_mt = 3 * t.P / 16;
  const int bx = (g.n_tiles + 7) / 8 * 8;     // padded to a multiple of the 8 XCDs
  if (t.n == 4) {
    hipLaunchKernelGGL(leaf_mfma_kernel<4>, dim3(bx, 1, nrhs), dim3(256), 0, s, t, g, f, M, L, V, G, mass_mt);
  } else if (t.n == 8) {
    hipLaunchKernelGGL(leaf_mfma_kernel<13>, dim3(bx, 1, nrhs), dim3(256), 0, s, t, g, f, M, L, V, G, mass_mt);
  } else {
    hipLaunchKernelGGL(leaf_mfma_kernel<16>, dim3(bx, 3, nrhs), dim3(256), 0, s, t, g, f, M, L, V, G, mass_mt);
  }
}

}  // namespace bx
