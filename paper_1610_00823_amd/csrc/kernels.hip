// Device kernels of the box code (gfx950).
//
// Expansions are stored per box as KP complex coefficients (re, im
// interleaved), scaled by powers of the box width h: multipole a~_k = a_k / h^k,
// local b~_l = b_l h^l.  With this scaling every translation operator is the
// same at every level; only a_0 log h terms and the 1/h of gradients carry the
// level, and they are applied here in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace bx {
namespace {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr int NOFF_DEV = 49;   // 7 x 7 same-level offsets (the V-list classes among them)

__device__ inline double box_h(double width, int level) { return ldexp(width, -level); }

typedef double dbl4 __attribute__((ext_vector_type(4)));

// FP64 MFMA 16x16x4 on gfx950.  Operand layouts (one value per lane):
//   A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, and accumulator
//   register r of lane l holds D[4 r + l / 16][l % 16].
__device__ inline dbl4 mfma4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}


// ------------------------------------------------- M2M, L2L and P2L GEMMs
// Complex operators act on interleaved (Re, Im) coefficient vectors as real
// matrices; 16 boxes per wave, A fragments streamed from the operator table
// (k split as k = (lane / 16) * KS + ks so that each lane's B run is contiguous).

// M2M for the internal boxes of one level, 16 parents per block: wave c
// applies the operator of child position c (2KP x 2KP, on interleaved
// coefficients) to the children at c, and the four partial results are summed
// in LDS in a fixed order.
template <int KPT>
__global__ void __launch_bounds__(256) m2m_mfma_kernel(DevTables t, DevTree g, const int *__restrict__ boxes,
                                                       int nbox, int child_base, double *__restrict__ M) {
  // child_base >= 0: the children of the i-th box of the list are boxes
  // child_base + 4 i .. + 3 (level-major Morton order), so their multipoles
  // are requested without waiting for the box index
  constexpr int R = 2 * KPT, MT = R / 16, KS = R / 4;
  __shared__ double part[4][16][R + 1];
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int i = blockIdx.x * 16 + col, rhs = blockIdx.y;
  const bool ok = i < nbox;
  double *Mr = M + (size_t)rhs * g.n_boxes * R;
  const int c0 = !ok ? 0 : (child_base >= 0 ? child_base + 4 * i : g.child0[boxes[i]]);
  const double *bp = Mr + (size_t)(c0 + c) * R + kq * KS;
  const double *A = t.m2m_frag + (size_t)c * MT * KS * 64;
  dbl4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  if constexpr (KPT <= 32) {
    // every operand requested at once: one memory round trip per level
    double bv[KS], av[MT][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bv[ks] = bp[ks];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[m][ks] = A[((size_t)m * KS + ks) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = mfma4(av[m][ks], ok ? bv[ks] : 0.0, acc[m]);
  } else {
    for (int ks = 0; ks < KS; ks += 4) {
      double bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = bp[ks + j];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = mfma4(A[((size_t)m * KS + ks + j) * 64 + lane], ok ? bv[j] : 0.0, acc[m]);
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[c][col][m * 16 + 4 * r + kq] = acc[m][r];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * R; e += 256) {
    const int cc = e / R, row = e % R, ii = blockIdx.x * 16 + cc;
    if (ii < nbox)
      Mr[(size_t)boxes[ii] * R + row] = ((part[0][cc][row] + part[1][cc][row]) + part[2][cc][row]) + part[3][cc][row];
  }
}

// L2L from the internal boxes of one level to their children at position
// c = blockIdx.z: A = L2L_c (2KP x 2KP), B = the parent's local expansion; wave
// w computes row tile w (of MT), so each wave's chain is short.  The result is
// added to the child's local expansion.
// Two levels in one launch, for levels too small to fill the chip (one
// launch each would be latency-bound).  A block takes 4 boxes G of the top
// level and their 16 children Q (column j = 4 g + q).
//   M2M: M(Q) = sum_c M2M_c M(child c of Q) for internal Q (stage 1, wave =
//   c, all 16 columns), then M(G) = sum_q M2M_q M(Q_q) (stage 2, wave = q,
//   columns 0..3); leaf children keep their P2M multipoles.
//   L2L: L(Q) += L2L_q L(G) (stage 1, wave = q, columns 0..3), then
//   L(child c of Q) += L2L_c L(Q) for internal Q (stage 2, wave = c).
// Both stages stage their 16 (or 4) columns through LDS.
template <int KPT>
__device__ inline void gemm_cols(const double *A, const double *bcol, bool ok, int lane, int kq, dbl4 *acc) {
  // acc[m] = A (MT row tiles of the 2 KP x 2 KP operator) times this lane's
  // column; up to KP = 32 every operand is requested before the first product
  constexpr int R = 2 * KPT, MT = R / 16, KS = R / 4;
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  if constexpr (KPT <= 32) {
    double bv[KS], av[MT][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bv[ks] = ok ? bcol[kq * KS + ks] : 0.0;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[m][ks] = A[((size_t)m * KS + ks) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = mfma4(av[m][ks], bv[ks], acc[m]);
  } else {
    for (int ks = 0; ks < KS; ks += 4) {
      double bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = ok ? bcol[kq * KS + ks + j] : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = mfma4(A[((size_t)m * KS + ks + j) * 64 + lane], bv[j], acc[m]);
    }
  }
}

template <int KPT>
__global__ void __launch_bounds__(256) m2m2_mfma_kernel(DevTables t, DevTree g, const int *__restrict__ boxes,
                                                        int nbox, double *__restrict__ M) {
  constexpr int R = 2 * KPT, MT = R / 16, RP = R + 1;
  __shared__ double part[4][16][RP];
  __shared__ double sQ[16][RP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int rhs = blockIdx.y;
  double *Mr = M + (size_t)rhs * g.n_boxes * R;
  // stage 1: column col = child Q (4 g + q) of top box g of this block
  const int gi = blockIdx.x * 4 + (col >> 2);
  const bool gok = gi < nbox;
  const int Q = gok ? g.child0[boxes[gi]] + (col & 3) : 0;
  const bool qint = gok && g.child0[Q] >= 0;
  dbl4 acc[MT];
  gemm_cols<KPT>(t.m2m_frag + (size_t)w * MT * (R / 4) * 64, Mr + (size_t)(qint ? g.child0[Q] + w : 0) * R, qint,
                 lane, kq, acc);
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[w][col][m * 16 + 4 * r + kq] = acc[m][r];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * R; e += 256) {
    const int cc = e / R, row = e % R, gg = blockIdx.x * 4 + (cc >> 2);
    if (gg >= nbox) continue;
    const int q = g.child0[boxes[gg]] + (cc & 3);
    if (g.child0[q] >= 0) {
      const double v = ((part[0][cc][row] + part[1][cc][row]) + part[2][cc][row]) + part[3][cc][row];
      sQ[cc][row] = v;
      Mr[(size_t)q * R + row] = v;
    } else {
      sQ[cc][row] = Mr[(size_t)q * R + row];     // a leaf: its P2M multipole
    }
  }
  __syncthreads();
  // stage 2: column col < 4 = top box col, wave = child position q
  const int g2 = blockIdx.x * 4 + col;
  const bool ok2 = col < 4 && g2 < nbox;
  gemm_cols<KPT>(t.m2m_frag + (size_t)w * MT * (R / 4) * 64, &sQ[ok2 ? col * 4 + w : 0][0], ok2, lane, kq, acc);
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[w][col][m * 16 + 4 * r + kq] = acc[m][r];
  __syncthreads();
  for (int e = threadIdx.x; e < 4 * R; e += 256) {
    const int cc = e / R, row = e % R, gg = blockIdx.x * 4 + cc;
    if (gg < nbox)
      Mr[(size_t)boxes[gg] * R + row] = ((part[0][cc][row] + part[1][cc][row]) + part[2][cc][row]) + part[3][cc][row];
  }
}

template <int KPT>
__global__ void __launch_bounds__(256) l2l2_mfma_kernel(DevTables t, DevTree g, const int *__restrict__ boxes,
                                                        int nbox, double *__restrict__ L) {
  constexpr int R = 2 * KPT, MT = R / 16, RP = R + 1;
  __shared__ double sQ[16][RP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int rhs = blockIdx.y;
  double *Lr = L + (size_t)rhs * g.n_boxes * R;
  // stage 1: column col < 4 = top box G, wave = child position q: L(Q) += L2L_q L(G)
  const int g1 = blockIdx.x * 4 + col;
  const bool ok1 = col < 4 && g1 < nbox;
  const int G = ok1 ? boxes[g1] : 0;
  const int Q1 = ok1 ? g.child0[G] + w : 0;
  double old[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) old[m][r] = Lr[(size_t)Q1 * R + m * 16 + 4 * r + kq];
  dbl4 acc[MT];
  gemm_cols<KPT>(t.l2l_frag + (size_t)w * MT * (R / 4) * 64, Lr + (size_t)G * R, ok1, lane, kq, acc);
  if (ok1)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = old[m][r] + acc[m][r];
        sQ[col * 4 + w][m * 16 + 4 * r + kq] = v;
        Lr[(size_t)Q1 * R + m * 16 + 4 * r + kq] = v;
      }
  __syncthreads();
  // stage 2: column col = child Q (4 g + q), wave = grandchild position c
  const int gi = blockIdx.x * 4 + (col >> 2);
  const bool gok = gi < nbox;
  const int Q = gok ? g.child0[boxes[gi]] + (col & 3) : 0;
  const bool qint = gok && g.child0[Q] >= 0;
  const int C = qint ? g.child0[Q] + w : 0;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) old[m][r] = Lr[(size_t)C * R + m * 16 + 4 * r + kq];
  gemm_cols<KPT>(t.l2l_frag + (size_t)w * MT * (R / 4) * 64, &sQ[col][0], qint, lane, kq, acc);
  if (qint)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) Lr[(size_t)C * R + m * 16 + 4 * r + kq] = old[m][r] + acc[m][r];
}

template <int KPT, bool WIDE>
__global__ void __launch_bounds__(256) l2l_mfma_kernel(DevTables t, DevTree g, const int *__restrict__ boxes,
                                                       int nbox, double *__restrict__ L) {
  // Each wave computes row tiles of one child position c for 16 parents: all
  // of them (c = wave) or, for levels with few boxes (WIDE: four times the
  // blocks), tiles wave, wave + 4, ... (c = blockIdx.z).  The parent's
  // expansion, the operator fragments and the child's current expansion are
  // all requested before the products, so a level costs one memory round trip.
  constexpr int R = 2 * KPT, MT = R / 16, KS = R / 4, NT = WIDE ? (MT + 3) / 4 : MT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int c = WIDE ? blockIdx.z : wave;
  const int i = blockIdx.x * 16 + col, rhs = blockIdx.y;
  const bool ok = i < nbox;
  const int box = ok ? boxes[i] : 0;
  double *Lr = L + (size_t)rhs * g.n_boxes * R;
  const double *bp = Lr + (size_t)box * R + kq * KS;
  double *Lc = Lr + (size_t)(ok ? g.child0[box] + c : 0) * R;
  const double *A = t.l2l_frag + (size_t)c * MT * KS * 64;
  int tm[NT];                                     // row tile of slot m (MT when there is none)
#pragma unroll
  for (int m = 0; m < NT; ++m) tm[m] = WIDE ? (wave + 4 * m < MT ? wave + 4 * m : MT) : m;
  dbl4 acc[NT];
#pragma unroll
  for (int m = 0; m < NT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  double old[NT][4];
#pragma unroll
  for (int m = 0; m < NT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) old[m][r] = Lc[(tm[m] < MT ? tm[m] : 0) * 16 + 4 * r + kq];
  if constexpr (KPT <= 32) {
    double bv[KS], av[NT][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bv[ks] = bp[ks];
#pragma unroll
    for (int m = 0; m < NT; ++m)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[m][ks] = A[((size_t)(tm[m] < MT ? tm[m] : 0) * KS + ks) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int m = 0; m < NT; ++m) acc[m] = mfma4(av[m][ks], ok ? bv[ks] : 0.0, acc[m]);
  } else {
    for (int ks = 0; ks < KS; ks += 4) {
      double bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = bp[ks + j];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < NT; ++m)
          acc[m] = mfma4(A[((size_t)(tm[m] < MT ? tm[m] : 0) * KS + ks + j) * 64 + lane], ok ? bv[j] : 0.0, acc[m]);
    }
  }
  if (ok)
#pragma unroll
    for (int m = 0; m < NT; ++m)
      if (tm[m] < MT)
#pragma unroll
        for (int r = 0; r < 4; ++r) Lc[tm[m] * 16 + 4 * r + kq] = old[m][r] + acc[m][r];
}

// X list: b~ += h^2 P2L_c f_s, b~_0 += h^2 log h (4 W . f_s), over 16-box tiles
// whose slots are the union of their X configurations (rows: 2KP interleaved
// coefficients, then the mass row).
template <int KPT>
__global__ void __launch_bounds__(256) p2l_mfma_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                       double *__restrict__ L) {
  constexpr int R = 2 * KPT, MT = (R + 16) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= g.n_xtiles) return;
  const int rhs = blockIdx.y, P = t.P, KS = P / 4;
  const int box = g.xtile_box[tile * 16 + col];
  const double *fr = f + (size_t)rhs * g.n_leaves * P;
  dbl4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  for (int sl = g.xtile_ptr[tile]; sl < g.xtile_ptr[tile + 1]; ++sl) {
    const int src = g.xslot_src[sl * 16 + col];
    const double *A = t.p2l_frag + (size_t)g.xslot_cfg[sl] * MT * KS * 64;
    const double *bp = fr + (size_t)(src >= 0 ? src : 0) * P + kq * KS;
    for (int ks = 0; ks < KS; ks += 4) {
      double bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = src >= 0 ? bp[ks + j] : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = mfma4(A[((size_t)m * KS + ks + j) * 64 + lane], bv[j], acc[m]);
    }
  }
  const double mass = __shfl(acc[R / 16][0], col);    // mass row R: tile R/16, register 0, lanes 0..15
  if (box < 0) return;
  const double h = box_h(g.width, g.lvl[box]), h2 = h * h;
  double *Lb = L + ((size_t)rhs * g.n_boxes + box) * R;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m * 16 + 4 * r + kq;
      if (row < R) Lb[row] += h2 * acc[m][r] + (row == 0 ? h2 * log(h) * mass : 0.0);
    }
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
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  const double *A = t.p2m_frag;
  for (int k0 = 0; k0 < KS; k0 += 4) {                  // KS = P/4 is a multiple of 4
    double bv[4], av[MT][4];                           // 4 k-steps of operands requested at once
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = fp[k0 + j];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) av[m][j] = A[((size_t)m * KS + k0 + j) * 64 + lane];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = mfma4(av[m][j], ok ? bv[j] : 0.0, acc[m]);
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
// for every offset) is the MFMA A operand; the B columns are (source, Re/Im)
// pairs, 8 sources per 16 columns.  The V lists of the four children of an
// internal box P (one wave each) all come from the 6 x 6 grid of boxes below
// P's neighbourhood, whose multipoles are staged in LDS (rows padded so that
// the 8 sources of a column group hit distinct banks).  Each block keeps H and
// the power table of the 49 offsets in LDS (the target powers (d/2)^-l are
// (-1)^l times the source powers), which leaves room for three blocks per CU,
// and works through a contiguous range of parents, with the next parent's grid
// and V entries requested while the current one is multiplied.  Writes
// (initialises) every box's local expansion; the last block writes the roots'
// zero expansions.
constexpr int M2L_BLOCKS = 1024;

template <int KPT>
__global__ void __launch_bounds__(256, KPT <= 32 ? 3 : 1) m2l_mfma_kernel(DevTables t, DevTree g,
                                                                               const double *__restrict__ M,
                                                                               double *__restrict__ L, int per_block) {
  constexpr int MT = KPT / 16, KS = KPT / 4;
  constexpr int PWS = KPT + 1;                 // padded rows: 8 offsets / sources per column group, distinct banks
  constexpr int GPT = (36 * KPT + 255) / 256;  // grid coefficients per thread
  __shared__ double2 spw[NOFF_DEV * PWS];     // (-d/2)^-k; the target powers (d/2)^-l are (-1)^l times these
  __shared__ double sH[KPT * (KPT + 1)];      // the core, rows padded
  __shared__ double2 sM[36 * PWS];
  __shared__ double slogd[NOFF_DEV];
  const int rhs = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, kq = lane >> 4, part = col & 1;
  const int nblk = gridDim.x - 1;
  if ((int)blockIdx.x == nblk) {               // the roots (level-0 boxes first) have no V list
    double *Lb = L + (size_t)rhs * g.n_boxes * KPT * 2;
    for (int i = threadIdx.x; i < 2 * KPT * g.n_roots; i += 256) Lb[i] = 0.0;
    return;
  }
  const int p0 = blockIdx.x * per_block;
  const int p1 = p0 + per_block < g.n_m2l_par ? p0 + per_block : g.n_m2l_par;
  if (p0 >= p1) return;                        // whole block: no barrier is skipped
  const double *Mr = M + (size_t)rhs * g.n_boxes * KPT * 2;
  for (int i = threadIdx.x; i < NOFF_DEV * KPT; i += 256) {
    spw[i / KPT * PWS + i % KPT] = ((const double2 *)t.pw_src)[i];
  }
  if (threadIdx.x < NOFF_DEV) slogd[threadIdx.x] = t.logd[threadIdx.x];
  for (int i = threadIdx.x; i < KPT * KPT; i += 256) sH[i / KPT * (KPT + 1) + i % KPT] = t.H[i];
  // this thread's share of a parent's grid: coefficient i = threadIdx.x + 256 j;
  // this lane's V entries (iteration it: entry 8 it + col/2 of its wave's
  // child) and the parent's first child and level, all requested one parent
  // ahead so that no load waits inside the source loop
  double2 gm[GPT];
  int en[4];
  int2 inf;
  auto grid_load = [&](int pp) {
    const int *grid = g.m2l_grid + (size_t)pp * 36;
    const int *ep = g.m2l_ent + ((size_t)pp * 4 + wave) * M2L_VMAX + (col >> 1);
#pragma unroll
    for (int it = 0; it < 4; ++it) en[it] = ep[8 * it];
    inf = ((const int2 *)g.m2l_info)[pp];
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
      const int i = threadIdx.x + 256 * j, sl = i < 36 * KPT ? i / KPT : 0;
      const int gb = grid[sl];
      gm[j] = ((const double2 *)(Mr + (size_t)(gb >= 0 ? gb : 0) * KPT * 2))[i % KPT];
      if (gb < 0 || i >= 36 * KPT) gm[j] = double2{0, 0};
    }
  };
  grid_load(p0);
  for (int pp = p0; pp < p1; ++pp) {
    __syncthreads();                           // the previous parent's grid is no longer read
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < 36 * KPT) sM[i / KPT * PWS + i % KPT] = gm[j];
    }
    int ent[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) ent[it] = en[it];
    const int box = inf.x + wave;
    const double logh = log(box_h(g.width, inf.y));
    __syncthreads();
    if (pp + 1 < p1) grid_load(pp + 1);        // in flight during this parent's products
    double acc[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][r] = 0.0;
    double a0 = 0.0;
    // one group of 8 V entries (dead lanes and dead groups add zeros)
    auto group = [&](int it) {
      const bool ok = ent[it] >= 0;
      const int s_c = ok ? ent[it] & 255 : 0, o_c = ok ? ent[it] >> 8 : 0;
      double bv[KS];
      const double2 *ap = &sM[s_c * PWS + kq * KS];
      const double2 *wp = &spw[o_c * PWS + kq * KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const double2 a = ap[ks], w = wp[ks];
        const double y = part ? a.x * w.y + a.y * w.x : a.x * w.x - a.y * w.y;
        bv[ks] = ok ? y : 0.0;
      }
      a0 += (ok && part == 0 && kq == 0) ? ap[0].x * (logh + slogd[o_c]) : 0.0;
      dbl4 c[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) c[m] = dbl4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int m = 0; m < MT; ++m) c[m] = mfma4(sH[(m * 16 + col) * (KPT + 1) + kq * KS + ks], bv[ks], c[m]);
      const double2 *qp = &spw[o_c * PWS];
      const double sg = (kq & 1) ? -1.0 : 1.0;     // (-1)^l, l = m 16 + 4 r + kq
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double z = c[m][r], zo = __shfl_xor(z, 1);
          const double zr = part ? zo : z, zi = part ? z : zo;
          const double2 q = qp[m * 16 + 4 * r + kq];
          const double v = part ? zr * q.y + zi * q.x : zr * q.x - zi * q.y;
          acc[m][r] += ok ? sg * v : 0.0;
        }
    };
    // entries are packed from the front: group it is live when its first entry is
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      if (__builtin_amdgcn_readfirstlane(ent[it]) < 0) break;
      group(it);
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
}

// --------------------------------------------------- fused leaf evaluation
// For each 64-leaf tile, one stacked-K FP64 MFMA GEMM over its slots:
//   near tables  (K = P,    B = f of the source leaf),
//   L2T          (K = 2KP,  B = local expansion of the target / h^2),
//   W list       (K = 2KP,  B = multipole of the source box / h^2),
// rows V (P), dV/dx1 (P), dV/dx2 (P); with mass = sum over slots of the
// operators' mass weights times B,
//   V = h^2 acc_V + (h^2 log h / 2pi) mass,  grad V = h acc_D,
// which carries the per-level scaling of the unit-box tables, the a_0 log h
// of the W multipoles and the 1/h of the gradients (the tables hold the rest).
// Block = 4 waves = 64 leaves.  The slot's B columns (64 x KC) are staged in
// LDS once per block (double buffered through registers, one barrier per
// chunk); wave w owns row tiles w, w+4, w+8, ... of its row group and all four
// 16-leaf column tiles, so each A fragment read from the operator table feeds
// four MFMAs.  Each block runs one work unit (tile, first row tile, row tiles
// per wave): heavy tiles are split by rows over several blocks, and the host
// orders the units so that each XCD gets a contiguous range, longest first.
constexpr int LEAF_TILE = 64;
#ifndef LEAF_PF
#define LEAF_PF 2   // k-steps of A fragments in flight in the FP64 leaf GEMM
#endif

template <int N>
struct Regs {
  double v[N];
};

// This thread's quarter (KC/4 values) of column scol of chunk c of slot sl
// (slot_src already offset to the column).
template <int KC>
__device__ __forceinline__ Regs<KC / 4> leaf_chunk_load(const int *__restrict__ slot_type,
                                                         const int *__restrict__ slot_src, const double *fr,
                                                         const double *Lr, const double *Mr, int sl, int c, int P,
                                                         int K2, int sq, double sinv_h2) {
  constexpr int PERT = KC / 4;
  const int type = slot_type[sl], src = slot_src[sl * LEAF_TILE];
  const double *bp = type == 0 ? fr + (size_t)(src >= 0 ? src : 0) * P
                               : (type == 1 ? Lr : Mr) + (size_t)(src >= 0 ? src : 0) * K2;
  const double sc = src < 0 ? 0.0 : (type == 0 ? 1.0 : sinv_h2);
  const double *q = bp + c * KC + sq * PERT;
  Regs<PERT> r;
#pragma unroll
  for (int j = 0; j < PERT; ++j) r.v[j] = sc * q[j];
  return r;
}

template <int TPW, int KC>
__global__ void __launch_bounds__(256, 2) leaf_mfma_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                           const double *__restrict__ M,
                                                           const double *__restrict__ L, double *__restrict__ V,
                                                           double *__restrict__ G, int accumulate) {
  constexpr int KSC = KC / 4, PERT = KC / 4, SB = KC + 1;
  __shared__ double sB[2][LEAF_TILE * SB];
  __shared__ double sMass[LEAF_TILE];
  const int tile = g.unit_tile[blockIdx.x];
  if (tile < 0) return;                        // whole block: no barrier is skipped
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), col = lane & 15,
            kq = lane >> 4;
  const int rhs = blockIdx.z, P = t.P, K2 = 2 * t.KP, MTR = 3 * P / 16;
  const int mtg = g.unit_mt[blockIdx.x] & 0xffff;   // first row tile of this unit
  const int ni = g.unit_mt[blockIdx.x] >> 16;       // row tiles per wave (<= TPW)
  // row tile of fragment i: i < ni computes; the others reread tile 0 (always in
  // the table) and feed no MFMA
  int ir[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) ir[i] = i < ni ? i : 0;
  const int s0 = g.tile_ptr[tile], s1 = g.tile_ptr[tile + 1];
  const double *fr = f + (size_t)rhs * g.n_leaves * P;
  const double *Lr = L + (size_t)rhs * g.n_boxes * K2, *Mr = M + (size_t)rhs * g.n_boxes * K2;
  const int *slot_type = g.slot_type, *slot_op = g.slot_op, *slot_aoff = g.slot_aoff;
  const double *leaf_frag = t.leaf_frag, *leaf_mass = t.leaf_mass;
  const int kmax = t.leaf_kmax;

  // staging role: 4 threads per column, each a quarter (PERT values) of the chunk
  const int scol = threadIdx.x >> 2, sq = threadIdx.x & 3;
  const int stgt = g.tile_tgt[tile * LEAF_TILE + scol];
  const double sinv_h2 = stgt >= 0 ? 1.0 / (box_h(g.width, g.leaf_level[stgt]) * box_h(g.width, g.leaf_level[stgt]))
                                   : 0.0;
  const int *slot_src = g.slot_src + scol;
  dbl4 acc[TPW][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[i][nt] = dbl4{0, 0, 0, 0};
  double mpart = 0.0;
  const int MTP = (MTR + 3) / 4 * 4;                // row tiles in the (padded) operator tables
  // A fragment of row tile i, k-step ks of chunk c of slot sl (every index valid:
  // the tables are padded to whole groups of row tiles)
  auto a_ptr = [&](int sl_, int c_) -> const double * {
    const int NC_ = (slot_type[sl_] == 0 ? P : K2) / KC;
    return leaf_frag + slot_aoff[sl_] + ((size_t)(mtg + wave) * NC_ + c_) * KSC * 64 + lane;
  };
  auto a_stride = [&](int sl_) -> size_t {          // from row tile i to i + 1 (4 tiles apart)
    const int NC_ = (slot_type[sl_] == 0 ? P : K2) / KC;
    return (size_t)4 * NC_ * KSC * 64;
  };
  (void)MTP;
  // A fragments run LEAF_PF k-steps ahead of the MFMAs (ring an[ks % LEAF_PF]);
  // the next chunk's B columns are requested right after this chunk's barrier,
  // so both latencies are covered by LEAF_PF k-steps of MFMA work.
  constexpr int D = LEAF_PF < KSC ? LEAF_PF : KSC;
  static_assert(KSC % D == 0, "prefetch depth must divide the chunk's k-steps");
  Regs<PERT> rb;
  double an[D][TPW];
  int sl = s0, c = 0, buf = 0;
  if (sl < s1) {
    const double *A0 = a_ptr(sl, 0);
    const size_t st0 = a_stride(sl);
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int i = 0; i < TPW; ++i) an[j][i] = A0[ir[i] * st0 + j * 64];
    rb = leaf_chunk_load<KC>(slot_type, slot_src, fr, Lr, Mr, sl, 0, P, K2, sq, sinv_h2);
  }
  while (sl < s1) {
    const int K = slot_type[sl] == 0 ? P : K2, NC = K / KC;
    {   // stage this chunk's B columns and add their mass weights
      const double *mw = leaf_mass + (size_t)slot_op[sl] * kmax + c * KC + sq * PERT;
      double *dst = &sB[buf][scol * SB + sq * PERT];
#pragma unroll
      for (int j = 0; j < PERT; ++j) {
        dst[j] = rb.v[j];
        mpart = fma(mw[j], rb.v[j], mpart);
      }
    }
    __syncthreads();
    int nsl = sl, nc = c + 1;
    if (nc >= NC) { ++nsl; nc = 0; }
    const bool more = nsl < s1;
    const double *Ac = a_ptr(sl, c);
    const size_t stc = a_stride(sl);
    const double *An = more ? a_ptr(nsl, nc) : Ac;
    const size_t stn = more ? a_stride(nsl) : stc;
    if (more) rb = leaf_chunk_load<KC>(slot_type, slot_src, fr, Lr, Mr, nsl, nc, P, K2, sq, sinv_h2);
    const double *S = sB[buf];
#pragma unroll
    for (int ks = 0; ks < KSC; ++ks) {
      double a[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) a[i] = an[ks % D][i];
      if (ks + D < KSC) {
#pragma unroll
        for (int i = 0; i < TPW; ++i) an[ks % D][i] = Ac[ir[i] * stc + (ks + D) * 64];
      } else if (more) {
#pragma unroll
        for (int i = 0; i < TPW; ++i) an[ks % D][i] = An[ir[i] * stn + (ks + D - KSC) * 64];
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const double b = S[(nt * 16 + col) * SB + kq * KSC + ks];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          if (i < ni) acc[i][nt] = mfma4(a[i], b, acc[i][nt]);
      }
    }
    sl = nsl;
    c = nc;
    buf ^= 1;
  }
  // mass of each column: sum over its 4 staging threads (adjacent lanes)
  mpart += __shfl_xor(mpart, 1);
  mpart += __shfl_xor(mpart, 2);
  if (sq == 0) sMass[scol] = mpart;
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int tgt = g.tile_tgt[tile * LEAF_TILE + nt * 16 + col];
    if (tgt < 0) continue;
    const double h = box_h(g.width, g.leaf_level[tgt]);
    const double lg = h * h * log(h) * kInv2Pi * sMass[nt * 16 + col];
    double *Vt = V + ((size_t)rhs * g.n_leaves + tgt) * P;
    double *Gt = G + ((size_t)rhs * g.n_leaves + tgt) * 2 * P;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int mt = mtg + wave + 4 * i;
      if (i >= ni || mt >= MTR) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + 4 * kq + r;        // the A rows of each tile are permuted to match
        if (row < P) Vt[row] = (accumulate ? Vt[row] : 0.0) + (h * h * acc[i][nt][r] + lg);
        else Gt[row - P] = (accumulate ? Gt[row - P] : 0.0) + h * acc[i][nt][r];
      }
    }
  }
}


// ------------------------------------------- split-precision near field
// The near-table products T f run on exact int8 slices.  A table row r is
// scaled by 2^E_r and the samples of one right-hand side by 2^Ef (max |f| <
// 2^Ef 127.5/128), each cut into integer slices of 7 bits (rounded to nearest):
//   T = 2^E_r sum_a t_a 2^-7(a+1),   f = 2^Ef sum_b s_b 2^-7(b+1).
// The products of slice group d = a + b all carry the scale 2^(E_r+Ef-7(d+2)),
// so v_mfma_i32_16x16x64_i8 sums them exactly in int32 (|t_a s_b| <= 127^2, 64
// terms per instruction, at most 6 pairs per group and 48 slots per tile stay
// below 2^31) across every slot of a tile; groups with a + b >= S are dropped.
// FP64 is used only to scale and add the S group sums of each output.
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ inline i32x4 mfma_i8(i32x4 a, i32x4 b, i32x4 c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

constexpr int NEAR_SG = 6;      // slice groups of the int8 kernel (tiles needing more stay FP64)
constexpr int NEAR_SMAX = 8;    // table slices stored
constexpr int FMAX_BLOCKS = 512;

// max |f| per right-hand side: block partial maxima
__global__ void __launch_bounds__(256) fmax_partial_kernel(const double *__restrict__ f, size_t count,
                                                           double *__restrict__ part) {
  const int rhs = blockIdx.y;
  const double *fr = f + (size_t)rhs * count;
  double m = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
    m = fmax(m, fabs(fr[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)rhs * gridDim.x + blockIdx.x] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}

// Sample scale, int8 slices fsl[rhs][b][leaf][k] (b < Sf) and per-leaf masses
// sum_k wq_k f_k.  Block = 256 threads = 256 / P leaves (P = 64) or one leaf
// (P = 256); every block reduces the partial maxima itself.
__global__ void __launch_bounds__(256) split_prep_kernel(const double *__restrict__ f, const double *__restrict__ wq,
                                                         int P, int n_leaves, const double *__restrict__ part,
                                                         int nparts, int Sf, double *__restrict__ fscale,
                                                         int8_t *__restrict__ fsl, double *__restrict__ lmass) {
  const int rhs = blockIdx.y, tid = threadIdx.x;
  const int lpb = P >= 256 ? 1 : 256 / P;
  const int leaf = blockIdx.x * lpb + tid / P, k = tid % P;
  const bool ok = leaf < n_leaves && tid < lpb * P;
  // this thread's sample and weight, requested together with the partial maxima
  const double x = ok ? f[((size_t)rhs * n_leaves + leaf) * P + k] : 0.0, wk = ok ? wq[k] : 0.0;
  __shared__ double sm[4];
  double m = 0.0;
  for (int i = tid; i < nparts; i += 256) m = fmax(m, part[(size_t)rhs * nparts + i]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((tid & 63) == 0) sm[tid >> 6] = m;
  __syncthreads();
  m = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
  __syncthreads();
  int e = 0;
  const double fr = m > 0.0 ? frexp(m, &e) : 0.0;
  if (fr * 128.0 >= 127.5) ++e;
  const double inv = m > 0.0 ? ldexp(1.0, -e) : 0.0;
  if (blockIdx.x == 0 && tid == 0) fscale[rhs] = m > 0.0 ? ldexp(1.0, e) : 1.0;
  if (ok) {
    double v = x * inv;
    for (int b = 0; b < Sf; ++b) {
      const double sc = v * 128.0, t = rint(sc);
      v = sc - t;
      fsl[(((size_t)rhs * Sf + b) * n_leaves + leaf) * P + k] = (int8_t)t;
    }
  }
  // per-leaf mass: P = 64 -> one wave per leaf; P = 256 -> four waves
  double w = ok ? wk * x : 0.0;
  for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
  if (P <= 64) {
    if ((tid & 63) == 0 && ok) lmass[(size_t)rhs * n_leaves + leaf] = w;
  } else {
    if ((tid & 63) == 0) sm[tid >> 6] = w;
    __syncthreads();
    if (tid == 0 && leaf < n_leaves) lmass[(size_t)rhs * n_leaves + leaf] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
  }
}

// Near (U list) field of one 64-leaf tile in int8 slices, plus L2T and the W
// list in FP64; writes V and G.  Two blocks of 4 waves share a work unit, one
// per half of the tile's 64 columns (block b: unit 8 (b / 16) + b % 8, half
// (b / 8) % 2, so both halves run on the unit's XCD), and two blocks fit on a
// CU, so one block's index loads and epilogue overlap the other's products.
// Wave w4 owns row tiles mt0 + w4 + 4i (i < TPW) and the 16-column tiles
// 2 half, 2 half + 1.  Per work item (slot, 64-wide K chunk) the B slices of
// the block's 32 columns are staged in LDS (double buffered, swizzled so that
// the 16-lane groups of a 16-byte read hit distinct banks); the A slices stream
// from the table two iterations ahead, in the slice order 0,5,1,4,2,3 that
// alternates long and short iterations.
template <int TPW, int NCH, int KCF>
__global__ void __launch_bounds__(256, 2) leaf_near_i8_kernel(DevTables t, DevTree g, const int8_t *__restrict__ fsl,
                                                             const double *__restrict__ lmass,
                                                             const double *__restrict__ fscale,
                                                             const double *__restrict__ f,
                                                             const double *__restrict__ M,
                                                             const double *__restrict__ L, double *__restrict__ V,
                                                             double *__restrict__ G) {
  constexpr int HC = LEAF_TILE / 2;                        // columns per block
  constexpr int SG = NEAR_SG, P = 64 * NCH, MTR = 3 * P / 16, PPT = SG * HC * 4 / 256;
  constexpr int KSC = KCF / 4, PERT = KCF / 8, SBF = KCF + 1;   // FP64 phase: chunks of KCF columns
  constexpr int BYTES_I8 = 2 * SG * HC * 4 * 16, BYTES_F64 = 2 * HC * SBF * 8;
  static_assert(SG * HC * 4 % 256 == 0, "staging pieces must divide over the block");
  __shared__ __attribute__((aligned(16))) unsigned char smem[BYTES_I8 > BYTES_F64 ? BYTES_I8 : BYTES_F64];
  __shared__ double sMass[HC];                            // per local column
  uint4(*sB)[SG * HC * 4] = (uint4(*)[SG * HC * 4])smem;  // [buf][slice][local column][16-byte piece]
  const int unit = (blockIdx.x >> 4) * 8 + (blockIdx.x & 7), half = (blockIdx.x >> 3) & 1;
  const int tile = g.nunit_tile[unit];
  if (tile < 0) return;                                    // whole block: no barrier is skipped
  const int tid = threadIdx.x, lane = tid & 63, w4 = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, kq = lane >> 4, rhs = blockIdx.z;
  const int mt0 = g.nunit_mt[unit] & 0xffff;               // first row tile of this unit
  const int ni = g.nunit_mt[unit] >> 16;                   // row tiles per wave: TPW, or 1 for a heavy tile's thirds
  const int NL = g.n_leaves, Sf = g.split_sf;
  const int s0 = g.nslot_ptr[tile], s1 = g.nslot_ptr[tile + 1], nitems = (s1 - s0) * NCH;
  const int nsl = g.tile_nsl[tile], Sv = nsl & 255, Sd = (nsl >> 8) & 255;
  int Si[TPW];
  size_t arow[TPW];                                        // A offset of each row tile (in 16-byte units)
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int mt = mt0 + w4 + 4 * i;
    Si[i] = (i >= ni || mt >= MTR) ? 0 : (mt * 16 < P ? Sv : Sd);
    arow[i] = (size_t)(i < ni && mt < MTR ? mt : mt0 + w4) * NCH * 64 + lane;
  }
  const int8_t *fr = fsl + (size_t)rhs * Sf * NL * P;
  const i32x4 *Atab = (const i32x4 *)t.near_i8;
  const size_t cfg_stride = (size_t)NEAR_SMAX * MTR * NCH * 64, sl_stride = (size_t)MTR * NCH * 64;
  // the tile's slot configurations and source leaves (at most 33 slots) in LDS:
  // index reads in the loop then never wait behind the vector-memory queue
  __shared__ int sCfg[33], sSrc[33 * 64];
  for (int i = tid; i < (s1 - s0) * 64; i += 256) sSrc[i] = g.nslot_src[(size_t)s0 * 64 + i];
  if (tid < s1 - s0) sCfg[tid] = g.nslot_cfg[s0 + tid];
  __syncthreads();

  i32x4 acc[TPW][2][SG];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int d = 0; d < SG; ++d) acc[i][nt][d] = i32x4{0, 0, 0, 0};

  // staging of item j (slot s0 + j / NCH, chunk j % NCH): piece q = tid + 256 m
  // is 16 bytes (k 16 kk..) of slice b of local column lc (tile column
  // HC half + lc)
  uint4 stg[PPT];
  bool sok[PPT];
  auto stage_load = [&](int j) {
    const int sl = j / NCH, ch = j % NCH;
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      const int q = tid + 256 * m, b = q >> 7, lc = (q >> 2) & (HC - 1), kk = q & 3;
      const int src = sSrc[sl * 64 + HC * half + lc];
      sok[m] = src >= 0;
      const int bb = b < Sf ? b : Sf - 1;
      stg[m] = *(const uint4 *)(fr + ((size_t)bb * NL + (src >= 0 ? src : 0)) * P + ch * 64 + kk * 16);
    }
  };
  auto stage_write = [&](int buf) {
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      const int q = tid + 256 * m, b = q >> 7, lc = (q >> 2) & (HC - 1), kk = q & 3;
      sB[buf][b * HC * 4 + lc * 4 + (kk ^ ((lc >> 2) & 3))] = sok[m] ? stg[m] : make_uint4(0, 0, 0, 0);
    }
  };
  // A fragments: a_cur for this iteration, a_nxt for the next, a_new two ahead
  // (shifted each iteration, so the pipeline runs across items of any length)
  i32x4 a_cur[TPW], a_nxt[TPW];
  auto a_load = [&](i32x4 *dst, int j, int a, auto nic) {
    constexpr int NI = decltype(nic)::value;
    const int ch = j % NCH;
    const size_t base = (size_t)sCfg[j / NCH] * cfg_stride + (size_t)a * sl_stride + ch * 64;
#pragma unroll
    for (int i = 0; i < NI; ++i) dst[i] = Atab[base + arow[i]];
  };

  // The slice counts are compile-time in the loop (one branch-free body per
  // class, chosen once per block): T0 for row tile i = 0, T1 for i = 1, 2 (the
  // two row types of a unit), each at least 3 and rounded up to T0 <= T1; extra
  // slice pairs only make the product more exact.
  const int T0 = Si[0] > 3 ? Si[0] : 3, T1r = Si[TPW - 1] > 3 ? Si[TPW - 1] : 3;
  const int T1 = ni < TPW ? T0 : (T1r > T0 ? T1r : T0);
  int Tsel[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) Tsel[i] = i >= ni ? 0 : (i == 0 ? T0 : T1);
  auto run = [&](auto t0c, auto t1c, auto nic) {
    constexpr int C0 = decltype(t0c)::value, C1 = decltype(t1c)::value, NI = decltype(nic)::value;
    // iteration idx handles slice a = SEQ(idx): 0, C1-1, 1, C1-2, ... (long and short alternate)
    auto seq = [](int idx) { return idx % 2 == 0 ? idx / 2 : C1 - 1 - idx / 2; };
    if (nitems > 0) {
      stage_load(0);
      stage_write(0);
      stage_load(nitems > 1 ? 1 : 0);
      a_load(a_cur, 0, seq(0), nic);
      a_load(a_nxt, 0, seq(1), nic);
    }
    for (int j = 0; j < nitems; ++j) {
      const int buf = j & 1, jn = j + 1 < nitems ? j + 1 : j, jnn = j + 2 < nitems ? j + 2 : jn;
      __syncthreads();                                     // item j staged; buffer buf ^ 1 free
      if (j + 1 < nitems) stage_write(buf ^ 1);
      const uint4 *S = sB[buf];
#pragma unroll
      for (int idx = 0; idx < C1; ++idx) {
        const int a = seq(idx);
        // fragments two iterations ahead (the next item's first two at the end)
        i32x4 a_new[TPW];
        if (idx + 2 < C1) a_load(a_new, j, seq(idx + 2), nic);
        else a_load(a_new, jn, seq(idx + 2 - C1), nic);
        if (idx == 1) stage_load(jnn);
#pragma unroll
        for (int b = 0; b < C1 - a; ++b) {
          i32x4 bv[2];
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            const int lc = nt * 16 + col;
            bv[nt] = __builtin_bit_cast(i32x4, S[b * HC * 4 + lc * 4 + (kq ^ ((lc >> 2) & 3))]);
          }
#pragma unroll
          for (int i = 0; i < NI; ++i)
            if (a + b < (i == 0 ? C0 : C1)) {
#pragma unroll
              for (int nt = 0; nt < 2; ++nt) acc[i][nt][a + b] = mfma_i8(a_cur[i], bv[nt], acc[i][nt][a + b]);
            }
        }
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          a_cur[i] = a_nxt[i];
          a_nxt[i] = a_new[i];
        }
      }
    }
  };
  using std::integral_constant;
#define BX_RUN(A, B_) run(integral_constant<int, A>(), integral_constant<int, B_>(), integral_constant<int, TPW>())
#define BX_RUN1(A) run(integral_constant<int, A>(), integral_constant<int, A>(), integral_constant<int, 1>())
  if (ni < TPW) {                                          // one row tile per wave
    if (T0 == 3) BX_RUN1(3); else if (T0 == 4) BX_RUN1(4); else if (T0 == 5) BX_RUN1(5); else BX_RUN1(6);
  } else if (T0 == 3) {
    if (T1 == 3) BX_RUN(3, 3); else if (T1 == 4) BX_RUN(3, 4); else if (T1 == 5) BX_RUN(3, 5); else BX_RUN(3, 6);
  } else if (T0 == 4) {
    if (T1 == 4) BX_RUN(4, 4); else if (T1 == 5) BX_RUN(4, 5); else BX_RUN(4, 6);
  } else if (T0 == 5) {
    if (T1 == 5) BX_RUN(5, 5); else BX_RUN(5, 6);
  } else {
    BX_RUN(6, 6);
  }
#undef BX_RUN1
#undef BX_RUN
  // U-list mass of column HC half + tid / 8: this thread's slots tid % 8 + 8 k
  // (at most 33 slots), all requested at once; summed over the column's 8
  // threads together with the FP64 slots' part below
  double mU = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int sl = (tid & 7) + 8 * k;
    const int src = sl < s1 - s0 ? sSrc[sl * 64 + HC * half + (tid >> 3)] : -1;
    if (src >= 0) mU = fma(t.split_cfg_w2[sCfg[sl]], lmass[(size_t)rhs * NL + src], mU);
  }
  // ---- FP64 phase: L2T, the W list and the U slots of tiles left in FP64,
  // seeded with the scaled int8 group sums.  The FP64 tables' rows are permuted
  // so that accumulator register r of a lane holds row 4 (lane / 16) + r, the
  // int8 layout, and the sums move over in place.
  const double fsc = fscale[rhs];
  dbl4 fa[TPW][2];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int mt = mt0 + w4 + 4 * i;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (i < ni && mt < MTR ? mt : 0) * 16 + 4 * kq + r;
        const double rs = t.split_row_scale[row] * fsc;
        double v = 0.0;
#pragma unroll
        for (int d = SG - 1; d >= 0; --d)
          if (d < Tsel[i]) v += (double)acc[i][nt][d][r] * ldexp(rs, -7 * (d + 2));
        fa[i][nt][r] = v;
      }
  }
  double *sF = (double *)smem;                             // [2][HC * SBF], local columns
  const int lcol = tid >> 3, scol = HC * half + lcol, sq = tid & 7;   // staging: 8 threads per column
  const int stgt = g.tile_tgt[tile * LEAF_TILE + scol];
  // the epilogue's targets (columns 16 (2 half + nt) + col) and their levels,
  // requested beside the staging target's
  int etgt[2], elev[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) etgt[nt] = g.tile_tgt[tile * LEAF_TILE + (2 * half + nt) * 16 + col];
  const double sh = stgt >= 0 ? box_h(g.width, g.leaf_level[stgt]) : 1.0;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) elev[nt] = g.leaf_level[etgt[nt] >= 0 ? etgt[nt] : 0];
  const double sinv_h2 = stgt >= 0 ? 1.0 / (sh * sh) : 0.0;
  const int f0 = g.tile_ptr[tile], f1 = g.tile_ptr[tile + 1], K2 = 2 * t.KP;
  const int *slot_type = g.slot_type, *slot_op = g.slot_op, *slot_aoff = g.slot_aoff, *slot_src = g.slot_src + scol;
  const double *fr64 = f + (size_t)rhs * NL * P;
  const double *Lr = L + (size_t)rhs * g.n_boxes * K2, *Mr = M + (size_t)rhs * g.n_boxes * K2;
  const double *leaf_frag = t.leaf_frag, *leaf_mass = t.leaf_mass;
  const int kmax = t.leaf_kmax;
  double mpart = mU;
  Regs<PERT> rb;
  int ir[TPW];                                             // row tile offset of fragment i (tile 0 for i >= ni)
#pragma unroll
  for (int i = 0; i < TPW; ++i) ir[i] = i < ni ? i : 0;
  auto f64_a = [&](int sl_, int c_) -> const double * {
    const int NC_ = (slot_type[sl_] == 0 ? P : K2) / KCF;
    return leaf_frag + slot_aoff[sl_] + ((size_t)(mt0 + w4) * NC_ + c_) * KSC * 64 + lane;
  };
  auto f64_stride = [&](int sl_) -> size_t {
    const int NC_ = (slot_type[sl_] == 0 ? P : K2) / KCF;
    return (size_t)4 * NC_ * KSC * 64;
  };
  auto f64_b = [&](int sl_, int c_) {
    const int type = slot_type[sl_], src = slot_src[sl_ * LEAF_TILE];
    const double *bp = type == 0 ? fr64 + (size_t)(src >= 0 ? src : 0) * P
                                 : (type == 1 ? Lr : Mr) + (size_t)(src >= 0 ? src : 0) * K2;
    const double sc = src < 0 ? 0.0 : (type == 0 ? 1.0 : sinv_h2);
    const double *q = bp + c_ * KCF + sq * PERT;
#pragma unroll
    for (int j = 0; j < PERT; ++j) rb.v[j] = sc * q[j];
  };
  int sl = f0, c = 0, buf = 0;
  __syncthreads();                                         // the int8 buffers are no longer read
  double an[2][TPW];
  if (sl < f1) {
    const double *A0 = f64_a(sl, 0);
    const size_t st0 = f64_stride(sl);
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int i = 0; i < TPW; ++i) an[jj][i] = A0[ir[i] * st0 + jj * 64];
    f64_b(sl, 0);
  }
  while (sl < f1) {
    const int NC = (slot_type[sl] == 0 ? P : K2) / KCF;
    {
      const double *mw = leaf_mass + (size_t)slot_op[sl] * kmax + c * KCF + sq * PERT;
      double *dst = sF + buf * HC * SBF + lcol * SBF + sq * PERT;
#pragma unroll
      for (int j = 0; j < PERT; ++j) {
        dst[j] = rb.v[j];
        mpart = fma(mw[j], rb.v[j], mpart);
      }
    }
    __syncthreads();
    int nsl = sl, nc = c + 1;
    if (nc >= NC) { ++nsl; nc = 0; }
    const bool more = nsl < f1;
    const double *Ac = f64_a(sl, c);
    const size_t stc = f64_stride(sl);
    const double *An = more ? f64_a(nsl, nc) : Ac;
    const size_t stn = more ? f64_stride(nsl) : stc;
    if (more) f64_b(nsl, nc);
    const double *Sx = sF + buf * HC * SBF;
#pragma unroll
    for (int ks = 0; ks < KSC; ++ks) {
      double a[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) a[i] = an[ks % 2][i];
      if (ks + 2 < KSC) {
#pragma unroll
        for (int i = 0; i < TPW; ++i) an[ks % 2][i] = Ac[ir[i] * stc + (ks + 2) * 64];
      } else if (more) {
#pragma unroll
        for (int i = 0; i < TPW; ++i) an[ks % 2][i] = An[ir[i] * stn + (ks + 2 - KSC) * 64];
      }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const double b = Sx[(nt * 16 + col) * SBF + kq * KSC + ks];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          if (i < ni) fa[i][nt] = mfma4(a[i], b, fa[i][nt]);
      }
    }
    sl = nsl;
    c = nc;
    buf ^= 1;
  }
  // mass per column: the sum over the column's 8 threads (U and FP64 slots)
  mpart += __shfl_xor(mpart, 1);
  mpart += __shfl_xor(mpart, 2);
  mpart += __shfl_xor(mpart, 4);
  if (sq == 0) sMass[lcol] = mpart;
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int tgt = etgt[nt];
    if (tgt < 0) continue;
    const double h = box_h(g.width, elev[nt]);
    const double lg = h * h * log(h) * kInv2Pi * sMass[nt * 16 + col];
    double *Vt = V + ((size_t)rhs * NL + tgt) * P;
    double *Gt = G + ((size_t)rhs * NL + tgt) * 2 * P;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int mt = mt0 + w4 + 4 * i;
      if (i >= ni || mt >= MTR) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + 4 * kq + r;
        if (row < P) Vt[row] = h * h * fa[i][nt][r] + lg;
        else Gt[row - P] = h * fa[i][nt][r];
      }
    }
  }
}

// ------------------------------------------------- interpolation at points
// One thread per (target, right-hand side): descend from the root to the leaf
// holding the point, then evaluate the n x n tensor Chebyshev interpolant of
// the leaf's values in barycentric form (first-kind nodes x_j = -cos((2j+1)pi/2n),
// weights (-1)^j sin((2j+1)pi/2n); a coordinate on a node takes that node's
// value exactly).
template <int N>
__device__ inline void cheb_basis(double u, double *l) {
  double w[N], s = 0.0;
  int hit = -1;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double th = (2 * j + 1) * 3.14159265358979323846 / (2 * N);
    const double xj = -cos(th), d = u - xj;
    if (d == 0.0) hit = j;
    w[j] = ((N - 1 - j) % 2 ? -1.0 : 1.0) * sin(th) / (d == 0.0 ? 1.0 : d);
    s += w[j];
  }
#pragma unroll
  for (int j = 0; j < N; ++j) l[j] = hit >= 0 ? (j == hit ? 1.0 : 0.0) : w[j] / s;
}

template <int N>
__global__ void __launch_bounds__(256) interpolate_kernel(DevTree g, const double *__restrict__ V,
                                                          const double *__restrict__ G, const double *__restrict__ xy,
                                                          long long n_targets, double *__restrict__ v_out,
                                                          double *__restrict__ g_out) {
  constexpr int P = N * N;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_targets) return;
  const int rhs = blockIdx.y;
  const double x = xy[2 * i], y = xy[2 * i + 1];
  // unit coordinates of the root square [0, 1)^2
  double ux = (x - g.cx) / g.width + 0.5, uy = (y - g.cy) / g.width + 0.5;
  int leaf = -1;
  double lx = 0.0, ly = 0.0;                   // position inside the leaf, in [-1, 1]
  if (ux >= 0.0 && ux <= 1.0 && uy >= 0.0 && uy <= 1.0) {
    int box = 0;
    double h = 1.0, x0 = 0.0, y0 = 0.0;
    while (g.child0[box] >= 0) {               // children in Morton order (cx + 2 cy)
      h *= 0.5;
      const int qx = ux >= x0 + h ? 1 : 0, qy = uy >= y0 + h ? 1 : 0;
      x0 += qx * h;
      y0 += qy * h;
      box = g.child0[box] + qx + 2 * qy;
    }
    leaf = g.leaf_of_box[box];
    lx = 2.0 * (ux - x0) / h - 1.0;
    ly = 2.0 * (uy - y0) / h - 1.0;
    lx = lx > 1.0 ? 1.0 : lx;                  // the root's right and top edges
    ly = ly > 1.0 ? 1.0 : ly;
  }
  if (leaf < 0) {
    if (V) v_out[(long long)rhs * n_targets + i] = __builtin_nan("");
    if (G) {
      g_out[((long long)rhs * n_targets + i) * 2] = __builtin_nan("");
      g_out[((long long)rhs * n_targets + i) * 2 + 1] = __builtin_nan("");
    }
    return;
  }
  double bx[N], by[N];
  cheb_basis<N>(lx, bx);
  cheb_basis<N>(ly, by);
  if (V) {
    const double *Vl = V + ((size_t)rhs * g.n_leaves + leaf) * P;
    double v = 0.0;
    for (int b = 0; b < N; ++b) {
      double r = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) r = fma(bx[a], Vl[b * N + a], r);
      v = fma(by[b], r, v);
    }
    v_out[(long long)rhs * n_targets + i] = v;
  }
  if (G) {
    const double *Gl = G + ((size_t)rhs * g.n_leaves + leaf) * 2 * P;
    for (int c = 0; c < 2; ++c) {
      double v = 0.0;
      for (int b = 0; b < N; ++b) {
        double r = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) r = fma(bx[a], Gl[c * P + b * N + a], r);
        v = fma(by[b], r, v);
      }
      g_out[((long long)rhs * n_targets + i) * 2 + c] = v;
    }
  }
}

}  // namespace

void launch_p2m(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *M, hipStream_t s) {
  dim3 grid((g.n_leaves + 63) / 64, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(p2m_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, f, M);
  else if (t.KP == 32) hipLaunchKernelGGL(p2m_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, f, M);
  else hipLaunchKernelGGL(p2m_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, f, M);
}
void launch_m2m(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int child_base, int nrhs,
                double *M, hipStream_t s) {
  if (nbox <= 0) return;
  dim3 grid((nbox + 15) / 16, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(m2m_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, boxes, nbox, child_base, M);
  else if (t.KP == 32) hipLaunchKernelGGL(m2m_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, boxes, nbox, child_base, M);
  else hipLaunchKernelGGL(m2m_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, boxes, nbox, child_base, M);
}
void launch_m2m2(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *M,
                 hipStream_t s) {
  if (nbox <= 0) return;
  dim3 grid((nbox + 3) / 4, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(m2m2_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, boxes, nbox, M);
  else if (t.KP == 32) hipLaunchKernelGGL(m2m2_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, boxes, nbox, M);
  else hipLaunchKernelGGL(m2m2_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, boxes, nbox, M);
}
void launch_l2l2(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *L,
                 hipStream_t s) {
  if (nbox <= 0) return;
  dim3 grid((nbox + 3) / 4, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(l2l2_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, boxes, nbox, L);
  else if (t.KP == 32) hipLaunchKernelGGL(l2l2_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, boxes, nbox, L);
  else hipLaunchKernelGGL(l2l2_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, boxes, nbox, L);
}
void launch_m2l(const DevTables &t, const DevTree &g, int nrhs, const double *M, double *L, hipStream_t s) {
  // blocks of contiguous parent ranges, plus one for the root
  const int mb = g.m2l_blocks > 0 ? g.m2l_blocks : M2L_BLOCKS;
  const int nb = g.n_m2l_par < mb ? (g.n_m2l_par > 0 ? g.n_m2l_par : 1) : mb;
  const int per = g.n_m2l_par > 0 ? (g.n_m2l_par + nb - 1) / nb : 0;
  dim3 grid(nb + 1, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(m2l_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, M, L, per);
  else if (t.KP == 32) hipLaunchKernelGGL(m2l_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, M, L, per);
  else hipLaunchKernelGGL(m2l_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, M, L, per);
}
void launch_p2l(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *L, hipStream_t s) {
  if (g.n_xtiles <= 0) return;
  dim3 grid((g.n_xtiles + 3) / 4, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(p2l_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, f, L);
  else if (t.KP == 32) hipLaunchKernelGGL(p2l_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, f, L);
  else hipLaunchKernelGGL(p2l_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, f, L);
}
void launch_l2l(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *L,
                hipStream_t s) {
  if (nbox <= 0) return;
  // levels with fewer than two blocks per CU of 16 parents spread the four
  // child positions over blocks as well
  const bool wide = (long long)(nbox + 15) / 16 * nrhs < 512;
  dim3 grid((nbox + 15) / 16, nrhs, wide ? 4 : 1);
  if (wide) {
    if (t.KP == 16) hipLaunchKernelGGL((l2l_mfma_kernel<16, true>), grid, dim3(256), 0, s, t, g, boxes, nbox, L);
    else if (t.KP == 32) hipLaunchKernelGGL((l2l_mfma_kernel<32, true>), grid, dim3(256), 0, s, t, g, boxes, nbox, L);
    else hipLaunchKernelGGL((l2l_mfma_kernel<48, true>), grid, dim3(256), 0, s, t, g, boxes, nbox, L);
  } else {
    if (t.KP == 16) hipLaunchKernelGGL((l2l_mfma_kernel<16, false>), grid, dim3(256), 0, s, t, g, boxes, nbox, L);
    else if (t.KP == 32) hipLaunchKernelGGL((l2l_mfma_kernel<32, false>), grid, dim3(256), 0, s, t, g, boxes, nbox, L);
    else hipLaunchKernelGGL((l2l_mfma_kernel<48, false>), grid, dim3(256), 0, s, t, g, boxes, nbox, L);
  }
}
void launch_leaf(const DevTables &t, const DevTree &g, const double *f, int nrhs, const double *M,
                 const double *L, double *V, double *G, bool accumulate, hipStream_t s) {
  const int acc = accumulate ? 1 : 0;
  if (g.n_units <= 0) return;
  const dim3 grid(g.n_units, 1, nrhs);      // one work unit per block (a multiple of the 8 XCDs)
  // K chunks of t.leaf_kc columns (a divisor of P and of 2 KP)
  if (t.n == 4) {         // 3 row tiles, K chunks of 16
    hipLaunchKernelGGL((leaf_mfma_kernel<1, 16>), grid, dim3(256), 0, s, t, g, f, M, L, V, G, acc);
  } else if (t.n == 8) {  // 12 row tiles: 3 per wave
    if (t.leaf_kc == 64) hipLaunchKernelGGL((leaf_mfma_kernel<3, 64>), grid, dim3(256), 0, s, t, g, f, M, L, V, G, acc);
    else hipLaunchKernelGGL((leaf_mfma_kernel<3, 32>), grid, dim3(256), 0, s, t, g, f, M, L, V, G, acc);
  } else {                // 48 row tiles: groups of 16, 4 per wave
    if (t.leaf_kc == 64) hipLaunchKernelGGL((leaf_mfma_kernel<4, 64>), grid, dim3(256), 0, s, t, g, f, M, L, V, G, acc);
    else hipLaunchKernelGGL((leaf_mfma_kernel<4, 32>), grid, dim3(256), 0, s, t, g, f, M, L, V, G, acc);
  }
}

void launch_split_prep(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *fpart,
                       double *fscale, int8_t *fsl, double *lmass, hipStream_t s) {
  const size_t count = (size_t)g.n_leaves * t.P;
  const int nparts = (int)std::min<size_t>(FMAX_BLOCKS, (count + 2047) / 2048);
  hipLaunchKernelGGL(fmax_partial_kernel, dim3(nparts, nrhs), dim3(256), 0, s, f, count, fpart);
  const int lpb = t.P >= 256 ? 1 : 256 / t.P;
  hipLaunchKernelGGL(split_prep_kernel, dim3((g.n_leaves + lpb - 1) / lpb, nrhs), dim3(256), 0, s, f, t.wq, t.P,
                     g.n_leaves, fpart, nparts, g.split_sf, fscale, fsl, lmass);
}

void launch_leaf_split(const DevTables &t, const DevTree &g, const int8_t *fsl, const double *lmass,
                       const double *fscale, const double *f, int nrhs, const double *M, const double *L, double *V,
                       double *G, hipStream_t s) {
  if (g.n_nunits <= 0) return;
  // two half-tile blocks per unit (the unit list is padded to a multiple of 8)
  const dim3 grid(2 * g.n_nunits, 1, nrhs);
#define BX_NEAR(NCH, KCF)                                                                                        \
  hipLaunchKernelGGL((leaf_near_i8_kernel<3, NCH, KCF>), grid, dim3(256), 0, s, t, g, fsl, lmass, fscale, f, M, L, \
                     V, G)
  if (t.n == 8 && t.leaf_kc == 64) BX_NEAR(1, 64);
  else if (t.n == 8) BX_NEAR(1, 32);
  else if (t.leaf_kc == 64) BX_NEAR(4, 64);
  else BX_NEAR(4, 32);
#undef BX_NEAR
}

void launch_interpolate(const DevTables &t, const DevTree &g, const double *V, const double *G, int nrhs,
                        const double *xy, long long n_targets, double *v_out, double *g_out, hipStream_t s) {
  const dim3 grid((unsigned)((n_targets + 255) / 256), nrhs);
  if (t.n == 4) hipLaunchKernelGGL(interpolate_kernel<4>, grid, dim3(256), 0, s, g, V, G, xy, n_targets, v_out, g_out);
  else if (t.n == 8) hipLaunchKernelGGL(interpolate_kernel<8>, grid, dim3(256), 0, s, g, V, G, xy, n_targets, v_out, g_out);
  else hipLaunchKernelGGL(interpolate_kernel<16>, grid, dim3(256), 0, s, g, V, G, xy, n_targets, v_out, g_out);
}

}  // namespace bx
