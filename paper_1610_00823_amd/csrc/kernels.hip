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
                                                       int nbox, double *__restrict__ M) {
  constexpr int R = 2 * KPT, MT = R / 16, KS = R / 4;
  __shared__ double part[4][16][R + 1];
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int i = blockIdx.x * 16 + col, rhs = blockIdx.y;
  const bool ok = i < nbox;
  const int box = ok ? boxes[i] : 0;
  double *Mr = M + (size_t)rhs * g.n_boxes * R;
  const double *bp = Mr + (size_t)((ok ? g.child0[box] : 0) + c) * R + kq * KS;
  const double *A = t.m2m_frag + (size_t)c * MT * KS * 64;
  dbl4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = dbl4{0, 0, 0, 0};
  for (int ks = 0; ks < KS; ks += 4) {
    double bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = ok ? bp[ks + j] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = mfma4(A[((size_t)m * KS + ks + j) * 64 + lane], bv[j], acc[m]);
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
template <int KPT>
__global__ void __launch_bounds__(256) l2l_mfma_kernel(DevTables t, DevTree g, const int *__restrict__ boxes,
                                                       int nbox, double *__restrict__ L) {
  constexpr int R = 2 * KPT, MT = R / 16, KS = R / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int i = blockIdx.x * 16 + col, rhs = blockIdx.y, c = blockIdx.z;
  const bool ok = i < nbox;
  const int box = ok ? boxes[i] : 0;
  double *Lr = L + (size_t)rhs * g.n_boxes * R;
  const double *bp = Lr + (size_t)box * R + kq * KS;
  const double *A = t.l2l_frag + (size_t)c * MT * KS * 64;
  for (int m = wave; m < MT; m += 4) {
    dbl4 acc = dbl4{0, 0, 0, 0};
#pragma unroll 4
    for (int ks = 0; ks < KS; ++ks) acc = mfma4(A[((size_t)m * KS + ks) * 64 + lane], ok ? bp[ks] : 0.0, acc);
    if (ok) {
      double *Lc = Lr + (size_t)(g.child0[box] + c) * R;
#pragma unroll
      for (int r = 0; r < 4; ++r) Lc[m * 16 + 4 * r + kq] += acc[r];
    }
  }
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
// rows V (P), dV/dx1 (P), dV/dx2 (P); with mass = sum over slots of the
// operators' mass weights times B,
//   V = h^2 acc_V + (h^2 log h / 2pi) mass,  grad V = h acc_D,
// which carries the per-level scaling of the unit-box tables, the a_0 log h
// of the W multipoles and the 1/h of the gradients (the tables hold the rest).
// Block = 4 waves = 64 leaves.  The slot's B columns (64 x KC) are staged in
// LDS once per block (double buffered through registers, one barrier per
// chunk); wave w owns row tiles w, w+4, w+8, ... of its row group and all four
// 16-leaf column tiles, so each A fragment read from the operator table feeds
// four MFMAs.  grid.y splits the rows into groups of 4*TPW tiles.
constexpr int LEAF_TILE = 64;

// logical block index that gives each XCD (blocks are dealt round-robin to
// the 8 XCDs) a contiguous range of tiles; -1 for padding blocks
__device__ inline int xcd_block(int b, int nb_logical) {
  const int per = (nb_logical + 7) / 8;
  const int l = (b % 8) * per + b / 8;
  return l < nb_logical ? l : -1;
}

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
                                                           double *__restrict__ G) {
  constexpr int KSC = KC / 4, PERT = KC / 4, SB = KC + 1;
  __shared__ double sB[2][LEAF_TILE * SB];
  __shared__ double sMass[LEAF_TILE];
  const int tile = xcd_block(blockIdx.x, g.n_tiles);
  if (tile < 0) return;                        // whole block: no barrier is skipped
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int rhs = blockIdx.z, P = t.P, K2 = 2 * t.KP, MTR = 3 * P / 16;
  const int mtg = blockIdx.y * 4 * TPW;        // first row tile of this group
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
  Regs<PERT> rb;
  int sl = s0, c = 0, buf = 0;
  if (sl < s1) rb = leaf_chunk_load<KC>(slot_type, slot_src, fr, Lr, Mr, sl, 0, P, K2, sq, sinv_h2);
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
    const double *A = leaf_frag + slot_aoff[sl] + (size_t)c * KSC * 64;
    int nsl = sl, nc = c + 1;
    if (nc >= NC) { ++nsl; nc = 0; }
    if (nsl < s1)                                  // next chunk in flight during the MFMAs
      rb = leaf_chunk_load<KC>(slot_type, slot_src, fr, Lr, Mr, nsl, nc, P, K2, sq, sinv_h2);
    const double *S = sB[buf];
#pragma unroll 4
    for (int ks = 0; ks < KSC; ++ks) {
      double a[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int mt = mtg + wave + 4 * i;
        a[i] = mt < MTR ? A[((size_t)mt * NC * KSC + ks) * 64 + lane] : 0.0;
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const double b = S[(nt * 16 + col) * SB + kq * KSC + ks];
#pragma unroll
        for (int i = 0; i < TPW; ++i) acc[i][nt] = mfma4(a[i], b, acc[i][nt]);
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
      if (mt >= MTR) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + 4 * r + kq;
        if (row < P) Vt[row] = h * h * acc[i][nt][r] + lg;
        else Gt[row - P] = h * acc[i][nt][r];
      }
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
void launch_m2m(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *M,
                hipStream_t s) {
  if (nbox <= 0) return;
  dim3 grid((nbox + 15) / 16, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(m2m_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, boxes, nbox, M);
  else if (t.KP == 32) hipLaunchKernelGGL(m2m_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, boxes, nbox, M);
  else hipLaunchKernelGGL(m2m_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, boxes, nbox, M);
}
void launch_m2l(const DevTables &t, const DevTree &g, int nrhs, const double *M, double *L, hipStream_t s) {
  dim3 grid((g.n_boxes + 3) / 4, nrhs);
  if (t.KP == 16) hipLaunchKernelGGL(m2l_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, M, L);
  else if (t.KP == 32) hipLaunchKernelGGL(m2l_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, M, L);
  else hipLaunchKernelGGL(m2l_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, M, L);
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
  dim3 grid((nbox + 15) / 16, nrhs, 4);
  if (t.KP == 16) hipLaunchKernelGGL(l2l_mfma_kernel<16>, grid, dim3(256), 0, s, t, g, boxes, nbox, L);
  else if (t.KP == 32) hipLaunchKernelGGL(l2l_mfma_kernel<32>, grid, dim3(256), 0, s, t, g, boxes, nbox, L);
  else hipLaunchKernelGGL(l2l_mfma_kernel<48>, grid, dim3(256), 0, s, t, g, boxes, nbox, L);
}
void launch_leaf(const DevTables &t, const DevTree &g, const double *f, int nrhs, const double *M,
                 const double *L, double *V, double *G, hipStream_t s) {
  const int bx = (g.n_tiles + 7) / 8 * 8;     // padded to a multiple of the 8 XCDs
  if (t.n == 4) {         // 3 row tiles, K chunks of 16
    hipLaunchKernelGGL((leaf_mfma_kernel<1, 16>), dim3(bx, 1, nrhs), dim3(256), 0, s, t, g, f, M, L, V, G);
  } else if (t.n == 8) {  // 12 row tiles: 3 per wave
    hipLaunchKernelGGL((leaf_mfma_kernel<3, 64>), dim3(bx, 1, nrhs), dim3(256), 0, s, t, g, f, M, L, V, G);
  } else {                // 48 row tiles: 3 groups of 16, 4 per wave
    hipLaunchKernelGGL((leaf_mfma_kernel<4, 64>), dim3(bx, 3, nrhs), dim3(256), 0, s, t, g, f, M, L, V, G);
  }
}

}  // namespace bx
