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
// the power tables of the 49 offsets sit in LDS, and the next 8 sources'
// multipoles are loaded while the current ones are multiplied.  Writes
// (initialises) every box's local expansion.
template <int KPT>
__global__ void __launch_bounds__(256) m2l_mfma_kernel(DevTables t, DevTree g, const double *__restrict__ M,
                                                       double *__restrict__ L) {
  constexpr int MT = KPT / 16, KS = KPT / 4;
  constexpr int PWS = KPT + 1;                 // padded row: 8 offsets per column group, distinct banks
  __shared__ double2 spw[2][NOFF_DEV * PWS];
  __shared__ double slogd[NOFF_DEV];
  for (int i = threadIdx.x; i < NOFF_DEV * KPT; i += 256) {
    spw[0][i / KPT * PWS + i % KPT] = ((const double2 *)t.pw_src)[i];
    spw[1][i / KPT * PWS + i % KPT] = ((const double2 *)t.pw_tgt)[i];
  }
  if (threadIdx.x < NOFF_DEV) slogd[threadIdx.x] = t.logd[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4, part = col & 1;
  const int box = blockIdx.x * 4 + wave;
  if (box >= g.n_boxes) return;                 // no barrier follows
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
  // Two-stage pipeline over groups of 8 sources (this lane: source e + col/2):
  // the data of group g+1 and the indices of group g+2 are requested before
  // group g is multiplied.
  auto idx = [&](int e, int &s_, int &o_, bool &ok_) {
    const int pe = e + (col >> 1);
    ok_ = pe < e1;
    const int pc = ok_ ? pe : (e1 > 0 ? e1 - 1 : 0);   // always a valid entry: the loads are unconditional
    s_ = g.v_src[pc];
    o_ = g.v_cfg[pc];
  };
  auto data = [&](int s_, double2 *dst) {
    const double2 *ap = (const double2 *)(Mr + (size_t)s_ * KPT * 2) + kq * KS;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) dst[ks] = ap[ks];
  };
  int s_c, o_c, s_n, o_n;
  bool ok_c, ok_n;
  double2 av[KS];
  idx(e0, s_c, o_c, ok_c);
  data(s_c, av);
  idx(e0 + 8, s_n, o_n, ok_n);
  for (int e = e0; e < e1; e += 8) {
    double2 an[KS];
    data(s_n, an);                                 // group g+1
    int s_nn, o_nn;
    bool ok_nn;
    idx(e + 16, s_nn, o_nn, ok_nn);                // group g+2
    double bv[KS];
    const double2 *wp = &spw[0][o_c * PWS + kq * KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const double2 a = av[ks], w = wp[ks];
      const double y = part ? a.x * w.y + a.y * w.x : a.x * w.x - a.y * w.y;
      bv[ks] = ok_c ? y : 0.0;
    }
    a0 += (ok_c && part == 0 && kq == 0) ? av[0].x * (logh + slogd[o_c]) : 0.0;
    dbl4 c[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) c[m] = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int m = 0; m < MT; ++m) c[m] = mfma4(hA[m][ks], bv[ks], c[m]);
    const double2 *qp = &spw[1][o_c * PWS];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double z = c[m][r], zo = __shfl_xor(z, 1);
        const double zr = part ? zo : z, zi = part ? z : zo;
        const double2 q = qp[m * 16 + 4 * r + kq];
        const double v = part ? zr * q.y + zi * q.x : zr * q.x - zi * q.y;
        acc[m][r] += ok_c ? v : 0.0;
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) av[ks] = an[ks];
    s_c = s_n; o_c = o_n; ok_c = ok_n;
    s_n = s_nn; o_n = o_nn; ok_n = ok_nn;
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
                                                           double *__restrict__ G) {
  constexpr int KSC = KC / 4, PERT = KC / 4, SB = KC + 1;
  __shared__ double sB[2][LEAF_TILE * SB];
  __shared__ double sMass[LEAF_TILE];
  const int tile = g.unit_tile[blockIdx.x];
  if (tile < 0) return;                        // whole block: no barrier is skipped
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
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
        if (row < P) Vt[row] = h * h * acc[i][nt][r] + lg;
        else Gt[row - P] = h * acc[i][nt][r];
      }
    }
  }
}


// ------------------------------------------- split-precision leaf evaluation
// As leaf_mfma_kernel, but the near-table slots run as exact BF16 slice
// products.  A table value is sum_a t_a 2^(Et - 8(a+1)) and a sample
// sum_b s_b 2^(Ef - 8(b+1)), integers |t_a|, |s_b| <= 256 stored with their
// scales (exact in BF16; Et per row type, Ef per source leaf).  Within one slot
// every product of slice group d = a + b has the same scale, and a 32-term
// v_mfma_f32_16x16x32_bf16 sum of them is an integer below 2^22 times that
// scale: exact in FP32 (a group of d+1 pairs over 64 k stays below 2^24 for
// d <= 3; later groups lie below 2^-24 of the result).  Each group's sum is
// added to the FP64 accumulator when the group is complete (groups of
// different scales are never mixed in one FP32 sum: the MFMA accumulation of
// such mixtures was measured to lose about 2^-33).  S per tile and row type
// comes from the tile's level.  L2T, W, the mass (log h) term and all scalings stay FP64.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ inline flt4 mfma_bf16(bf16x8 a, bf16x8 b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// power-of-two scale 2^e >= max |f| of each leaf (1 for an all-zero leaf)
__global__ void __launch_bounds__(64) leaf_scale_kernel(const double *__restrict__ f, int P, int n_leaves,
                                                        double *__restrict__ fscale) {
  const int leaf = blockIdx.x, rhs = blockIdx.y;
  const double *fl = f + ((size_t)rhs * n_leaves + leaf) * P;
  double m = 0.0;
  for (int j = threadIdx.x; j < P; j += 64) m = fmax(m, fabs(fl[j]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (threadIdx.x == 0) {
    int e = 0;
    frexp(m, &e);
    fscale[(size_t)rhs * n_leaves + leaf] = m > 0.0 ? ldexp(1.0, e) : 1.0;
  }
}

__device__ inline uint32_t bf16_bits(double v) { return __float_as_uint((float)v) >> 16; }

template <int TPW, int KC>
__global__ void __launch_bounds__(256, 1) leaf_split_kernel(DevTables t, DevTree g, const double *__restrict__ f,
                                                            const double *__restrict__ fscale,
                                                            const double *__restrict__ M,
                                                            const double *__restrict__ L, double *__restrict__ V,
                                                            double *__restrict__ G) {
  constexpr int SMAX = 6, PERT = KC / 4, SB = KC + 1, SBH = KC + 8, NST = KC / 32, KSC = KC / 4;
  constexpr int BYTES64 = LEAF_TILE * SB * 8, BYTES16 = SMAX * LEAF_TILE * SBH * 2;
  __shared__ __attribute__((aligned(16))) unsigned char smem[BYTES64 > BYTES16 ? BYTES64 : BYTES16];
  __shared__ double sMass[LEAF_TILE];
  double *sB = (double *)smem;
  uint16_t *sH = (uint16_t *)smem;
  const int tile = g.unit_tile[blockIdx.x];
  if (tile < 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, kq = lane >> 4;
  const int rhs = blockIdx.z, P = t.P, K2 = 2 * t.KP, MTR = 3 * P / 16, NCU = P / KC;
  const int mtg = g.unit_mt[blockIdx.x] & 0xffff, ni = g.unit_mt[blockIdx.x] >> 16;
  const int s0 = g.tile_ptr[tile], s1 = g.tile_ptr[tile + 1];
  const int nsl_v = g.tile_nsl[tile] & 255, nsl_d = g.tile_nsl[tile] >> 8;
  const int nsl = nsl_v > nsl_d ? nsl_v : nsl_d;
  const double *fr = f + (size_t)rhs * g.n_leaves * P;
  const double *fs = fscale + (size_t)rhs * g.n_leaves;
  const double *Lr = L + (size_t)rhs * g.n_boxes * K2, *Mr = M + (size_t)rhs * g.n_boxes * K2;
  const int *slot_type = g.slot_type, *slot_op = g.slot_op, *slot_aoff = g.slot_aoff;
  const double *leaf_frag = t.leaf_frag, *leaf_mass = t.leaf_mass;
  const int kmax = t.leaf_kmax;
  const int scol = threadIdx.x >> 2, sq = threadIdx.x & 3;
  const int stgt = g.tile_tgt[tile * LEAF_TILE + scol];
  const double sinv_h2 = stgt >= 0 ? 1.0 / (box_h(g.width, g.leaf_level[stgt]) * box_h(g.width, g.leaf_level[stgt]))
                                   : 0.0;
  const int *slot_src = g.slot_src + scol;
  int tns[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) tns[i] = i >= ni ? 0 : ((mtg + wave + 4 * i) * 16 < P ? nsl_v : nsl_d);
  const uint4 *Ab = (const uint4 *)t.near_bf16;
  // A slice fragments of row tile i (rows beyond the tables read tile 0: zero work is masked later)
  auto a_base = [&](int op, int a, int i, int c_) -> size_t {
    const int mt = mtg + wave + 4 * (i < ni ? i : 0);
    return ((((size_t)op * SMAX + a) * MTR + (mt < MTR ? mt : 0)) * NCU + c_) * NST * 64 + lane;
  };

  dbl4 acc[TPW][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[i][nt] = dbl4{0, 0, 0, 0};
  double mpart = 0.0;
  Regs<PERT> rb;
  int sl = s0, c = 0;
  if (sl < s1) rb = leaf_chunk_load<KC>(slot_type, slot_src, fr, Lr, Mr, sl, 0, P, K2, sq, sinv_h2);
  while (sl < s1) {
    const int type = slot_type[sl], K = type == 0 ? P : K2, NC = K / KC;
    __syncthreads();                               // the previous chunk's readers are done
    {
      const double *mw = leaf_mass + (size_t)slot_op[sl] * kmax + c * KC + sq * PERT;
#pragma unroll
      for (int j = 0; j < PERT; ++j) mpart = fma(mw[j], rb.v[j], mpart);
      if (type == 0) {   // samples: slices with their true scales 2^(Ef - 8(b+1))
        const int src = slot_src[sl * LEAF_TILE];
        const double sc = src >= 0 ? fs[src] : 1.0, inv = src >= 0 ? 1.0 / sc : 0.0;
        double r[PERT];
#pragma unroll
        for (int j = 0; j < PERT; ++j) r[j] = rb.v[j] * inv;
        double p2 = sc;
        for (int b = 0; b < nsl; ++b) {
          p2 *= 1.0 / 256.0;
          uint4 *dst = (uint4 *)(sH + ((size_t)b * LEAF_TILE + scol) * SBH + sq * PERT);
#pragma unroll
          for (int j8 = 0; j8 < PERT / 8; ++j8) {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              uint32_t hv[2];
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                const int j = j8 * 8 + 2 * q + e;
                const double v = r[j] * 256.0, tr = trunc(v);
                r[j] = v - tr;
                hv[e] = bf16_bits(tr * p2);
              }
              w[q] = hv[0] | (hv[1] << 16);
            }
            dst[j8] = make_uint4(w[0], w[1], w[2], w[3]);
          }
        }
      } else {
        double *dst = sB + scol * SB + sq * PERT;
#pragma unroll
        for (int j = 0; j < PERT; ++j) dst[j] = rb.v[j];
      }
    }
    __syncthreads();
    int nsl2 = sl, nc = c + 1;
    if (nc >= NC) { ++nsl2; nc = 0; }
    if (nsl2 < s1) rb = leaf_chunk_load<KC>(slot_type, slot_src, fr, Lr, Mr, nsl2, nc, P, K2, sq, sinv_h2);
    if (type == 0) {
      // slice pairs (a, b) in order of d = a + b; one exact FP32 sum per group d
      const int op = slot_op[sl];
      flt4 g32[TPW][4];
#pragma unroll
      for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) g32[i][nt] = flt4{0, 0, 0, 0};
      uint4 an[TPW][NST];
#pragma unroll
      for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int st = 0; st < NST; ++st) an[i][st] = Ab[a_base(op, 0, i, c) + st * 64];
#pragma unroll
      for (int pi = 0; pi < SMAX * (SMAX + 1) / 2; ++pi) {
        // pair pi: group d, a = pi - d(d+1)/2, b = d - a
        int d = 0;
        while ((d + 1) * (d + 2) / 2 <= pi) ++d;
        const int a = pi - d * (d + 1) / 2, b = d - a;
        if (d >= nsl) break;
        bf16x8 av[TPW][NST];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
#pragma unroll
          for (int st = 0; st < NST; ++st) av[i][st] = __builtin_bit_cast(bf16x8, an[i][st]);
        {   // next pair's table slice in flight
          int d2 = 0;
          while ((d2 + 1) * (d2 + 2) / 2 <= pi + 1) ++d2;
          const int a2 = pi + 1 - d2 * (d2 + 1) / 2;
          if (pi + 1 < SMAX * (SMAX + 1) / 2 && d2 < nsl) {
#pragma unroll
            for (int i = 0; i < TPW; ++i)
#pragma unroll
              for (int st = 0; st < NST; ++st) an[i][st] = Ab[a_base(op, a2, i, c) + st * 64];
          }
        }
#pragma unroll
        for (int st = 0; st < NST; ++st)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const uint4 u = *(const uint4 *)(sH + ((size_t)b * LEAF_TILE + nt * 16 + col) * SBH + st * 32 + kq * 8);
            const bf16x8 bv = __builtin_bit_cast(bf16x8, u);
#pragma unroll
            for (int i = 0; i < TPW; ++i)
              if (d < tns[i]) g32[i][nt] = mfma_bf16(av[i][st], bv, g32[i][nt]);
          }
        if (a == d) {   // last pair of group d: add its exact sum
#pragma unroll
          for (int i = 0; i < TPW; ++i)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[i][nt][r] += (double)g32[i][nt][r];
              g32[i][nt] = flt4{0, 0, 0, 0};
            }
        }
      }
    } else {
      const double *A = leaf_frag + slot_aoff[sl];
#pragma unroll 4
      for (int ks = 0; ks < KSC; ++ks) {
        double av[TPW];
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          av[i] = A[(((size_t)(mtg + wave + 4 * (i < ni ? i : 0)) * NC + c) * KSC + ks) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const double b = sB[(nt * 16 + col) * SB + kq * KSC + ks];
#pragma unroll
          for (int i = 0; i < TPW; ++i)
            if (i < ni) acc[i][nt] = mfma4(av[i], b, acc[i][nt]);
        }
      }
    }
    sl = nsl2;
    c = nc;
  }
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
        const int row = mt * 16 + 4 * kq + r;
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
  if (g.n_units <= 0) return;
  const dim3 grid(g.n_units, 1, nrhs);      // one work unit per block (a multiple of the 8 XCDs)
  if (t.n == 4) {         // 3 row tiles, K chunks of 16
    hipLaunchKernelGGL((leaf_mfma_kernel<1, 16>), grid, dim3(256), 0, s, t, g, f, M, L, V, G);
  } else if (t.n == 8) {  // 12 row tiles: 3 per wave
    hipLaunchKernelGGL((leaf_mfma_kernel<3, 64>), grid, dim3(256), 0, s, t, g, f, M, L, V, G);
  } else {                // 48 row tiles: groups of 16, 4 per wave
    hipLaunchKernelGGL((leaf_mfma_kernel<4, 64>), grid, dim3(256), 0, s, t, g, f, M, L, V, G);
  }
}

void launch_leaf_split(const DevTables &t, const DevTree &g, const double *f, double *fscale, int nrhs,
                       const double *M, const double *L, double *V, double *G, hipStream_t s) {
  hipLaunchKernelGGL(leaf_scale_kernel, dim3(g.n_leaves, nrhs), dim3(64), 0, s, f, t.P, g.n_leaves, fscale);
  if (g.n_units <= 0) return;
  const dim3 grid(g.n_units, 1, nrhs);
  if (t.n == 8) {
    hipLaunchKernelGGL((leaf_split_kernel<3, 64>), grid, dim3(256), 0, s, t, g, f, fscale, M, L, V, G);
  } else {
    hipLaunchKernelGGL((leaf_split_kernel<4, 64>), grid, dim3(256), 0, s, t, g, f, fscale, M, L, V, G);
  }
}

}  // namespace bx
