// Device kernels of the box code and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

namespace bx {

// Device copies of the unit-box operators (see bx_internal.h for layouts).
struct DevTables {
  int n, P, p, nt, KP, MR;
  const double *wq, *near_, *p2m, *m2m, *l2l, *H, *pw_src, *pw_tgt, *logd, *l2t, *m2t, *p2l;
  // Fragment-major A operands of the fused leaf GEMM (near tables, L2T, W) and of P2M:
  // frag[((op * MT + mt) * KS + ks) * 64 + lane] = A[mt*16 + lane%16][(lane/16) * KS + ks],
  // K = 4 KS; the k index is split so that each lane's B operand is contiguous.
  const double *leaf_frag, *p2m_frag;
  const double *leaf_mass;   // [54][KMAX] mass-row weights of the leaf operators
  int leaf_kmax;
  int leaf_kc;               // K chunk width of the leaf fragments (divides P and 2 KP)
  // split contexts: int8 slices of the near tables (layout in bx_internal.h),
  // the per-row scales 2^E_r [3P] and the mass factors w_c^2 of the 33 configurations
  const int8_t *near_i8;
  const double *split_row_scale, *split_cfg_w2;
  // M2M 4 x [2KP][2KP] and L2L 4 x [2KP][2KP] on interleaved coefficients, and
  // P2L per X configuration [2KP + mass row, padded][P], all fragment-major.
  const double *m2m_frag, *l2l_frag, *p2l_frag;
};

// Device copy of a tree's hierarchy and lists (CSR by target, sorted).
constexpr int M2L_VMAX = 32;   // longest V list (27) rounded up to 4 groups of 8

struct DevTree {
  int n_leaves, n_boxes, n_levels;
  double width, cx, cy;      // root width and centre (of the first tree of a forest)
  int n_roots;               // level-0 boxes: 1, or the trees of a forest
  const int *lvl;          // [NB]
  const int *child0;       // [NB]
  const int *parent;       // [NB]
  const int *leaf_of_box;  // [NB]
  const int *box_of_leaf;  // [NL]
  const int *leaf_level;   // [NL]
  // U: per target leaf, CSR of (source leaf, config)
  const int *u_ptr, *u_src, *u_cfg;
  // V: per target box, CSR of (source box, offset class, slot of the source in
  // the 6 x 6 grid of its target's parent)
  const int *v_ptr, *v_src, *v_cfg, *v_slot;
  // M2L sibling groups: the internal boxes and their 6 x 6 grids (box or -1)
  int n_m2l_par, m2l_blocks;   // sibling groups, persistent M2L blocks
  const int *m2l_par;      // [n_m2l_par]
  const int *m2l_grid;     // [n_m2l_par][36]
  const int *m2l_ent;      // [n_m2l_par][4 children][M2L_VMAX]: grid slot | offset class << 8, or -1
  const int *m2l_info;     // [n_m2l_par][2]: first child box, child level
  // W: per target leaf, CSR of (source box, config)
  const int *w_ptr, *w_src, *w_cfg;
  // X: per target box, CSR of (source leaf, config)
  const int *x_ptr, *x_src, *x_cfg;
  // X-list GEMM tiles: 16 target boxes per tile, slots = union of X configurations
  int n_xtiles;
  const int *xtile_box;    // [n_xtiles][16], -1 = padding
  const int *xtile_ptr;    // [n_xtiles + 1]
  const int *xslot_cfg;    // [n_xslots]
  const int *xslot_src;    // [n_xslots][16] source leaf, -1 = none
  // fused leaf GEMM tiling: 64-target tiles; each slot is one A operand (a near
  // table, L2T or a W configuration) applied to 64 gathered B columns
  int n_tiles;
  const int *tile_tgt;     // [n_tiles][64], -1 = padding
  const int *tile_ptr;     // [n_tiles + 1] into slots
  const int *slot_aoff;    // [n_slots] offset of the A fragments in leaf_frag
  const int *slot_op;      // [n_slots] operator index (near c, 33 = L2T, 34 + W c)
  const int *slot_type;    // [n_slots] 0: samples f of a source leaf (K = P); 1: local expansion
                           // of the target's box; 2: multipole of a source box (K = 2 KP)
  const int *slot_src;     // [n_slots][64] leaf or box index, -1 = none
  const int *tile_nsl;     // [n_tiles] split contexts: slices of the V rows | gradient rows << 8 (tiles of one
                           // level); 0 for a tile whose near field runs in FP64
  // work units of the leaf kernels in launch order (one block each): tile (-1 =
  // empty block) and first row tile | (row tiles per wave) << 16
  int n_units;
  const int *unit_tile, *unit_mt;
  // split contexts: the U slots of each tile for the int8 kernel (the FP64 slots
  // above then hold L2T, the W list and the U slots of tiles left in FP64), its
  // work units (tile, first row tile) and the number of sample slices
  const int *nslot_ptr;    // [n_tiles + 1]
  const int *nslot_cfg;    // [n_nslots]
  const int *nslot_src;    // [n_nslots][64] source leaf, -1 = none
  int n_nunits, split_sf;
  const int *nunit_tile, *nunit_mt;
};

// Expansion storage: [n_rhs][NB][KP] complex (interleaved re, im).
void launch_p2m(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *M, hipStream_t s);
// Upward pass step for the internal boxes `boxes` of one level.
void launch_m2m(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int child_base, int nrhs,
                double *M, hipStream_t s);   // child_base: see m2m_mfma_kernel (-1: look children up)
// two levels per launch: boxes = internal boxes of the upper level
void launch_m2m2(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *M,
                 hipStream_t s);
void launch_l2l2(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *L,
                 hipStream_t s);
void launch_m2l(const DevTables &t, const DevTree &g, int nrhs, const double *M, double *L, hipStream_t s);
void launch_p2l(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *L, hipStream_t s);
// Downward pass step from the internal boxes `boxes` of one level to their children.
void launch_l2l(const DevTables &t, const DevTree &g, const int *boxes, int nbox, int nrhs, double *L,
                hipStream_t s);
// Near tables + L2T + W list for every leaf (the slots of the tree's tiles):
// writes V and G, or adds to them when accumulate is set.
void launch_leaf(const DevTables &t, const DevTree &g, const double *f, int nrhs, const double *M,
                 const double *L, double *V, double *G, bool accumulate, hipStream_t s);
// Split precision: per-RHS sample scale fscale [n_rhs], int8 sample slices fsl
// [n_rhs][split_sf][N_L][P] and per-leaf masses lmass [n_rhs][N_L]; fpart holds
// [n_rhs][512] partial maxima.
void launch_split_prep(const DevTables &t, const DevTree &g, const double *f, int nrhs, double *fpart,
                       double *fscale, int8_t *fsl, double *lmass, hipStream_t s);
// Split precision leaf phase: int8 near field of every tile, then (in the same
// kernel, FP64) L2T, the W list and the near field of tiles left in FP64; writes V and G.
void launch_leaf_split(const DevTables &t, const DevTree &g, const int8_t *fsl, const double *lmass,
                       const double *fscale, const double *f, int nrhs, const double *M, const double *L, double *V,
                       double *G, hipStream_t s);

// Interpolants of V and G (either may be null) at n_targets points xy [n][2]:
// v_out [n_rhs][n], g_out [n_rhs][n][2]; NaN outside the root box.
void launch_interpolate(const DevTables &t, const DevTree &g, const double *V, const double *G, int nrhs,
                        const double *xy, long long n_targets, double *v_out, double *g_out, hipStream_t s);

}  // namespace bx
