// Internal declarations of the box-code library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/boxfmm.h"

namespace bx {

constexpr int NCFG_U = 33;   // near (U-list) configurations of a level-restricted tree
constexpr int NCFG_W = 20;   // fine non-adjacent boxes whose parents are adjacent (W list)
constexpr int NCFG_X = 20;   // coarse non-adjacent leaves adjacent to the parent (X list)
constexpr int NOFF = 49;     // 7 x 7 same-level offsets; the 40 with max(|dx|,|dy|) >= 2 are V-list classes

// Geometry of a source box relative to a unit target box centred at 0.
struct Rel {
  double cx, cy, w;
};
void u_configs(Rel out[NCFG_U]);
// W and X positions: lower-left (a, b) of the smaller box relative to the
// lower-left of the larger one, in units of the smaller box's width.
void wx_positions(int a[NCFG_W], int b[NCFG_W]);

// Unit-box operators in FP64 (host).  KP = expansion length padded to 16.
struct Tables {
  int n = 0, P = 0, p = 0, nt = 0, KP = 0;
  int MR = 0;                      // near rows: 3P + 1 (mass row) padded to 16
  std::vector<double> wq;          // [P] weights int L_j over the unit box
  std::vector<double> near_;       // [33][MR][P]: rows V (P), d1 (P), d2 (P), mass (1)
  std::vector<double> p2m;         // [2 KP][P]: Re a_k rows then Im a_k rows
  std::vector<double> m2m;         // [4][nt][nt][2] complex, child position c = cx + 2 cy
  std::vector<double> l2l;         // [4][nt][nt][2] complex
  std::vector<double> H;           // [KP][KP] real, M2L core (row l, column k)
  std::vector<double> pw_src;      // [49][KP][2] (-d/2)^-k
  std::vector<double> pw_tgt;      // [49][KP][2] (d/2)^-l
  std::vector<double> logd;        // [49] log|d|
  std::vector<double> l2t;         // [3P][2 KP]: columns Re b_l then Im b_l
  std::vector<double> m2t;         // [20][3P][2 KP]
  std::vector<double> p2l;         // [20][2 KP][P]
};

int build_tables(Tables &T, int n, int p, double tol, int nthreads);

// Fragment-major A operands of the fused leaf GEMM: 33 near tables (K = P),
// then L2T, then the 20 W operators (K = 2 KP); 3P rows each (V, dV/dx1,
// dV/dx2).  K is cut into chunks of KC = min(64, P) columns:
// frag[((mt * NC + c) * KSC + ks) * 64 + lane] = A[mt*16 + lane%16][c*KC + (lane/16)*KSC + ks],
// NC = K / KC, KSC = KC / 4.  The mass row of each operator (its weights for
// the log h term) is kept apart: mass[op][k], op = near c, 33 = L2T, 34 + W c.
struct LeafFragLayout {
  int MTR, KC, KMAX;         // row tiles, chunk width, mass-vector stride
  int64_t near0, near_step, l2t, w0, w_step, total;
};
LeafFragLayout leaf_frag_layout(int n, int p);
void build_leaf_frag(const Tables &T, std::vector<double> &out, std::vector<double> &mass);

// Split (int8-slice) form of the near tables.  Row r of every near table has
// one power-of-two scale 2^E_r (max |T[r][k]| over configurations and k is at
// most 2^E_r 127.5/128); a value is x = 2^E_r sum_a t_a 2^-7(a+1) + residual
// with integer slices t_a rounded to nearest (|t_0| <= 127, |t_a| <= 64 after).
// Fragments for v_mfma_i32_16x16x64_i8 (16 bytes per lane):
// a[((((c * SMAX + a) * MTR + mt) * NCH + ch) * 64 + lane) * 16 + e]
//   = slice a of T_c[mt*16 + lane%16][ch*64 + (lane/16)*16 + e],  MTR = 3P/16, NCH = P/64.
constexpr int SPLIT_SMAX = 8;   // table slices stored
constexpr int SPLIT_SG = 6;     // slice count the int8 kernel handles; tiles needing more stay FP64
struct SplitTables {
  std::vector<int8_t> a;
  std::vector<double> row_scale;      // [3P] 2^E_r
  std::vector<double> err_v, err_d;   // [SMAX + 1]: error bound with s slices for samples |f| < 1, per row type
  std::vector<double> cfg_w2;         // [33] mass weight factor (source width / target width)^2
};
void build_split_tables(const Tables &T, SplitTables &S);
// Slices needed at level l so that the slice error stays below tol times
// ||f||_inf W^2 (values) or ||f||_inf W (gradients), W the root width; 0 when
// more than SPLIT_SG would be needed.
int split_slices(const SplitTables &S, int level, double tol, bool grad_rows);
void build_p2m_frag(const Tables &T, std::vector<double> &out);
// M2M 4 x [2KP][2KP], L2L 4 x [2KP][2KP] on interleaved coefficients, and the
// 20 P2L operators [2KP + mass row, padded to 16][P], fragment-major.
void build_m2m_frag(const Tables &T, std::vector<double> &out);
void build_l2l_frag(const Tables &T, std::vector<double> &out);
void build_p2l_frag(const Tables &T, std::vector<double> &out);
uint64_t tables_checksum(const Tables &T);
bool save_tables(const Tables &T, const std::string &path);
bool load_tables(Tables &T, const std::string &path, int n, int p);

// Host tree: box hierarchy and interaction lists.
inline uint64_t box_key(int l, int64_t x, int64_t y) {
  return ((uint64_t)l << 58) | ((uint64_t)x << 29) | (uint64_t)y;
}

struct HostTree {
  double cx = 0, cy = 0, width = 1;
  int n_leaves = 0, n_boxes = 0, n_levels = 0;
  std::vector<int> lvl, bx, by;           // per box (sorted by level, then Morton)
  std::vector<int> parent, child0;        // child0 = first of 4 contiguous children, -1 for a leaf
  std::vector<int> leaf_of_box;           // descriptor index, -1 for internal boxes
  std::vector<int> box_of_leaf;           // [n_leaves]
  std::vector<int> level_start;           // [n_levels + 1]
  // lists: (target, source, config)
  std::vector<int> u_t, u_s, u_c;         // target leaf, source leaf (descriptor indices)
  std::vector<int> v_t, v_s, v_c;         // target box, source box, offset class (0..48)
  std::vector<int> w_t, w_s, w_c;         // target leaf, source box, config
  std::vector<int> x_t, x_s, x_c;         // target box, source leaf, config
};

int build_tree(HostTree &T, const bx_tree_desc &d, std::string &err);
// Several trees as one structure (level-major boxes, leaves tree after tree);
// box_tree[b] receives the tree of each merged box.
int merge_forest(const std::vector<HostTree> &parts, HostTree &T, std::vector<int> &box_tree, std::string &err);

void set_error(const std::string &msg);

}  // namespace bx
