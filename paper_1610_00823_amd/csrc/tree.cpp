// Host construction of the box hierarchy and interaction lists of a
// level-restricted quadtree (section 3.1: root at level 0, four children per
// split, adjacent leaves at most one level apart).
//
// The near field of a leaf B is the set of leaves touching B (the leaves whose
// interiors meet the 3h box around B); every other (source leaf, target)
// pair is covered exactly once by one of
//   U(B)  leaf B: adjacent leaves                      -> near tables
//   V(B)  any box: children of the parent's colleagues
//         that do not touch B                         -> multipole to local
//   W(B)  leaf B: children of B's colleagues that do
//         not touch B (with their descendants)         -> multipole to targets
//   X(B)  any box: leaves at the parent's level that
//         touch the parent but not B                    -> sources to local
// and the local expansions are passed down from parents to children.
#include <algorithm>
#include <chrono>
#include <unordered_map>

#include "bx_internal.h"

namespace bx {
namespace {

inline uint64_t morton(uint32_t x, uint32_t y) {
  uint64_t m = 0;
  for (int b = 0; b < 30; ++b) {
    m |= (uint64_t)((x >> b) & 1u) << (2 * b);
    m |= (uint64_t)((y >> b) & 1u) << (2 * b + 1);
  }
  return m;
}

// Do the closed squares (l1,x1,y1) and (l2,x2,y2) touch (corners included)?
inline bool touch(int l1, int64_t x1, int64_t y1, int l2, int64_t x2, int64_t y2) {
  int L = std::max(l1, l2);
  int64_t s1 = (int64_t)1 << (L - l1), s2 = (int64_t)1 << (L - l2);
  int64_t ax0 = x1 * s1, ax1 = ax0 + s1, ay0 = y1 * s1, ay1 = ay0 + s1;
  int64_t bx0 = x2 * s2, bx1 = bx0 + s2, by0 = y2 * s2, by1 = by0 + s2;
  return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

}  // namespace

int build_tree(HostTree &T, const bx_tree_desc &d, std::string &err) {
  const int NL = d.n_leaves;
  if (NL <= 0 || !d.level || !d.ix || !d.iy || !(d.width > 0)) {
    err = "tree descriptor: empty leaf set or null array or non-positive width";
    return BX_E_ARG;
  }
  T = HostTree();
  T.cx = d.cx; T.cy = d.cy; T.width = d.width; T.n_leaves = NL;
  int maxl = 0;
  for (int i = 0; i < NL; ++i) {
    int l = d.level[i];
    if (l < 0 || l > 29) { err = "leaf level outside 0..29"; return BX_E_INVALID_TREE; }
    int64_t m = (int64_t)1 << l;
    if (d.ix[i] < 0 || d.iy[i] < 0 || d.ix[i] >= m || d.iy[i] >= m) {
      err = "leaf position outside the root box";
      return BX_E_INVALID_TREE;
    }
    maxl = std::max(maxl, l);
  }
  // exact area: sum 4^(maxl - l) must equal 4^maxl
  {
    unsigned __int128 area = 0;
    for (int i = 0; i < NL; ++i) area += (unsigned __int128)1 << (2 * (maxl - d.level[i]));
    if (area != ((unsigned __int128)1 << (2 * maxl))) {
      err = area > ((unsigned __int128)1 << (2 * maxl)) ? "leaves overlap" : "leaves do not cover the root box";
      return BX_E_INVALID_TREE;
    }
  }
  std::unordered_map<uint64_t, int> leaf_at;   // key -> descriptor index
  leaf_at.reserve(NL * 2);
  for (int i = 0; i < NL; ++i) {
    uint64_t k = box_key(d.level[i], d.ix[i], d.iy[i]);
    if (!leaf_at.emplace(k, i).second) { err = "repeated leaf"; return BX_E_INVALID_TREE; }
  }
  std::unordered_map<uint64_t, int> internal;   // key -> placeholder
  internal.reserve(NL);
  for (int i = 0; i < NL; ++i) {
    int l = d.level[i];
    int64_t x = d.ix[i], y = d.iy[i];
    while (l > 0) {
      --l; x >>= 1; y >>= 1;
      uint64_t k = box_key(l, x, y);
      if (leaf_at.count(k)) { err = "a leaf contains another leaf"; return BX_E_INVALID_TREE; }
      if (!internal.emplace(k, 0).second) break;
    }
  }
  // boxes sorted by (level, Morton)
  struct Bx { int l, x, y, leaf; uint64_t m; };
  std::vector<Bx> boxes;
  boxes.reserve(NL + internal.size());
  for (int i = 0; i < NL; ++i) boxes.push_back({d.level[i], d.ix[i], d.iy[i], i, 0});
  for (auto &kv : internal) {
    uint64_t k = kv.first;
    boxes.push_back({(int)(k >> 58), (int)((k >> 29) & ((1u << 29) - 1)), (int)(k & ((1u << 29) - 1)), -1, 0});
  }
  for (auto &b : boxes) b.m = morton(b.x, b.y);
  std::sort(boxes.begin(), boxes.end(), [](const Bx &a, const Bx &b) {
    return a.l != b.l ? a.l < b.l : a.m < b.m;
  });
  const int NB = (int)boxes.size();
  T.n_boxes = NB;
  T.n_levels = maxl + 1;
  T.lvl.resize(NB); T.bx.resize(NB); T.by.resize(NB);
  T.parent.assign(NB, -1); T.child0.assign(NB, -1); T.leaf_of_box.resize(NB);
  T.box_of_leaf.assign(NL, -1);
  T.level_start.assign(T.n_levels + 1, 0);
  std::unordered_map<uint64_t, int> id;
  id.reserve(NB * 2);
  for (int b = 0; b < NB; ++b) {
    T.lvl[b] = boxes[b].l; T.bx[b] = boxes[b].x; T.by[b] = boxes[b].y;
    T.leaf_of_box[b] = boxes[b].leaf;
    if (boxes[b].leaf >= 0) T.box_of_leaf[boxes[b].leaf] = b;
    id[box_key(boxes[b].l, boxes[b].x, boxes[b].y)] = b;
    T.level_start[boxes[b].l + 1] = b + 1;
  }
  for (int l = 1; l <= T.n_levels; ++l) T.level_start[l] = std::max(T.level_start[l], T.level_start[l - 1]);
  auto find = [&](int l, int64_t x, int64_t y) -> int {
    if (l < 0 || x < 0 || y < 0 || x >= ((int64_t)1 << l) || y >= ((int64_t)1 << l)) return -1;
    auto it = id.find(box_key(l, x, y));
    return it == id.end() ? -1 : it->second;
  };
  for (int b = 0; b < NB; ++b) {
    if (T.lvl[b] > 0) T.parent[b] = find(T.lvl[b] - 1, T.bx[b] >> 1, T.by[b] >> 1);
    if (T.leaf_of_box[b] < 0) {
      int c = find(T.lvl[b] + 1, 2 * T.bx[b], 2 * T.by[b]);
      // Morton order keeps the four children contiguous: (0,0), (1,0), (0,1), (1,1)
      T.child0[b] = c;
      for (int q = 0; q < 4; ++q)
        if (find(T.lvl[b] + 1, 2 * T.bx[b] + (q & 1), 2 * T.by[b] + (q >> 1)) != c + q) {
          err = "internal error: children not contiguous";
          return BX_E_INVALID_TREE;
        }
    }
  }
  // level restriction: a leaf's neighbours at its own level either exist and,
  // if subdivided, have leaf children wherever they touch it, or are covered by
  // a leaf one level up.
  for (int b = 0; b < NB; ++b) {
    if (T.leaf_of_box[b] < 0) continue;
    int l = T.lvl[b];
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        int64_t nx = T.bx[b] + dx, ny = T.by[b] + dy;
        if (nx < 0 || ny < 0 || nx >= ((int64_t)1 << l) || ny >= ((int64_t)1 << l)) continue;
        int nb = find(l, nx, ny);
        if (nb < 0) {
          if (find(l - 1, nx >> 1, ny >> 1) < 0) { err = "tree is not level-restricted"; return BX_E_NOT_BALANCED; }
        } else if (T.leaf_of_box[nb] < 0) {
          for (int q = 0; q < 4; ++q) {
            int c = T.child0[nb] + q;
            if (touch(l, T.bx[b], T.by[b], l + 1, T.bx[c], T.by[c]) && T.leaf_of_box[c] < 0) {
              err = "tree is not level-restricted";
              return BX_E_NOT_BALANCED;
            }
          }
        }
      }
  }
  // --------------------------------------------------------------- lists
  Rel cfg[NCFG_U];
  u_configs(cfg);
  int pa[NCFG_W], pb[NCFG_W];
  wx_positions(pa, pb);
  auto u_config = [&](int tb, int sb) -> int {
    // relative centre and width of the source in units of the target width
    int lt = T.lvl[tb], ls = T.lvl[sb], L = std::max(lt, ls);
    double st = std::ldexp(1.0, L - lt), ss = std::ldexp(1.0, L - ls);
    double tcx = (T.bx[tb] + 0.5) * st, tcy = (T.by[tb] + 0.5) * st;
    double scx = (T.bx[sb] + 0.5) * ss, scy = (T.by[sb] + 0.5) * ss;
    double rx = (scx - tcx) / st, ry = (scy - tcy) / st, rw = ss / st;
    for (int c = 0; c < NCFG_U; ++c)
      if (cfg[c].cx == rx && cfg[c].cy == ry && cfg[c].w == rw) return c;
    return -1;
  };
  auto wx_config = [&](int64_t a, int64_t b) -> int {
    for (int c = 0; c < NCFG_W; ++c)
      if (pa[c] == a && pb[c] == b) return c;
    return -1;
  };
  for (int b = 0; b < NB; ++b) {
    int l = T.lvl[b];
    int64_t x = T.bx[b], y = T.by[b];
    bool leaf = T.leaf_of_box[b] >= 0;
    if (leaf) {
      int tl = T.leaf_of_box[b];
      std::vector<int> seen;
      auto add_u = [&](int sb) {
        if (std::find(seen.begin(), seen.end(), sb) != seen.end()) return;
        seen.push_back(sb);
        T.u_t.push_back(tl); T.u_s.push_back(T.leaf_of_box[sb]); T.u_c.push_back(u_config(b, sb));
      };
      add_u(b);
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy) continue;
          int64_t nx = x + dx, ny = y + dy;
          if (nx < 0 || ny < 0 || nx >= ((int64_t)1 << l) || ny >= ((int64_t)1 << l)) continue;
          int nb = find(l, nx, ny);
          if (nb < 0) {
            add_u(find(l - 1, nx >> 1, ny >> 1));   // coarse leaf
          } else if (T.leaf_of_box[nb] >= 0) {
            add_u(nb);
          } else {
            for (int q = 0; q < 4; ++q) {
              int c = T.child0[nb] + q;
              if (touch(l, x, y, l + 1, T.bx[c], T.by[c])) add_u(c);
              else {  // W: a child of a colleague that does not touch the leaf
                T.w_t.push_back(tl); T.w_s.push_back(c);
                T.w_c.push_back(wx_config(T.bx[c] - 2 * x, T.by[c] - 2 * y));
              }
            }
          }
        }
    }
    if (l >= 2) {   // V: children of the parent's colleagues that do not touch b
      int pbx = (int)(x >> 1), pby = (int)(y >> 1);
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy) continue;
          int nb = find(l - 1, pbx + dx, pby + dy);
          if (nb < 0 || T.leaf_of_box[nb] >= 0) continue;
          for (int q = 0; q < 4; ++q) {
            int c = T.child0[nb] + q;
            int ox = T.bx[c] - (int)x, oy = T.by[c] - (int)y;
            if (std::max(std::abs(ox), std::abs(oy)) < 2) continue;
            T.v_t.push_back(b); T.v_s.push_back(c); T.v_c.push_back((oy + 3) * 7 + (ox + 3));
          }
        }
    }
    if (l >= 1) {   // X: leaves at the parent's level touching the parent but not b
      int pbx = (int)(x >> 1), pby = (int)(y >> 1);
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy) continue;
          int nb = find(l - 1, pbx + dx, pby + dy);
          if (nb < 0 || T.leaf_of_box[nb] < 0) continue;
          if (touch(l, x, y, l - 1, T.bx[nb], T.by[nb])) continue;
          T.x_t.push_back(b); T.x_s.push_back(T.leaf_of_box[nb]);
          T.x_c.push_back(wx_config(x - 2 * (int64_t)T.bx[nb], y - 2 * (int64_t)T.by[nb]));
        }
    }
  }
  for (size_t i = 0; i < T.u_c.size(); ++i)
    if (T.u_c[i] < 0) { err = "internal error: unknown near configuration"; return BX_E_NOT_BALANCED; }
  for (size_t i = 0; i < T.w_c.size(); ++i)
    if (T.w_c[i] < 0) { err = "internal error: unknown W configuration"; return BX_E_INVALID_TREE; }
  for (size_t i = 0; i < T.x_c.size(); ++i)
    if (T.x_c[i] < 0) { err = "internal error: unknown X configuration"; return BX_E_INVALID_TREE; }
  return BX_OK;
}

// A forest as one tree structure: boxes level-major (all trees' level-l boxes
// together, tree after tree, each in its own order, so children stay
// contiguous), leaves in descriptor order tree after tree, every list index
// offset into the merged numbering.  The trees must share the root width (the
// operators depend on the box widths); their interaction lists never meet.
int merge_forest(const std::vector<HostTree> &P, HostTree &T, std::vector<int> &box_tree, std::string &err) {
  T = HostTree();
  T.width = P[0].width;
  T.cx = P[0].cx;
  T.cy = P[0].cy;
  const int K = (int)P.size();
  std::vector<int> leaf_off(K + 1, 0);
  for (int k = 0; k < K; ++k) {
    if (P[k].width != T.width) {
      err = "trees of a forest must share the root width";
      return BX_E_UNSUPPORTED;
    }
    T.n_levels = std::max(T.n_levels, P[k].n_levels);
    leaf_off[k + 1] = leaf_off[k] + P[k].n_leaves;
  }
  T.n_leaves = leaf_off[K];
  std::vector<std::vector<int>> gid(K);
  for (int k = 0; k < K; ++k) gid[k].assign(P[k].n_boxes, -1);
  T.level_start.assign(T.n_levels + 1, 0);
  int nb = 0;
  for (int l = 0; l < T.n_levels; ++l) {
    T.level_start[l] = nb;
    for (int k = 0; k < K; ++k)
      if (l < P[k].n_levels)
        for (int b = P[k].level_start[l]; b < P[k].level_start[l + 1]; ++b) gid[k][b] = nb++;
  }
  T.level_start[T.n_levels] = nb;
  T.n_boxes = nb;
  T.lvl.assign(nb, 0); T.bx.assign(nb, 0); T.by.assign(nb, 0);
  T.parent.assign(nb, -1); T.child0.assign(nb, -1); T.leaf_of_box.assign(nb, -1);
  T.box_of_leaf.assign(T.n_leaves, -1);
  box_tree.assign(nb, 0);
  for (int k = 0; k < K; ++k) {
    const HostTree &Q = P[k];
    for (int b = 0; b < Q.n_boxes; ++b) {
      const int g = gid[k][b];
      T.lvl[g] = Q.lvl[b]; T.bx[g] = Q.bx[b]; T.by[g] = Q.by[b];
      T.parent[g] = Q.parent[b] >= 0 ? gid[k][Q.parent[b]] : -1;
      T.child0[g] = Q.child0[b] >= 0 ? gid[k][Q.child0[b]] : -1;
      T.leaf_of_box[g] = Q.leaf_of_box[b] >= 0 ? leaf_off[k] + Q.leaf_of_box[b] : -1;
      box_tree[g] = k;
    }
    for (int i = 0; i < Q.n_leaves; ++i) T.box_of_leaf[leaf_off[k] + i] = gid[k][Q.box_of_leaf[i]];
    auto leaf = [&](int i) { return leaf_off[k] + i; };
    auto box = [&](int b) { return gid[k][b]; };
    for (size_t e = 0; e < Q.u_t.size(); ++e) {
      T.u_t.push_back(leaf(Q.u_t[e])); T.u_s.push_back(leaf(Q.u_s[e])); T.u_c.push_back(Q.u_c[e]);
    }
    for (size_t e = 0; e < Q.v_t.size(); ++e) {
      T.v_t.push_back(box(Q.v_t[e])); T.v_s.push_back(box(Q.v_s[e])); T.v_c.push_back(Q.v_c[e]);
    }
    for (size_t e = 0; e < Q.w_t.size(); ++e) {
      T.w_t.push_back(leaf(Q.w_t[e])); T.w_s.push_back(box(Q.w_s[e])); T.w_c.push_back(Q.w_c[e]);
    }
    for (size_t e = 0; e < Q.x_t.size(); ++e) {
      T.x_t.push_back(box(Q.x_t[e])); T.x_s.push_back(leaf(Q.x_s[e])); T.x_c.push_back(Q.x_c[e]);
    }
  }
  return BX_OK;
}

}  // namespace bx
