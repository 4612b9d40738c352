// C ABI of the box-code library: contexts, table build/upload, tree upload
// and the stream-ordered evaluation of V and grad V.
#include <algorithm>
#include <unordered_map>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bx_internal.h"
#include "kernels.h"
#include "mlp.h"

struct bx_ctx {
  int n = 0, p = 0, device = 0;
  int n_cu = 256;                        // compute units of the device
  uint32_t flags = 0;
  double split_tol = 1e-11;              // slice-truncation tolerance of the split near tables
  bx::SplitTables split;
  bool ready = false;
  bool profiling = false;
  std::vector<hipEvent_t> ev;            // recorded event pairs, phase-tagged
  std::vector<int> ev_phase;
  int ev_evals = 0;
  hipStream_t capture_stream = nullptr;  // private stream used only to capture graphs
  bx::Tables T;
  std::vector<void *> dev;    // device allocations owned by the context
  bx::DevTables dt{};
};

struct GraphEntry {
  const double *f = nullptr;
  double *V = nullptr, *G = nullptr;
  int nrhs = 0;
  hipGraphExec_t exec = nullptr;
};

struct bx_tree {
  bx_ctx *ctx = nullptr;
  GraphEntry graphs[4];                  // captured evaluations, keyed by (f, V, G, n_rhs)
  int graph_next = 0;
  bx::HostTree H;
  std::vector<int> int_start;            // per level: offset of its internal boxes in int_boxes
  std::vector<int> int_child_base;       // per level: first child of its internal boxes if contiguous, else -1
  const int *int_boxes = nullptr;        // device
  std::vector<void *> dev;
  bx::DevTree dg{};
  double *M = nullptr, *L = nullptr;   // expansions, grown with n_rhs
  // split contexts: per-RHS sample scales, partial maxima, int8 sample slices, per-leaf masses
  double *fscale = nullptr, *fpart = nullptr, *lmass = nullptr;
  int8_t *fsl = nullptr;
  int split_sf = 1;
  int exp_rhs = 0;
  double upload_ms = 0.0;
  int64_t n_slots = 0;
  int n_trees = 1;
  std::vector<int> box_tree;           // tree of each box (forests)
  // host copies of the tilings, for rebuilding the work units (autotuning)
  std::vector<int> h_tile_ptr, h_nslot_ptr, h_tile_nsl;
  bool split = false;
  std::vector<void *> unit_bufs;       // device work-unit arrays
  double tune_heavy = 1.0;             // heavy-tile threshold, in balanced shares of a resident block (1.5 split)
  double tune_f64_weight = 16.0;       // split kernel: an FP64 slot's cost in int8 slice pairs
  int tune_m2l_blocks = 4096;          // persistent M2L blocks
  int tune_fuse = 0;                // two-level M2M / L2L launches when the middle level has at most this many internal boxes
};

struct bx_mlp {
  bx::MlpDev d{};
  int step = 0;          // Adam steps since the parameters were set
  void *block = nullptr; // one allocation for every buffer
};

namespace bx {
namespace {
thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(BX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class Tv>
int upload(std::vector<void *> &owned, const std::vector<Tv> &h, const Tv **out, hipStream_t s) {
  *out = nullptr;
  if (h.empty()) {  // keep a valid pointer for empty lists
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, 16);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(BX_E_OOM, "hipMalloc") : hip_fail(e, "hipMalloc");
    owned.push_back(p);
    *out = (const Tv *)p;
    return BX_OK;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, h.size() * sizeof(Tv));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(BX_E_OOM, "hipMalloc") : hip_fail(e, "hipMalloc");
  owned.push_back(p);
  e = hipMemcpyAsync(p, h.data(), h.size() * sizeof(Tv), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  *out = (const Tv *)p;
  return BX_OK;
}

// CSR by target from (target, source, config) triples.
void csr(int ntgt, const std::vector<int> &t, const std::vector<int> &s, const std::vector<int> &c,
         std::vector<int> &ptr, std::vector<int> &src, std::vector<int> &cfg) {
  ptr.assign(ntgt + 1, 0);
  for (int x : t) ptr[x + 1]++;
  for (int i = 0; i < ntgt; ++i) ptr[i + 1] += ptr[i];
  std::vector<int> pos(ptr.begin(), ptr.end() - 1);
  src.resize(t.size());
  cfg.resize(t.size());
  for (size_t i = 0; i < t.size(); ++i) {
    int k = pos[t[i]]++;
    src[k] = s[i];
    cfg[k] = c[i];
  }
}

}  // namespace

void set_error(const std::string &msg) { g_err = msg; }

}  // namespace bx

using namespace bx;

extern "C" {

const char *bx_last_error(void) { return g_err.c_str(); }

int bx_create(bx_ctx **out, int n_nodes, int p_exp, uint32_t flags) {
  if (!out) return fail(BX_E_ARG, "bx_create: out is NULL");
  *out = nullptr;
  if (n_nodes != 4 && n_nodes != 8 && n_nodes != 16) return fail(BX_E_UNSUPPORTED, "bx_create: n must be 4, 8 or 16");
  if (p_exp < 8 || p_exp > 47) return fail(BX_E_UNSUPPORTED, "bx_create: p must be in 8..47");
  uint32_t prec = flags & ~(uint32_t)BX_HOST_ONLY;
  if (prec != BX_FP64 && prec != BX_SPLIT_INT8) return fail(BX_E_UNSUPPORTED, "bx_create: unknown flags");
  if (prec == BX_SPLIT_INT8 && n_nodes == 4)
    return fail(BX_E_UNSUPPORTED, "bx_create: split near tables need n = 8 or 16");
  int dev = 0;
  if (!(flags & BX_HOST_ONLY)) {
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  }
  int n_cu = 256;
  if (!(flags & BX_HOST_ONLY)) {
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  }
  bx_ctx *c = new (std::nothrow) bx_ctx;
  if (!c) return fail(BX_E_OOM, "bx_create");
  c->n = n_nodes;
  c->p = p_exp;
  c->flags = flags;
  c->device = dev;
  c->n_cu = n_cu;
  *out = c;
  return BX_OK;
}

int bx_build_tables(bx_ctx *ctx, double quad_tol, const char *cache_dir) {
  if (!ctx) return fail(BX_E_ARG, "bx_build_tables: ctx is NULL");
  double tol = quad_tol > 0 ? quad_tol : 1e-15;
  Tables &T = ctx->T;
  bool loaded = false;
  std::string path;
  if (cache_dir && *cache_dir) {
    char name[128];
    std::snprintf(name, sizeof name, "/boxfmm_tables_n%d_p%d.bin", ctx->n, ctx->p);
    path = std::string(cache_dir) + name;
    loaded = load_tables(T, path, ctx->n, ctx->p);
  }
  if (!loaded) {
    int rc = build_tables(T, ctx->n, ctx->p, tol, 0);
    if (rc) return fail(rc, "bx_build_tables: table construction failed");
    if (!path.empty()) save_tables(T, path);   // a failed cache write is not an error
  }
  if (ctx->flags & BX_SPLIT_INT8) build_split_tables(T, ctx->split);
  if (ctx->flags & BX_HOST_ONLY) {
    ctx->ready = true;
    return BX_OK;
  }
  for (void *p : ctx->dev) (void)hipFree(p);
  ctx->dev.clear();
  DevTables &d = ctx->dt;
  d.n = T.n; d.P = T.P; d.p = T.p; d.nt = T.nt; d.KP = T.KP; d.MR = T.MR;
  hipStream_t s = nullptr;
  int rc = 0;
  if ((rc = upload(ctx->dev, T.wq, &d.wq, s)) || (rc = upload(ctx->dev, T.near_, &d.near_, s)) ||
      (rc = upload(ctx->dev, T.p2m, &d.p2m, s)) || (rc = upload(ctx->dev, T.m2m, &d.m2m, s)) ||
      (rc = upload(ctx->dev, T.l2l, &d.l2l, s)) || (rc = upload(ctx->dev, T.H, &d.H, s)) ||
      (rc = upload(ctx->dev, T.pw_src, &d.pw_src, s)) || (rc = upload(ctx->dev, T.pw_tgt, &d.pw_tgt, s)) ||
      (rc = upload(ctx->dev, T.logd, &d.logd, s)) || (rc = upload(ctx->dev, T.l2t, &d.l2t, s)) ||
      (rc = upload(ctx->dev, T.m2t, &d.m2t, s)) || (rc = upload(ctx->dev, T.p2l, &d.p2l, s)))
    return rc;
  std::vector<double> lf, lm, pf, mf, llf, xf;
  build_leaf_frag(T, lf, lm);
  build_p2m_frag(T, pf);
  build_m2m_frag(T, mf);
  build_l2l_frag(T, llf);
  build_p2l_frag(T, xf);
  d.leaf_kmax = leaf_frag_layout(T.n, T.p).KMAX;
  d.leaf_kc = leaf_frag_layout(T.n, T.p).KC;
  if ((rc = upload(ctx->dev, lf, &d.leaf_frag, s)) || (rc = upload(ctx->dev, lm, &d.leaf_mass, s)) ||
      (rc = upload(ctx->dev, pf, &d.p2m_frag, s)) ||
      (rc = upload(ctx->dev, mf, &d.m2m_frag, s)) || (rc = upload(ctx->dev, llf, &d.l2l_frag, s)) ||
      (rc = upload(ctx->dev, xf, &d.p2l_frag, s)))
    return rc;
  d.near_i8 = nullptr;
  d.split_row_scale = d.split_cfg_w2 = nullptr;
  if ((ctx->flags & BX_SPLIT_INT8) &&
      ((rc = upload(ctx->dev, ctx->split.a, &d.near_i8, s)) ||
       (rc = upload(ctx->dev, ctx->split.row_scale, &d.split_row_scale, s)) ||
       (rc = upload(ctx->dev, ctx->split.cfg_w2, &d.split_cfg_w2, s))))
    return rc;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "bx_build_tables: upload");
  ctx->ready = true;
  return BX_OK;
}

namespace bx {
namespace {
struct Unit {
  int tile, mt;
  double cost;
};

// Launch order of work units: each XCD (blocks are dealt to the 8 XCDs
// round-robin) receives a contiguous range of units of equal total cost, for
// the L2 locality of the operator tables, in decreasing cost, so that the
// dispatcher runs longest-first.  Padding blocks get tile -1.
void order_units(const std::vector<Unit> &units, std::vector<int> &unit_tile, std::vector<int> &unit_mt) {
  double sum = 0;
  for (const Unit &u : units) sum += u.cost;
  std::vector<std::vector<Unit>> part(8);
  double run = 0;
  for (const Unit &u : units) {
    const int x = std::min(7, (int)(8.0 * run / std::max(sum, 1e-300)));
    part[x].push_back(u);
    run += u.cost;
  }
  size_t per = 0;
  for (auto &v : part) {
    std::stable_sort(v.begin(), v.end(), [](const Unit &a, const Unit &b) { return a.cost > b.cost; });
    per = std::max(per, v.size());
  }
  unit_tile.assign(8 * per, -1);
  unit_mt.assign(8 * per, 0);
  for (int x = 0; x < 8; ++x)
    for (size_t j = 0; j < part[x].size(); ++j) {
      unit_tile[8 * j + x] = part[x][j].tile;
      unit_mt[8 * j + x] = part[x][j].mt;
    }
}

// Work units of the FP64 leaf kernel: (tile, first row tile | row tiles per
// wave << 16).  A unit costs about its slot count times its rows; tiles far
// above the balanced share of one resident block are split by rows (one row
// tile per wave), so that no single tile sets the kernel's duration.
void leaf_units(const std::vector<int> &tile_ptr, int n, int blocks_per_cu, int n_cu, double heavy_factor,
                std::vector<int> &unit_tile, std::vector<int> &unit_mt) {
  const int P = n * n, MTR = std::max(1, 3 * P / 16);
  const int TPW = n == 4 ? 1 : (n == 8 ? 3 : 4), G = (MTR + 4 * TPW - 1) / (4 * TPW);
  const int ntiles = (int)tile_ptr.size() - 1;
  auto cost_of = [](int slots, int ni) { return slots * (ni + 0.35); };
  double total = 0;
  for (int tt = 0; tt < ntiles; ++tt) total += G * cost_of(tile_ptr[tt + 1] - tile_ptr[tt], TPW);
  const double share = total / std::max(1, blocks_per_cu * n_cu);
  std::vector<Unit> units;
  for (int tt = 0; tt < ntiles; ++tt) {
    const int ns = tile_ptr[tt + 1] - tile_ptr[tt];
    if (ns == 0) continue;
    const bool heavy = TPW > 1 && cost_of(ns, TPW) > heavy_factor * share;
    for (int gg = 0; gg < G; ++gg) {
      if (!heavy) units.push_back({tt, gg * 4 * TPW | TPW << 16, cost_of(ns, TPW)});
      else
        for (int j = 0; j < TPW; ++j) units.push_back({tt, (gg * 4 * TPW + 4 * j) | 1 << 16, cost_of(ns, 1)});
    }
  }
  order_units(units, unit_tile, unit_mt);
}
}  // namespace
}  // namespace bx

// Work units of the leaf kernels from the tree's tilings and tuning
// parameters, uploaded (replacing earlier ones).
static int upload_units(bx_ctx *ctx, bx_tree *t, hipStream_t s) {
  std::vector<int> unit_tile, unit_mt, nunit_tile, nunit_mt;
  leaf_units(t->h_tile_ptr, ctx->n, 2, ctx->n_cu, t->tune_heavy, unit_tile, unit_mt);
  if (t->split) {   // int8 kernel: every tile (it writes V and G), 12 row tiles per block
    const int MTR = 3 * ctx->n * ctx->n / 16, ntiles = (int)t->h_tile_nsl.size();
    const std::vector<int> &tp = t->h_tile_ptr, &np = t->h_nslot_ptr, &nsl = t->h_tile_nsl;
    // a unit's cost: its int8 slice pairs and its FP64 slots (weighted by a
    // tuned number of pairs); tiles far above the balanced share of one
    // resident block are split into thirds by rows (one row tile per wave)
    auto cost_of = [&](int tt) {
      const int sv = std::max(3, nsl[tt] & 255), sd = std::max(3, nsl[tt] >> 8);
      const double pairs = (sv * (sv + 1) / 2.0 + 2.0 * sd * (sd + 1) / 2.0) / 3.0;
      return 1.0 + (np[tt + 1] - np[tt]) * pairs + t->tune_f64_weight * (tp[tt + 1] - tp[tt]);
    };
    double total = 0;
    for (int tt = 0; tt < ntiles; ++tt) total += cost_of(tt) * (MTR / 12);
    const double share = total / std::max(1, ctx->n_cu);
    std::vector<Unit> nu;
    for (int tt = 0; tt < ntiles; ++tt) {
      const double c = cost_of(tt);
      const bool heavy = c > t->tune_heavy * share;
      for (int mt0 = 0; mt0 < MTR; mt0 += 12) {
        if (!heavy) nu.push_back({tt, mt0 | 3 << 16, c});
        else
          for (int j = 0; j < 3; ++j) nu.push_back({tt, (mt0 + 4 * j) | 1 << 16, c / 3 + 0.5});
      }
    }
    order_units(nu, nunit_tile, nunit_mt);
    // the int8 kernel maps block b to unit 8 (b / 16) + b % 8 of a list padded to whole rows of 8
    if (nunit_tile.size() % 8 != 0) return fail(BX_E_ARG, "upload_units: unit list not padded to 8");
  }
  // upload the new lists first; the old ones stay in use until all copies succeeded
  std::vector<void *> bufs;
  const int *ut = nullptr, *um = nullptr, *nt = nullptr, *nm = nullptr;
  int rc;
  if ((rc = upload(bufs, unit_tile, &ut, s)) || (rc = upload(bufs, unit_mt, &um, s)) ||
      (rc = upload(bufs, nunit_tile, &nt, s)) || (rc = upload(bufs, nunit_mt, &nm, s))) {
    (void)hipStreamSynchronize(s);
    for (void *p : bufs) (void)hipFree(p);
    return rc;
  }
  // the host vectors die here: the copies must have completed
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    for (void *p : bufs) (void)hipFree(p);
    return hip_fail(e, "upload_units");
  }
  for (void *p : t->unit_bufs) (void)hipFree(p);
  t->unit_bufs.swap(bufs);
  DevTree &g = t->dg;
  g.unit_tile = ut;
  g.unit_mt = um;
  g.nunit_tile = nt;
  g.nunit_mt = nm;
  g.n_units = (int)unit_tile.size();
  g.n_nunits = (int)nunit_tile.size();
  g.m2l_blocks = t->tune_m2l_blocks;
  return BX_OK;
}

int bx_tree_upload(bx_ctx *ctx, const bx_tree_desc *trees, int n_trees, bx_tree **out, bx_stream_t stream) {
  if (!ctx || !trees || !out) return fail(BX_E_ARG, "bx_tree_upload: NULL argument");
  *out = nullptr;
  if (n_trees < 1) return fail(BX_E_ARG, "bx_tree_upload: n_trees < 1");
  auto t0 = std::chrono::steady_clock::now();
  bx_tree *t = new (std::nothrow) bx_tree;
  if (!t) return fail(BX_E_OOM, "bx_tree_upload");
  t->ctx = ctx;
  t->n_trees = n_trees;
  std::string err;
  int rc = BX_OK;
  if (n_trees == 1) {
    rc = build_tree(t->H, trees[0], err);
    t->box_tree.assign(t->H.n_boxes, 0);
  } else {   // a forest: each tree validated and listed on its own, then merged
    std::vector<HostTree> parts(n_trees);
    for (int k = 0; k < n_trees && !rc; ++k) {
      rc = build_tree(parts[k], trees[k], err);
      if (rc) err = "tree " + std::to_string(k) + ": " + err;
    }
    if (!rc) rc = merge_forest(parts, t->H, t->box_tree, err);
  }
  if (rc) {
    delete t;
    return fail(rc, "bx_tree_upload: " + err);
  }
  HostTree &H = t->H;
  hipStream_t s = (hipStream_t)stream;
  DevTree &g = t->dg;
  g.n_leaves = H.n_leaves; g.n_boxes = H.n_boxes; g.n_levels = H.n_levels; g.width = H.width;
  g.cx = H.cx; g.cy = H.cy;
  g.n_roots = H.n_levels > 0 ? H.level_start[1] : 0;
  std::vector<int> leaf_level(H.n_leaves);
  for (int i = 0; i < H.n_leaves; ++i) leaf_level[i] = H.lvl[H.box_of_leaf[i]];
  std::vector<int> up, us, uc, vp, vs, vc, wp, ws, wc, xp, xs, xc;
  csr(H.n_leaves, H.u_t, H.u_s, H.u_c, up, us, uc);
  csr(H.n_boxes, H.v_t, H.v_s, H.v_c, vp, vs, vc);
  csr(H.n_leaves, H.w_t, H.w_s, H.w_c, wp, ws, wc);
  csr(H.n_boxes, H.x_t, H.x_s, H.x_c, xp, xs, xc);
  // fused leaf GEMM tiles: leaves sorted by their set of near and W
  // configurations, TL per tile; each tile's slots are the union of its
  // leaves' configurations plus one L2T slot.
  const int TL = 64;
  const LeafFragLayout FL = leaf_frag_layout(ctx->n, ctx->p);
  std::vector<uint64_t> sig(H.n_leaves, 0);
  for (int i = 0; i < H.n_leaves; ++i) {
    for (int e = up[i]; e < up[i + 1]; ++e) sig[i] |= 1ull << uc[e];
    for (int e = wp[i]; e < wp[i + 1]; ++e) sig[i] |= 1ull << (NCFG_U + wc[e]);
  }
  std::vector<int> order(H.n_leaves);
  for (int i = 0; i < H.n_leaves; ++i) order[i] = i;
  // split contexts: tiles hold one level (the slice count depends on it)
  const bool split = (ctx->flags & BX_SPLIT_INT8) != 0;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (split && leaf_level[a] != leaf_level[b]) return leaf_level[a] > leaf_level[b];
    return sig[a] < sig[b];
  });
  std::vector<int> tile_first;   // tile -> index in order of its first leaf
  for (int i = 0; i < H.n_leaves;) {
    tile_first.push_back(i);
    int j = i + 1;
    while (j < H.n_leaves && j - i < TL && (!split || leaf_level[order[j]] == leaf_level[order[i]])) ++j;
    i = j;
  }
  int ntiles = (int)tile_first.size();
  tile_first.push_back(H.n_leaves);
  std::vector<int> tile_nsl(ntiles, 0), nslot_ptr(ntiles + 1, 0), nslot_cfg, nslot_src;
  int split_sf = 1;
  std::vector<int> tile_tgt((size_t)ntiles * TL, -1), tile_ptr(ntiles + 1, 0), slot_aoff, slot_type, slot_src,
      slot_op;
  for (int tt = 0; tt < ntiles; ++tt) {
    uint64_t uni = 0;
    for (int k = 0; k < TL && tile_first[tt] + k < tile_first[tt + 1]; ++k) {
      int leaf = order[tile_first[tt] + k];
      tile_tgt[(size_t)tt * TL + k] = leaf;
      uni |= sig[leaf];
    }
    bool near_i8 = false;
    if (split) {   // slices of the V rows (low byte) and of the gradient rows (next byte)
      const int lv = leaf_level[order[tile_first[tt]]];
      const int sv = split_slices(ctx->split, lv, ctx->split_tol, false),
                sd = split_slices(ctx->split, lv, ctx->split_tol, true);
      near_i8 = sv > 0 && sd > 0;   // otherwise more slices than the int8 kernel keeps: FP64
      tile_nsl[tt] = near_i8 ? sv | sd << 8 : 0;
      if (near_i8) split_sf = std::max(split_sf, std::max(3, std::max(sv, sd)));   // the kernel uses at least 3
    }
    for (int c = 0; c < NCFG_U; ++c) {
      if (!(uni >> c & 1)) continue;
      if (near_i8) {
        nslot_cfg.push_back(c);
      } else {
        slot_aoff.push_back((int)(FL.near0 + c * FL.near_step));
        slot_type.push_back(0);
        slot_op.push_back(c);
      }
      std::vector<int> &dst = near_i8 ? nslot_src : slot_src;
      for (int k = 0; k < TL; ++k) {
        int leaf = tile_tgt[(size_t)tt * TL + k], src = -1;
        if (leaf >= 0)
          for (int e = up[leaf]; e < up[leaf + 1]; ++e)
            if (uc[e] == c) src = us[e];
        dst.push_back(src);
      }
    }
    nslot_ptr[tt + 1] = (int)nslot_cfg.size();
    slot_aoff.push_back((int)FL.l2t);
    slot_type.push_back(1);
    slot_op.push_back(NCFG_U);
    for (int k = 0; k < TL; ++k) {
      int leaf = tile_tgt[(size_t)tt * TL + k];
      slot_src.push_back(leaf >= 0 ? H.box_of_leaf[leaf] : -1);
    }
    for (int c = 0; c < NCFG_W; ++c) {
      if (!(uni >> (NCFG_U + c) & 1)) continue;
      slot_aoff.push_back((int)(FL.w0 + c * FL.w_step));
      slot_type.push_back(2);
      slot_op.push_back(NCFG_U + 1 + c);
      for (int k = 0; k < TL; ++k) {
        int leaf = tile_tgt[(size_t)tt * TL + k], src = -1;
        if (leaf >= 0)
          for (int e = wp[leaf]; e < wp[leaf + 1]; ++e)
            if (wc[e] == c) src = ws[e];
        slot_src.push_back(src);
      }
    }
    tile_ptr[tt + 1] = (int)slot_type.size();
  }
  g.n_tiles = ntiles;
  t->h_tile_ptr = tile_ptr;
  t->h_nslot_ptr = nslot_ptr;
  t->h_tile_nsl = tile_nsl;
  t->split = split;
  t->tune_heavy = (ctx->flags & BX_SPLIT_INT8) ? 1.5 : 1.0;   // the measured best of each leaf kernel
  g.split_sf = split_sf;
  t->split_sf = split_sf;
  // X-list tiles: target boxes with X entries, sorted by configuration set
  std::vector<int> xb;
  std::vector<uint32_t> xsig(H.n_boxes, 0);
  for (int b = 0; b < H.n_boxes; ++b)
    if (xp[b + 1] > xp[b]) {
      xb.push_back(b);
      for (int e = xp[b]; e < xp[b + 1]; ++e) xsig[b] |= 1u << xc[e];
    }
  std::stable_sort(xb.begin(), xb.end(), [&](int a, int b) { return xsig[a] < xsig[b]; });
  const int nxt = ((int)xb.size() + 15) / 16;
  std::vector<int> xtile_box((size_t)nxt * 16, -1), xtile_ptr(nxt + 1, 0), xslot_cfg, xslot_src;
  for (int tt = 0; tt < nxt; ++tt) {
    uint32_t uni = 0;
    for (int k = 0; k < 16 && tt * 16 + k < (int)xb.size(); ++k) {
      xtile_box[(size_t)tt * 16 + k] = xb[tt * 16 + k];
      uni |= xsig[xb[tt * 16 + k]];
    }
    for (int c = 0; c < NCFG_X; ++c) {
      if (!(uni >> c & 1)) continue;
      xslot_cfg.push_back(c);
      for (int k = 0; k < 16; ++k) {
        int b = xtile_box[(size_t)tt * 16 + k], src = -1;
        if (b >= 0)
          for (int e = xp[b]; e < xp[b + 1]; ++e)
            if (xc[e] == c) src = xs[e];
        xslot_src.push_back(src);
      }
    }
    xtile_ptr[tt + 1] = (int)xslot_cfg.size();
  }
  g.n_xtiles = nxt;
  // M2L by sibling groups: for every internal box P, the 6 x 6 grid of boxes
  // one level below P's 3 x 3 neighbourhood (children of P's colleagues), from
  // which the V lists of P's four children are drawn; each V entry records the
  // grid slot of its source.
  std::vector<int> m2l_par, m2l_grid, v_slot(vs.size(), -1), m2l_ent, m2l_info;
  {
    std::vector<std::unordered_map<uint64_t, int>> at_tree(t->n_trees);   // per tree: key -> box
    for (int b = 0; b < H.n_boxes; ++b) at_tree[t->box_tree[b]][box_key(H.lvl[b], H.bx[b], H.by[b])] = b;
    for (int P = 0; P < H.n_boxes; ++P) {
      if (H.child0[P] < 0) continue;
      const int l = H.lvl[P];
      m2l_par.push_back(P);
      const std::unordered_map<uint64_t, int> &at = at_tree[t->box_tree[P]];
      for (int i = 0; i < 36; ++i) m2l_grid.push_back(-1);
      int *grid = &m2l_grid[m2l_grid.size() - 36];
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t qx = (int64_t)H.bx[P] + dx, qy = (int64_t)H.by[P] + dy;
          if (qx < 0 || qy < 0 || qx >= ((int64_t)1 << l) || qy >= ((int64_t)1 << l)) continue;
          auto it = at.find(box_key(l, qx, qy));
          if (it == at.end() || H.child0[it->second] < 0) continue;
          for (int q = 0; q < 4; ++q) grid[(2 * (dy + 1) + (q >> 1)) * 6 + 2 * (dx + 1) + (q & 1)] = H.child0[it->second] + q;
        }
      for (int q = 0; q < 4; ++q) {   // the V entries of each child: their slots in this grid
        const int tb = H.child0[P] + q;
        for (int e = vp[tb]; e < vp[tb + 1]; ++e) {
          const int src = vs[e], gx = H.bx[src] - (2 * H.bx[P] - 2), gy = H.by[src] - (2 * H.by[P] - 2);
          if (gx < 0 || gx >= 6 || gy < 0 || gy >= 6 || grid[gy * 6 + gx] != src) {
            bx_tree_destroy(t);
            return fail(BX_E_INVALID_TREE, "bx_tree_upload: V-list source outside its parent's grid");
          }
          v_slot[e] = gy * 6 + gx;
        }
        // packed entries of this child: slot | offset class << 8, padded with -1
        if (vp[tb + 1] - vp[tb] > M2L_VMAX) {
          bx_tree_destroy(t);
          return fail(BX_E_INVALID_TREE, "bx_tree_upload: V list longer than 32");
        }
        for (int j = 0; j < M2L_VMAX; ++j) {
          const int e = vp[tb] + j;
          m2l_ent.push_back(e < vp[tb + 1] ? v_slot[e] | vc[e] << 8 : -1);
        }
      }
      m2l_info.push_back(H.child0[P]);
      m2l_info.push_back(l + 1);
    }
    g.n_m2l_par = (int)m2l_par.size();
  }
  // internal boxes of each level (the M2M targets and the L2L sources)
  t->int_start.assign(H.n_levels + 1, 0);
  std::vector<int> ib;
  for (int l = 0; l < H.n_levels; ++l) {
    t->int_start[l] = (int)ib.size();
    for (int b = H.level_start[l]; b < H.level_start[l + 1]; ++b)
      if (H.leaf_of_box[b] < 0) ib.push_back(b);
  }
  t->int_start[H.n_levels] = (int)ib.size();
  // per level: the first child of the level's internal boxes when the children
  // are contiguous in list order (4 per box, level-major Morton order), else -1
  t->int_child_base.assign(H.n_levels, -1);
  for (int l = 0; l + 1 < H.n_levels; ++l) {
    const int base = H.level_start[l + 1];
    bool contiguous = true;
    for (int i = t->int_start[l]; i < t->int_start[l + 1] && contiguous; ++i)
      contiguous = H.child0[ib[i]] == base + 4 * (i - t->int_start[l]);
    t->int_child_base[l] = contiguous ? base : -1;
  }
  t->n_slots = (int64_t)slot_type.size();
  if (ctx->flags & BX_HOST_ONLY) {
    t->upload_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = t;
    return BX_OK;
  }
  if ((rc = upload(t->dev, H.lvl, &g.lvl, s)) || (rc = upload(t->dev, H.child0, &g.child0, s)) ||
      (rc = upload(t->dev, H.parent, &g.parent, s)) || (rc = upload(t->dev, H.leaf_of_box, &g.leaf_of_box, s)) ||
      (rc = upload(t->dev, H.box_of_leaf, &g.box_of_leaf, s)) || (rc = upload(t->dev, leaf_level, &g.leaf_level, s)) ||
      (rc = upload(t->dev, up, &g.u_ptr, s)) || (rc = upload(t->dev, us, &g.u_src, s)) ||
      (rc = upload(t->dev, uc, &g.u_cfg, s)) || (rc = upload(t->dev, vp, &g.v_ptr, s)) ||
      (rc = upload(t->dev, vs, &g.v_src, s)) || (rc = upload(t->dev, vc, &g.v_cfg, s)) ||
      (rc = upload(t->dev, wp, &g.w_ptr, s)) || (rc = upload(t->dev, ws, &g.w_src, s)) ||
      (rc = upload(t->dev, wc, &g.w_cfg, s)) || (rc = upload(t->dev, xp, &g.x_ptr, s)) ||
      (rc = upload(t->dev, xs, &g.x_src, s)) || (rc = upload(t->dev, xc, &g.x_cfg, s)) ||
      (rc = upload(t->dev, xtile_box, &g.xtile_box, s)) || (rc = upload(t->dev, xtile_ptr, &g.xtile_ptr, s)) ||
      (rc = upload(t->dev, xslot_cfg, &g.xslot_cfg, s)) || (rc = upload(t->dev, xslot_src, &g.xslot_src, s)) ||
      (rc = upload(t->dev, ib, &t->int_boxes, s)) || (rc = upload(t->dev, m2l_par, &g.m2l_par, s)) ||
      (rc = upload(t->dev, m2l_grid, &g.m2l_grid, s)) || (rc = upload(t->dev, v_slot, &g.v_slot, s)) ||
      (rc = upload(t->dev, m2l_ent, &g.m2l_ent, s)) || (rc = upload(t->dev, m2l_info, &g.m2l_info, s)) ||
      (rc = upload(t->dev, tile_tgt, &g.tile_tgt, s)) || (rc = upload(t->dev, tile_ptr, &g.tile_ptr, s)) ||
      (rc = upload(t->dev, slot_aoff, &g.slot_aoff, s)) || (rc = upload(t->dev, slot_type, &g.slot_type, s)) ||
      (rc = upload(t->dev, slot_op, &g.slot_op, s)) || (rc = upload(t->dev, tile_nsl, &g.tile_nsl, s)) ||
      (rc = upload(t->dev, slot_src, &g.slot_src, s)) || (rc = upload_units(ctx, t, s)) ||
      (split && ((rc = upload(t->dev, nslot_ptr, &g.nslot_ptr, s)) || (rc = upload(t->dev, nslot_cfg, &g.nslot_cfg, s)) ||
                 (rc = upload(t->dev, nslot_src, &g.nslot_src, s))))) {
    bx_tree_destroy(t);
    return rc;
  }
  // host vectors die at return: the copies must have completed
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    bx_tree_destroy(t);
    return hip_fail(e, "bx_tree_upload");
  }
  t->upload_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = t;
  return BX_OK;
}

static void drop_graphs(bx_tree *t) {
  for (GraphEntry &e : t->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    e = GraphEntry();
  }
}

static void free_split_buffers(bx_tree *t) {
  if (t->fscale) (void)hipFree(t->fscale);
  if (t->fpart) (void)hipFree(t->fpart);
  if (t->lmass) (void)hipFree(t->lmass);
  if (t->fsl) (void)hipFree(t->fsl);
  t->fscale = t->fpart = t->lmass = nullptr;
  t->fsl = nullptr;
}

static int ensure_expansions(bx_tree *t, int nrhs) {
  if (t->exp_rhs >= nrhs) return BX_OK;
  drop_graphs(t);
  if (t->M) (void)hipFree(t->M);
  if (t->L) (void)hipFree(t->L);
  t->M = t->L = nullptr;
  t->exp_rhs = 0;
  size_t bytes = (size_t)nrhs * t->H.n_boxes * t->ctx->T.KP * 2 * sizeof(double);
  free_split_buffers(t);
  hipError_t e = hipMalloc((void **)&t->M, bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&t->L, bytes);
  if (e == hipSuccess && (t->ctx->flags & BX_SPLIT_INT8)) {
    const size_t NL = t->H.n_leaves, P = t->ctx->T.P;
    e = hipMalloc((void **)&t->fscale, (size_t)nrhs * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&t->fpart, (size_t)nrhs * 512 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&t->lmass, (size_t)nrhs * NL * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&t->fsl, (size_t)nrhs * t->split_sf * NL * P);
  }
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(BX_E_OOM, "expansion buffers") : hip_fail(e, "hipMalloc");
  t->exp_rhs = nrhs;
  return BX_OK;
}

// Enqueue one evaluation on stream s (phases in order; per-phase events when profiling).
static int enqueue_eval(bx_ctx *ctx, bx_tree *t, const double *f, int nrhs, double *V, double *G, hipStream_t s) {
  const DevTables &d = ctx->dt;
  const DevTree &g = t->dg;
  const HostTree &H = t->H;
  int rc = BX_OK;
  hipEvent_t e0 = nullptr;
  auto mark = [&](int phase, bool start) -> int {
    if (!ctx->profiling) return BX_OK;
    hipEvent_t ev;
    hipError_t he = hipEventCreate(&ev);
    if (he == hipSuccess) he = hipEventRecord(ev, s);
    if (he != hipSuccess) return hip_fail(he, "profiling event");
    if (start) {
      e0 = ev;
    } else {
      ctx->ev.push_back(e0);
      ctx->ev.push_back(ev);
      ctx->ev_phase.push_back(phase);
    }
    return BX_OK;
  };
  if ((rc = mark(BX_PH_P2M, true))) return rc;
  launch_p2m(d, g, f, nrhs, t->M, s);
  if ((rc = mark(BX_PH_P2M, false)) || (rc = mark(BX_PH_M2M, true))) return rc;
  // levels whose internal boxes are few run two to a launch (latency-bound otherwise)
  auto n_int = [&](int l) { return t->int_start[l + 1] - t->int_start[l]; };
  for (int l = H.n_levels - 2; l >= 0;) {
    if (l >= 1 && n_int(l) <= t->tune_fuse) {
      launch_m2m2(d, g, t->int_boxes + t->int_start[l - 1], n_int(l - 1), nrhs, t->M, s);
      l -= 2;
    } else {
      launch_m2m(d, g, t->int_boxes + t->int_start[l], n_int(l), t->int_child_base[l], nrhs, t->M, s);
      l -= 1;
    }
  }
  if ((rc = mark(BX_PH_M2M, false)) || (rc = mark(BX_PH_M2L, true))) return rc;
  launch_m2l(d, g, nrhs, t->M, t->L, s);
  if ((rc = mark(BX_PH_M2L, false)) || (rc = mark(BX_PH_P2L, true))) return rc;
  launch_p2l(d, g, f, nrhs, t->L, s);
  if ((rc = mark(BX_PH_P2L, false)) || (rc = mark(BX_PH_L2L, true))) return rc;
  for (int l = 0; l + 1 < H.n_levels;) {
    if (l + 2 < H.n_levels && n_int(l + 1) <= t->tune_fuse) {
      launch_l2l2(d, g, t->int_boxes + t->int_start[l], n_int(l), nrhs, t->L, s);
      l += 2;
    } else {
      launch_l2l(d, g, t->int_boxes + t->int_start[l], n_int(l), nrhs, t->L, s);
      l += 1;
    }
  }
  if ((rc = mark(BX_PH_L2L, false)) || (rc = mark(BX_PH_LEAF, true))) return rc;
  if (ctx->flags & BX_SPLIT_INT8) {
    launch_split_prep(d, g, f, nrhs, t->fpart, t->fscale, t->fsl, t->lmass, s);
    launch_leaf_split(d, g, t->fsl, t->lmass, t->fscale, f, nrhs, t->M, t->L, V, G, s);
  } else {
    launch_leaf(d, g, f, nrhs, t->M, t->L, V, G, false, s);
  }
  if ((rc = mark(BX_PH_LEAF, false))) return rc;
  if (ctx->profiling) ctx->ev_evals++;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BX_OK;
}

static int eval_impl(bx_ctx *ctx, const bx_tree *tree_c, const double *f, int nrhs, double *V, double *G,
                     bx_stream_t stream) {
  if (!ctx || !tree_c || !f || nrhs <= 0) return fail(BX_E_ARG, "volume eval: NULL argument or n_rhs <= 0");
  if (!ctx->ready) return fail(BX_E_NO_TABLES, "volume eval: bx_build_tables has not been called");
  if (ctx->flags & BX_HOST_ONLY) return fail(BX_E_UNSUPPORTED, "volume eval: host-only context");
  bx_tree *t = const_cast<bx_tree *>(tree_c);
  if (t->ctx != ctx) return fail(BX_E_ARG, "volume eval: tree belongs to another context");
  if (((uintptr_t)f | (uintptr_t)V | (uintptr_t)G) & 7) return fail(BX_E_ARG, "volume eval: misaligned pointer");
  int rc = ensure_expansions(t, nrhs);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->profiling) return enqueue_eval(ctx, t, f, nrhs, V, G, s);
  // replay a captured graph of the whole evaluation when the buffers match
  for (GraphEntry &e : t->graphs)
    if (e.exec && e.f == f && e.V == V && e.G == G && e.nrhs == nrhs) {
      hipError_t he = hipGraphLaunch(e.exec, s);
      return he == hipSuccess ? BX_OK : hip_fail(he, "hipGraphLaunch");
    }
  if (!ctx->capture_stream) {
    hipError_t he = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_fail(he, "hipStreamCreateWithFlags");
  }
  hipStream_t cs = ctx->capture_stream;
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) return hip_fail(he, "hipStreamBeginCapture");
  rc = enqueue_eval(ctx, t, f, nrhs, V, G, cs);
  hipGraph_t graph = nullptr;
  he = hipStreamEndCapture(cs, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (he != hipSuccess) return hip_fail(he, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (he != hipSuccess) return hip_fail(he, "hipGraphInstantiate");
  GraphEntry &slot = t->graphs[t->graph_next];
  t->graph_next = (t->graph_next + 1) % 4;
  if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
  slot.f = f; slot.V = V; slot.G = G; slot.nrhs = nrhs; slot.exec = exec;
  he = hipGraphLaunch(exec, s);
  return he == hipSuccess ? BX_OK : hip_fail(he, "hipGraphLaunch");
}

int bx_volume_eval_grad(bx_ctx *ctx, const bx_tree *tree, const double *f_dev, int n_rhs, double *V_dev,
                        double *G_dev, bx_stream_t stream) {
  if (!V_dev || !G_dev) return fail(BX_E_ARG, "bx_volume_eval_grad: NULL output");
  return eval_impl(ctx, tree, f_dev, n_rhs, V_dev, G_dev, stream);
}

static int scratch_eval(bx_ctx *ctx, const bx_tree *tree, const double *f, int nrhs, double *V, double *G,
                        bool wantV, bx_stream_t stream) {
  if (!ctx || !tree) return fail(BX_E_ARG, "volume eval: NULL argument");
  size_t np = (size_t)nrhs * tree->H.n_leaves * ctx->T.P;
  double *tmp = nullptr;
  hipError_t e = hipMallocAsync((void **)&tmp, np * (wantV ? 2 : 1) * sizeof(double), (hipStream_t)stream);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(BX_E_OOM, "scratch output") : hip_fail(e, "hipMallocAsync");
  int rc = wantV ? eval_impl(ctx, tree, f, nrhs, V, tmp, stream) : eval_impl(ctx, tree, f, nrhs, tmp, G, stream);
  (void)hipFreeAsync(tmp, (hipStream_t)stream);
  return rc;
}

int bx_volume_eval(bx_ctx *ctx, const bx_tree *tree, const double *f_dev, int n_rhs, double *V_dev,
                   bx_stream_t stream) {
  if (!V_dev) return fail(BX_E_ARG, "bx_volume_eval: NULL output");
  return scratch_eval(ctx, tree, f_dev, n_rhs, V_dev, nullptr, true, stream);
}

int bx_volume_grad(bx_ctx *ctx, const bx_tree *tree, const double *f_dev, int n_rhs, double *G_dev,
                   bx_stream_t stream) {
  if (!G_dev) return fail(BX_E_ARG, "bx_volume_grad: NULL output");
  return scratch_eval(ctx, tree, f_dev, n_rhs, nullptr, G_dev, false, stream);
}

int bx_interpolate(const bx_ctx *ctx, const bx_tree *tree, const double *V, const double *G, int n_rhs,
                   const double *xy, int64_t n_targets, double *v_out, double *g_out, bx_stream_t stream) {
  if (!ctx || !tree || !xy || n_rhs <= 0 || n_targets < 0 || (!V && !G) || (V && !v_out) || (G && !g_out))
    return fail(BX_E_ARG, "bx_interpolate: NULL argument, n_rhs <= 0 or n_targets < 0");
  if (!ctx->ready) return fail(BX_E_NO_TABLES, "bx_interpolate: bx_build_tables has not been called");
  if (ctx->flags & BX_HOST_ONLY) return fail(BX_E_UNSUPPORTED, "bx_interpolate: host-only context");
  if (tree->ctx != ctx) return fail(BX_E_ARG, "bx_interpolate: tree belongs to another context");
  if (tree->n_trees != 1) return fail(BX_E_UNSUPPORTED, "bx_interpolate: one tree, not a forest");
  if (n_targets == 0) return BX_OK;
  launch_interpolate(ctx->dt, tree->dg, V, G, n_rhs, xy, (long long)n_targets, v_out, g_out, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BX_OK : hip_fail(e, "bx_interpolate");
}

int bx_tree_tuning(bx_ctx *ctx, bx_tree *tree, const double tune[4], bx_stream_t stream) {
  if (!ctx || !tree || !tune) return fail(BX_E_ARG, "bx_tree_tuning: NULL argument");
  if (tree->ctx != ctx) return fail(BX_E_ARG, "bx_tree_tuning: tree belongs to another context");
  if (tune[2] > 0 && (tune[2] != std::floor(tune[2]) || tune[2] > 65535))
    return fail(BX_E_ARG, "bx_tree_tuning: M2L blocks must be an integer in [1, 65535]");
  if (tune[3] != std::floor(tune[3]) || tune[3] < -1 || tune[3] > 1e9)
    return fail(BX_E_ARG, "bx_tree_tuning: the two-level threshold must be an integer >= -1");
  if (ctx->flags & BX_HOST_ONLY) return fail(BX_E_UNSUPPORTED, "bx_tree_tuning: host-only context");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);   // no evaluation may still read the old work lists
  if (e != hipSuccess) return hip_fail(e, "bx_tree_tuning");
  const double old_heavy = tree->tune_heavy, old_w = tree->tune_f64_weight;
  const int old_blocks = tree->tune_m2l_blocks, old_fuse = tree->tune_fuse;
  if (tune[0] > 0) tree->tune_heavy = tune[0];
  if (tune[1] > 0) tree->tune_f64_weight = tune[1];
  if (tune[2] > 0) tree->tune_m2l_blocks = (int)tune[2];
  if (tune[3] >= 0) tree->tune_fuse = (int)tune[3];   // -1 keeps it; 0 turns two-level launches off
  drop_graphs(tree);
  const int rc = upload_units(ctx, tree, s);
  if (rc) {                                            // the old work lists are still in place
    tree->tune_heavy = old_heavy;
    tree->tune_f64_weight = old_w;
    tree->tune_m2l_blocks = old_blocks;
    tree->tune_fuse = old_fuse;
  }
  return rc;
}

int bx_tree_tuning_get(const bx_tree *tree, double tune[4]) {
  if (!tree || !tune) return fail(BX_E_ARG, "bx_tree_tuning_get: NULL argument");
  tune[0] = tree->tune_heavy;
  tune[1] = tree->tune_f64_weight;
  tune[2] = tree->tune_m2l_blocks;
  tune[3] = tree->tune_fuse;
  return BX_OK;
}

int bx_autotune(bx_ctx *ctx, bx_tree *tree, const double *f, int nrhs, double *V, double *G, int reps,
                double best[5], bx_stream_t stream) {
  if (!ctx || !tree || !V || !G) return fail(BX_E_ARG, "bx_autotune: NULL argument");
  if (reps < 1) return fail(BX_E_ARG, "bx_autotune: reps < 1");
  if (ctx->profiling) return fail(BX_E_ARG, "bx_autotune: profiling is enabled");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t he = hipEventCreate(&ev[0]);
  if (he == hipSuccess) he = hipEventCreate(&ev[1]);
  if (he != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return hip_fail(he, "bx_autotune events");
  }
  // median of 3 batches of `reps` evaluations (after one untimed evaluation,
  // which also captures the graph), milliseconds per evaluation
  auto time_it = [&](double *ms) -> int {
    int rc = bx_volume_eval_grad(ctx, tree, f, nrhs, V, G, stream);
    if (rc) return rc;
    double t[3];
    for (int k = 0; k < 3; ++k) {
      hipError_t e = hipEventRecord(ev[0], s);
      for (int r = 0; r < reps && !rc && e == hipSuccess; ++r) rc = bx_volume_eval_grad(ctx, tree, f, nrhs, V, G, stream);
      if (rc) return rc;
      if (e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float x = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&x, ev[0], ev[1]);
      if (e != hipSuccess) return hip_fail(e, "bx_autotune timing");
      t[k] = x / reps;
    }
    std::sort(t, t + 3);
    *ms = t[1];
    return BX_OK;
  };
  double cur[4] = {tree->tune_heavy, tree->tune_f64_weight, (double)tree->tune_m2l_blocks, (double)tree->tune_fuse};
  const double start[4] = {cur[0], cur[1], cur[2], cur[3]};
  double best_ms = 0;
  int rc = bx_tree_tuning(ctx, tree, cur, stream);
  if (!rc) rc = time_it(&best_ms);
  static const double cand_m2l[] = {1024, 2048, 3072, 4096, 6144, 8192};
  static const double cand_heavy[] = {0.75, 1.0, 1.25, 1.5, 2.0, 1e30};
  static const double cand_w[] = {2, 4, 8, 16, 32, 64};
  static const double cand_fuse[] = {0, 512, 2048};
  struct Axis { int k; const double *v; int n; };
  const Axis axes[4] = {{2, cand_m2l, 6}, {0, cand_heavy, 6}, {1, cand_w, (ctx->flags & BX_SPLIT_INT8) ? 6 : 0},
                        {3, cand_fuse, 3}};
  for (const Axis &a : axes) {
    for (int i = 0; i < a.n && !rc; ++i) {
      if (a.v[i] == cur[a.k]) continue;
      double trial[4] = {cur[0], cur[1], cur[2], cur[3]}, ms = 0;
      trial[a.k] = a.v[i];
      if ((rc = bx_tree_tuning(ctx, tree, trial, stream)) || (rc = time_it(&ms))) break;
      if (ms < best_ms) {
        best_ms = ms;
        cur[a.k] = a.v[i];
      }
    }
  }
  // leave the best setting in place, with its result in V and G (on failure,
  // the setting the tuner started from)
  if (rc) {
    (void)bx_tree_tuning(ctx, tree, start, stream);
  }
  if (!rc) rc = bx_tree_tuning(ctx, tree, cur, stream);
  if (!rc) rc = bx_volume_eval_grad(ctx, tree, f, nrhs, V, G, stream);
  if (!rc) {
    he = hipStreamSynchronize(s);
    if (he != hipSuccess) rc = hip_fail(he, "bx_autotune");
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (!rc && best) {
    best[0] = cur[0];
    best[1] = cur[1];
    best[2] = cur[2];
    best[3] = cur[3];
    best[4] = best_ms;
  }
  return rc;
}

int bx_expansion_read(const bx_ctx *ctx, const bx_tree *tree, int which, int64_t box, int rhs, double *out,
                      bx_stream_t stream) {
  if (!ctx || !tree || !out || (which != 0 && which != 1) || box < 0 || box >= tree->H.n_boxes || rhs < 0)
    return fail(BX_E_ARG, "bx_expansion_read: bad argument");
  if (tree->ctx != ctx) return fail(BX_E_ARG, "bx_expansion_read: tree belongs to another context");
  if (!tree->M || rhs >= tree->exp_rhs) return fail(BX_E_UNSUPPORTED, "bx_expansion_read: no evaluation with this rhs");
  const int KP = ctx->T.KP, nt = ctx->p + 1;
  std::vector<double> v((size_t)2 * KP);
  const double *src = (which == 0 ? tree->M : tree->L) + ((size_t)rhs * tree->H.n_boxes + box) * KP * 2;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(v.data(), src, v.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "bx_expansion_read");
  // stored: multipole a_k / h^k, local b_l h^l (h = the box width)
  const double h = tree->H.width * std::ldexp(1.0, -tree->H.lvl[box]);
  double sc = 1.0;
  for (int k = 0; k < nt; ++k) {
    out[2 * k] = v[2 * k] * sc;
    out[2 * k + 1] = v[2 * k + 1] * sc;
    sc = which == 0 ? sc * h : sc / h;
  }
  return BX_OK;
}

int bx_split_tolerance(bx_ctx *ctx, double tol) {
  if (!ctx || !(tol > 0.0) || tol >= 1.0) return fail(BX_E_ARG, "bx_split_tolerance: need 0 < tol < 1");
  ctx->split_tol = tol;
  return BX_OK;
}

int bx_profile(bx_ctx *ctx, int enable) {
  if (!ctx) return fail(BX_E_ARG, "bx_profile: ctx is NULL");
  ctx->profiling = enable != 0;
  return BX_OK;
}

int bx_profile_read(bx_ctx *ctx, double *ms, int *n_evals) {
  if (!ctx || !ms || !n_evals) return fail(BX_E_ARG, "bx_profile_read: NULL argument");
  int rc = BX_OK;
  for (size_t i = 0; i < ctx->ev_phase.size(); ++i) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(ctx->ev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ctx->ev[2 * i], ctx->ev[2 * i + 1]);
    if (e != hipSuccess && rc == BX_OK) rc = hip_fail(e, "bx_profile_read");
    ms[ctx->ev_phase[i]] += t;
  }
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  *n_evals = ctx->ev_evals;
  ctx->ev.clear();
  ctx->ev_phase.clear();
  ctx->ev_evals = 0;
  return rc;
}

// Algorithmic flops and bytes of one phase for one right-hand side.
static void phase_cost(const bx_ctx *ctx, const HostTree &H, int ph, double *flops, double *bytes) {
  const double P = ctx->n * ctx->n, nt = ctx->p + 1, NL = H.n_leaves, NB = H.n_boxes, C = 16.0 * nt;
  double nint = 0;
  for (int b = 0; b < H.n_boxes; ++b) nint += H.leaf_of_box[b] < 0;
  double U = (double)H.u_t.size(), Vp = (double)H.v_t.size(), W = (double)H.w_t.size(),
         X = (double)H.x_t.size();
  *flops = *bytes = 0;
  switch (ph) {
    case BX_PH_P2M: *flops = 2.0 * 2 * nt * P * NL; *bytes = NL * (8 * P + C); break;
    case BX_PH_M2M: *flops = 8.0 * nt * (nt + 1) / 2 * 4 * nint; *bytes = (4 * nint + nint) * C; break;
    case BX_PH_M2L: *flops = Vp * (4.0 * nt * nt + 12.0 * nt); *bytes = NB * C + NB * C; break;
    case BX_PH_P2L: *flops = X * 2.0 * 2 * nt * P; *bytes = X * 8 * P + 2 * NB * C; break;
    case BX_PH_L2L: *flops = 8.0 * nt * (nt + 1) / 2 * (NB - 1); *bytes = (NB - 1) * 2 * C; break;
    case BX_PH_LEAF:   // near tables (with the mass row) + L2T + W, fused
      *flops = U * 2.0 * (3 * P + 1) * P + 2.0 * 3 * P * 2 * nt * NL + 2.0 * (3 * P + 1) * 2 * nt * W;
      *bytes = NL * 8 * P + NL * C + NL * 24 * P;
      break;
    default: break;
  }
}

int bx_query(const bx_ctx *ctx, const bx_tree *tree, int what, double *out) {
  if (!ctx || !out) return fail(BX_E_ARG, "bx_query: NULL argument");
  const Tables &T = ctx->T;
  const int P = ctx->n * ctx->n, nt = ctx->p + 1;
  switch (what) {
    case BX_Q_NODES: *out = ctx->n; return BX_OK;
    case BX_Q_ORDER: *out = ctx->p; return BX_OK;
    default: break;
  }
  if (!tree) return fail(BX_E_ARG, "bx_query: this quantity needs a tree");
  const HostTree &H = tree->H;
  (void)T;
  double nb_internal = 0;
  for (int b = 0; b < H.n_boxes; ++b) nb_internal += H.leaf_of_box[b] < 0;
  switch (what) {
    case BX_Q_N_LEAVES: *out = H.n_leaves; break;
    case BX_Q_N_BOXES: *out = H.n_boxes; break;
    case BX_Q_N_LEVELS: *out = H.n_levels; break;
    case BX_Q_NEAR_PAIRS: *out = (double)H.u_t.size(); break;
    case BX_Q_V_PAIRS: *out = (double)H.v_t.size(); break;
    case BX_Q_W_PAIRS: *out = (double)H.w_t.size(); break;
    case BX_Q_X_PAIRS: *out = (double)H.x_t.size(); break;
    case BX_Q_NEAR_FLOPS:   // 3P x P table product plus the P-term mass row, per U pair
      *out = (double)H.u_t.size() * 2.0 * (3.0 * P + 1.0) * P;
      break;
    case BX_Q_FAR_FLOPS: {
      double p2m = 2.0 * 2 * nt * P * H.n_leaves;              // real 2nt x P product
      double m2m = 8.0 * nt * (nt + 1) / 2 * 4 * nb_internal;   // 4 triangular complex products
      double l2l = 8.0 * nt * (nt + 1) / 2 * (H.n_boxes - 1);
      double m2l = (double)H.v_t.size() * (4.0 * nt * nt + 12.0 * nt);   // real core on complex data + scalings
      double x = (double)H.x_t.size() * 2.0 * 2 * nt * P;
      double w = (double)H.w_t.size() * 2.0 * 3 * P * 2 * nt;
      double l2t = 2.0 * 3 * P * 2 * nt * H.n_leaves;
      *out = p2m + m2m + l2l + m2l + x + w + l2t;
      break;
    }
    case BX_Q_NEAR_TILES: *out = tree->dg.n_tiles; break;
    case BX_Q_NEAR_SLOTS: *out = (double)tree->n_slots; break;
    case BX_Q_UPLOAD_MS: *out = tree->upload_ms; break;
    case BX_Q_SPLIT_PRODUCTS: {   // int8 slice products per near table entry, averaged over leaves
      if (!(ctx->flags & BX_SPLIT_INT8)) { *out = 0; break; }
      double num = 0, den = 0;
      for (int i = 0; i < H.n_leaves; ++i) {
        int sv = split_slices(ctx->split, H.lvl[H.box_of_leaf[i]], ctx->split_tol, false);
        int sd = split_slices(ctx->split, H.lvl[H.box_of_leaf[i]], ctx->split_tol, true);
        if (sv > 0 && sd > 0)   // V rows : gradient rows = 1 : 2; leaves left in FP64 count 0
          num += (sv * (sv + 1) / 2.0 + 2.0 * sd * (sd + 1) / 2.0) / 3.0;
        den += 1;
      }
      *out = den > 0 ? num / den : 0;
      break;
    }
    default: {
      double fl, by;
      if (what >= BX_Q_PHASE_FLOPS && what < BX_Q_PHASE_FLOPS + BX_N_PHASES) {
        phase_cost(ctx, H, what - BX_Q_PHASE_FLOPS, &fl, &by);
        *out = fl;
      } else if (what >= BX_Q_PHASE_BYTES && what < BX_Q_PHASE_BYTES + BX_N_PHASES) {
        phase_cost(ctx, H, what - BX_Q_PHASE_BYTES, &fl, &by);
        *out = by;
      } else {
        return fail(BX_E_ARG, "bx_query: unknown quantity");
      }
    }
  }
  return BX_OK;
}

int bx_table_copy(const bx_ctx *ctx, int which, double *out, int64_t cap, int64_t *count) {
  if (!ctx || !count) return fail(BX_E_ARG, "bx_table_copy: NULL argument");
  if (!ctx->ready) return fail(BX_E_NO_TABLES, "bx_table_copy: bx_build_tables has not been called");
  const Tables &T = ctx->T;
  const std::vector<double> *v[12] = {&T.near_, &T.p2m, &T.m2m, &T.l2l, &T.H, &T.pw_src,
                                      &T.pw_tgt, &T.logd, &T.l2t, &T.m2t, &T.p2l, &T.wq};
  if (which >= 12 && which <= 14) {   // split tables, as doubles
    if (!(ctx->flags & BX_SPLIT_INT8)) return fail(BX_E_ARG, "bx_table_copy: not a split context");
    const SplitTables &S = ctx->split;
    std::vector<double> tmp;
    if (which == 12) {   // slices [33][SMAX][3P][P] in natural order
      const int P = T.P, R = 3 * P, MTR = R / 16, NCH = P / 64;
      tmp.resize((size_t)NCFG_U * SPLIT_SMAX * R * P);
      for (int c = 0; c < NCFG_U; ++c)
        for (int a = 0; a < SPLIT_SMAX; ++a)
          for (int r = 0; r < R; ++r)
            for (int k = 0; k < P; ++k) {
              const int mt = r / 16, lane = r % 16 + 16 * (k % 64 / 16), ch = k / 64;
              tmp[(((size_t)c * SPLIT_SMAX + a) * R + r) * P + k] =
                  S.a[(((((size_t)c * SPLIT_SMAX + a) * MTR + mt) * NCH + ch) * 64 + lane) * 16 + k % 16];
            }
    } else if (which == 13) {
      tmp = S.row_scale;
    } else {
      tmp = S.err_v;
      tmp.insert(tmp.end(), S.err_d.begin(), S.err_d.end());
    }
    *count = (int64_t)tmp.size();
    if (out) std::memcpy(out, tmp.data(), (size_t)std::min<int64_t>(cap, *count) * sizeof(double));
    return BX_OK;
  }
  if (which < 0 || which >= 12) return fail(BX_E_ARG, "bx_table_copy: unknown table");
  *count = (int64_t)v[which]->size();
  if (out) std::memcpy(out, v[which]->data(), (size_t)std::min<int64_t>(cap, *count) * sizeof(double));
  return BX_OK;
}

int bx_tree_list(const bx_tree *tree, int kind, int64_t *out, int64_t cap, int64_t *count) {
  if (!tree || !count) return fail(BX_E_ARG, "bx_tree_list: NULL argument");
  const HostTree &H = tree->H;
  const std::vector<int> *T = nullptr, *S = nullptr, *C = nullptr;
  bool tbox = false, sbox = false;
  switch (kind) {
    case 0: T = &H.u_t; S = &H.u_s; C = &H.u_c; break;
    case 1: T = &H.v_t; S = &H.v_s; C = &H.v_c; tbox = sbox = true; break;
    case 2: T = &H.w_t; S = &H.w_s; C = &H.w_c; sbox = true; break;
    case 3: T = &H.x_t; S = &H.x_s; C = &H.x_c; tbox = true; break;
    default: return fail(BX_E_ARG, "bx_tree_list: unknown kind");
  }
  *count = (int64_t)T->size();
  if (!out) return BX_OK;
  auto key = [&](int b) { return (int64_t)box_key(H.lvl[b], H.bx[b], H.by[b]); };
  int64_t m = std::min<int64_t>(cap, *count);
  for (int64_t i = 0; i < m; ++i) {
    out[3 * i] = tbox ? key((*T)[i]) : (*T)[i];
    out[3 * i + 1] = sbox ? key((*S)[i]) : (*S)[i];
    out[3 * i + 2] = (*C)[i];
  }
  return BX_OK;
}

void bx_tree_destroy(bx_tree *tree) {
  if (!tree) return;
  drop_graphs(tree);
  for (void *p : tree->dev) (void)hipFree(p);
  if (tree->M) (void)hipFree(tree->M);
  if (tree->L) (void)hipFree(tree->L);
  free_split_buffers(tree);
  for (void *p : tree->unit_bufs) (void)hipFree(p);
  delete tree;
}

void bx_destroy(bx_ctx *ctx) {
  if (!ctx) return;
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  for (void *p : ctx->dev) (void)hipFree(p);
  delete ctx;
}

int bx_mlp_features(const double *samples_dev, const int8_t *level_dev, int64_t n_boxes, uint16_t *x_dev,
                    bx_stream_t stream) {
  if (n_boxes < 0 || (n_boxes > 0 && (!samples_dev || !level_dev || !x_dev)))
    return fail(BX_E_ARG, "bx_mlp_features: NULL pointer or n_boxes < 0");
  if (((uintptr_t)x_dev & 15) || ((uintptr_t)samples_dev & 7)) return fail(BX_E_ARG, "bx_mlp_features: misaligned");
  launch_mlp_features(samples_dev, level_dev, (long long)n_boxes, x_dev, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BX_OK : hip_fail(e, "bx_mlp_features");
}

int bx_mlp_set_params(bx_mlp *net, const float *params_host, bx_stream_t stream) {
  if (!net) return fail(BX_E_ARG, "bx_mlp_set_params: NULL network");
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)MLP_NPARAM * sizeof(float);
  hipError_t e = params_host ? hipMemcpyAsync(net->d.theta, params_host, bytes, hipMemcpyHostToDevice, s)
                             : hipMemsetAsync(net->d.theta, 0, bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(net->d.m, 0, bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(net->d.v, 0, bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(net->d.grad, 0, bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(net->d.loss, 0, sizeof(float), s);
  if (e == hipSuccess) {
    launch_mlp_refresh(net->d, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // params_host may die after the call
  if (e != hipSuccess) return hip_fail(e, "bx_mlp_set_params");
  net->step = 0;
  return BX_OK;
}

int bx_mlp_create(bx_mlp **out, const float *params_host, bx_stream_t stream) {
  if (!out) return fail(BX_E_ARG, "bx_mlp_create: NULL output");
  *out = nullptr;
  bx_mlp *net = new bx_mlp;
  const size_t nf = ((size_t)MLP_NPARAM + 63) / 64 * 64;            // floats per FP32 array, 256-byte multiple
  const size_t bytes = 4 * nf * sizeof(float) + 256 +                  // theta, grad, m, v; loss
                       (size_t)(MLP_HID * MLP_IN + 2 * MLP_HID * MLP_HID) * sizeof(uint16_t);
  hipError_t e = hipMalloc(&net->block, bytes);
  if (e != hipSuccess) {
    delete net;
    return e == hipErrorOutOfMemory ? fail(BX_E_OOM, "bx_mlp_create") : hip_fail(e, "bx_mlp_create");
  }
  float *f = (float *)net->block;
  net->d.theta = f;
  net->d.grad = f + nf;
  net->d.m = f + 2 * nf;
  net->d.v = f + 3 * nf;
  net->d.loss = f + 4 * nf;
  uint16_t *h = (uint16_t *)(f + 4 * nf + 64);
  net->d.w1b = h;
  net->d.w2b = h + MLP_HID * MLP_IN;
  net->d.w2tb = net->d.w2b + MLP_HID * MLP_HID;
  int rc = bx_mlp_set_params(net, params_host, stream);
  if (rc) {
    bx_mlp_destroy(net);
    return rc;
  }
  *out = net;
  return BX_OK;
}

int bx_mlp_forward(const bx_mlp *net, const uint16_t *x_dev, int64_t n, float *logit_dev, bx_stream_t stream) {
  if (!net || n < 0 || (n > 0 && (!x_dev || !logit_dev))) return fail(BX_E_ARG, "bx_mlp_forward: bad argument");
  if ((uintptr_t)x_dev & 15) return fail(BX_E_ARG, "bx_mlp_forward: x_dev must be 16-byte aligned");
  launch_mlp_forward(net->d, x_dev, (long long)n, logit_dev, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BX_OK : hip_fail(e, "bx_mlp_forward");
}

int bx_mlp_grad(bx_mlp *net, const uint16_t *x_dev, const float *y_dev, int64_t n, bx_stream_t stream) {
  if (!net || n < 0 || (n > 0 && (!x_dev || !y_dev))) return fail(BX_E_ARG, "bx_mlp_grad: bad argument");
  if ((uintptr_t)x_dev & 15) return fail(BX_E_ARG, "bx_mlp_grad: x_dev must be 16-byte aligned");
  launch_mlp_grad(net->d, x_dev, y_dev, (long long)n, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BX_OK : hip_fail(e, "bx_mlp_grad");
}

int bx_mlp_adam(bx_mlp *net, float lr, float beta1, float beta2, float eps, bx_stream_t stream) {
  if (!net || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(BX_E_ARG, "bx_mlp_adam: need lr >= 0, 0 <= betas < 1, eps > 0");
  const int t = net->step + 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, t)), c2 = 1.0 / (1.0 - std::pow((double)beta2, t));
  launch_mlp_adam(net->d, lr, beta1, beta2, eps, (float)c1, (float)c2, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "bx_mlp_adam");
  net->step = t;
  return BX_OK;
}

int bx_mlp_read(const bx_mlp *net, int which, float *out_host, int64_t cap, bx_stream_t stream) {
  if (!net || !out_host || which < 0 || which > 4) return fail(BX_E_ARG, "bx_mlp_read: bad argument");
  const float *src[5] = {net->d.theta, net->d.grad, net->d.m, net->d.v, net->d.loss};
  const int64_t count = which == 4 ? 1 : MLP_NPARAM;
  if (cap < count) return fail(BX_E_ARG, "bx_mlp_read: cap too small");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(out_host, src[which], count * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? BX_OK : hip_fail(e, "bx_mlp_read");
}

void bx_mlp_destroy(bx_mlp *net) {
  if (!net) return;
  if (net->block) (void)hipFree(net->block);
  delete net;
}

}  // extern "C"
