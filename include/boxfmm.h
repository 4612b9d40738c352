/*
 * boxfmm.h -- C ABI of the MI355X box-code volume potential library.
 *
 * The library evaluates, at every collocation node of a level-restricted
 * quadtree, the volume potential of the piecewise polynomial source and its
 * gradient (section 3, eq. volumeint3; gradient by the second volume
 * integral of section 3.2, eq. volumeint3x):
 *
 *     V(x) = int_Box G(x - y) f~(y) dy,   grad V(x) = int_Box grad_x G(x - y) f~(y) dy,
 *     G(r) = log|r| / (2 pi),
 *
 * where f~ is, on each leaf, the degree-(n-1) tensor polynomial through the
 * leaf's samples at first-kind Chebyshev nodes (section 3.1).  As in the box
 * code of section 3.1, far interactions go through multipole and local
 * expansions and near ones through precomputed tables for a unit box,
 * scaled per level (section 3.1, last paragraph).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: BX_OK (0) on success, a negative BX_E_* code otherwise.
 *   bx_last_error() gives a message for the calling thread's last failure.
 *   No C++ exception crosses this interface.
 * - Nodes: xi_j = -cos((2j+1) pi / 2n), j = 0..n-1, on [-1,1], scaled to
 *   each leaf.  A leaf's n*n samples are stored with the x index fastest.
 * - Device buffers (f, V, G) are owned by the caller, allocated on the
 *   context's device, contiguous, 8-byte aligned FP64.  The library reads f
 *   and writes V, G inside the call's stream order and keeps no reference
 *   after the call returns.
 * - Layouts: f[n_rhs][n_leaves][n][n], V[n_rhs][n_leaves][n][n],
 *   G[n_rhs][n_leaves][2][n][n] (component 0 = dV/dx1, 1 = dV/dx2).  Leaf
 *   order is the order of the tree descriptor.
 * - Calls that take a stream enqueue work on it and return without
 *   synchronising; the caller synchronises.  A NULL stream is the default
 *   stream.
 * - Objects: bx_ctx and bx_tree are opaque and owned by the library; free
 *   them with bx_destroy / bx_tree_destroy.  A tree may only be used with
 *   the context that created it.  Concurrent calls on one context from
 *   several threads are not supported.
 */
#ifndef BOXFMM_H
#define BOXFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bx_ctx bx_ctx;
typedef struct bx_tree bx_tree;
typedef void *bx_stream_t;   /* a hipStream_t */

enum {
  BX_OK = 0,
  BX_E_ARG = -1,            /* null or inconsistent argument */
  BX_E_NOT_BALANCED = -2,   /* adjacent leaves (corners included) differ by more than one level */
  BX_E_INVALID_TREE = -3,   /* leaves overlap, repeat, fall outside the root or leave holes */
  BX_E_UNSUPPORTED = -4,    /* node count or expansion order outside the supported set */
  BX_E_HIP = -5,            /* a HIP runtime call failed */
  BX_E_OOM = -6,            /* device or host allocation failed */
  BX_E_NO_TABLES = -7       /* evaluation before bx_build_tables */
};

/* Precision of the near-field table products. */
enum {
  BX_FP64 = 0,              /* FP64 MFMA throughout */
  BX_SPLIT_INT8 = 1,        /* near tables as exact int8 slice products with int32 accumulation,
                               recombined in FP64 (far field, log terms and sums stay FP64) */
  BX_HOST_ONLY = 0x100      /* or-ed in: no device is touched; tables and trees are built on the
                               host for inspection only and evaluation returns BX_E_UNSUPPORTED */
};

/*
 * Create a context on the current HIP device.
 *   n_nodes: collocation nodes per side, one of 4, 8, 16.
 *   p_exp:   expansion order p (coefficients 0..p), 8 <= p <= 47.
 *   flags:   BX_FP64 or BX_SPLIT_INT8, optionally or-ed with BX_HOST_ONLY.
 * Errors: BX_E_ARG (out NULL), BX_E_UNSUPPORTED, BX_E_HIP.
 */
int bx_create(bx_ctx **out, int n_nodes, int p_exp, uint32_t flags);

/*
 * Build the unit-box operators on the host in FP64 and upload them: the
 * near-field tables for the 33 neighbour configurations of a level-restricted
 * tree (section 3.1: a finite set of near interactions up to scale), for V and
 * both gradient components, and the expansion operators.  Blocks the calling
 * thread.  quad_tol <= 0 selects the default (1e-15).  cache_dir may be NULL;
 * if given, tables are read from / written to a file keyed by (n, p) there and
 * rebuilt when the file is missing or fails its checksum.
 * Errors: BX_E_ARG, BX_E_HIP, BX_E_OOM.
 */
int bx_build_tables(bx_ctx *ctx, double quad_tol, const char *cache_dir);

/* Host description of one tree: the root box and its leaves (copied by upload). */
typedef struct {
  double cx, cy, width;     /* root box centre and width */
  int32_t n_leaves;
  const int8_t *level;      /* [n_leaves], 0 = root, at most 29 */
  const int32_t *ix;        /* [n_leaves], 0 <= ix < 2^level, from the left edge */
  const int32_t *iy;        /* [n_leaves], 0 <= iy < 2^level, from the bottom edge */
} bx_tree_desc;

/*
 * Validate a leaf set (it must tile the root exactly and be level-restricted,
 * section 3.1), build the box hierarchy and the interaction lists on the host,
 * and upload them.  With n_trees > 1 the trees form a forest evaluated as one:
 * each tree is validated and listed on its own (no interaction crosses trees),
 * the leaves are numbered tree after tree in descriptor order (the layout of f,
 * V and G), every level-synchronous pass covers all trees at that level, and
 * one captured graph runs the whole forest.  The trees of a forest must share
 * the root width (centres may differ); bx_interpolate takes single trees only.
 * The stream orders the uploads.  Errors: BX_E_ARG, BX_E_INVALID_TREE (with the
 * tree's index in the message), BX_E_NOT_BALANCED, BX_E_UNSUPPORTED (widths
 * differ), BX_E_HIP, BX_E_OOM.
 */
int bx_tree_upload(bx_ctx *ctx, const bx_tree_desc *trees, int n_trees, bx_tree **out,
                   bx_stream_t stream);

/* V and grad V at every node of every leaf, for n_rhs right-hand sides. */
int bx_volume_eval_grad(bx_ctx *ctx, const bx_tree *tree, const double *f_dev, int n_rhs,
                        double *V_dev, double *G_dev, bx_stream_t stream);

/* V only (the gradient is still formed internally and discarded). */
int bx_volume_eval(bx_ctx *ctx, const bx_tree *tree, const double *f_dev, int n_rhs,
                   double *V_dev, bx_stream_t stream);

/* grad V only. */
int bx_volume_grad(bx_ctx *ctx, const bx_tree *tree, const double *f_dev, int n_rhs,
                   double *G_dev, bx_stream_t stream);

/* Quantities for reports, written to *out (host). */
enum {
  BX_Q_N_LEAVES = 0, BX_Q_N_BOXES = 1, BX_Q_N_LEVELS = 2, BX_Q_NODES = 3, BX_Q_ORDER = 4,
  BX_Q_NEAR_PAIRS = 5,       /* U-list (target, source) pairs */
  BX_Q_V_PAIRS = 6,          /* V-list pairs (M2L) */
  BX_Q_W_PAIRS = 7,          /* W-list pairs (multipole to targets) */
  BX_Q_X_PAIRS = 8,          /* X-list pairs (sources to local) */
  BX_Q_NEAR_FLOPS = 9,       /* algorithmic FP64 flops of the near-table products, one RHS */
  BX_Q_FAR_FLOPS = 10,       /* algorithmic flops of P2M, M2M, M2L, W, X, L2L, L2T, one RHS */
  BX_Q_NEAR_TILES = 11,      /* 16-target tiles of the near kernel */
  BX_Q_NEAR_SLOTS = 12,      /* (tile, configuration) slots of the near kernel */
  BX_Q_UPLOAD_MS = 13,       /* host time of the last bx_tree_upload, milliseconds */
  BX_Q_SPLIT_PRODUCTS = 14,  /* split contexts: mean int8 slice products per near table entry, over leaves */
  /* algorithmic FP64 flops of one evaluation phase, one RHS: add the phase index */
  BX_Q_PHASE_FLOPS = 20,
  /* algorithmic bytes of one evaluation phase (each operand read and each result
     written once from HBM; operator tables excluded), one RHS: add the phase index */
  BX_Q_PHASE_BYTES = 40
};

/* Evaluation phases, in stream order. */
enum {
  BX_PH_P2M = 0,     /* leaf samples to multipoles */
  BX_PH_M2M = 1,     /* upward pass, one launch per level */
  BX_PH_M2L = 2,     /* V list: multipole to local, all levels in one launch */
  BX_PH_P2L = 3,     /* X list: coarse leaf samples to local */
  BX_PH_L2L = 4,     /* downward pass, one launch per level */
  BX_PH_LEAF = 5,    /* near tables (U list), local expansions and W-list multipoles
                        to the nodes, in one fused kernel */
  BX_N_PHASES = 6
};
int bx_query(const bx_ctx *ctx, const bx_tree *tree, int what, double *out);

/*
 * Copy one host-side interaction list of a tree, for checks of the list
 * builder.  kind: 0 = U (target leaf, source leaf, config), 1 = V (target box,
 * source box, offset class), 2 = W (target leaf, source box, config),
 * 3 = X (target box, source leaf, config); boxes are given as
 * (level << 58 | ix << 29 | iy) keys, leaves by descriptor index.  With
 * out == NULL only *count is written; otherwise up to cap triples
 * (int64 each) are copied.
 */
int bx_tree_list(const bx_tree *tree, int kind, int64_t *out, int64_t cap, int64_t *count);

/*
 * Copy one of the context's host FP64 operator tables (after bx_build_tables),
 * for checks of the table builder.  which: 0 near tables [33][MR][P] (rows:
 * V for the P targets, dV/dx1, dV/dx2, then the mass row, zero padding to MR,
 * a multiple of 16), 1 P2M [2 KP][P], 2 M2M [4][p+1][p+1][2], 3 L2L
 * [4][p+1][p+1][2], 4 M2L core [KP][KP], 5 M2L source powers [49][KP][2],
 * 6 M2L target powers [49][KP][2], 7 log|d| [49], 8 L2T [3P][2 KP],
 * 9 M2T [20][3P][2 KP], 10 P2L [20][2 KP][P], 11 unit-box weights [P];
 * KP = p+1 rounded up to 16.  Split contexts also: 12 int8 slices of the near
 * tables [33][8][3P][P] (slice a of row r: T[r][k] ~ scale_r sum_a s_a
 * 2^-7(a+1)), 13 row scales [3P], 14 slice error bounds [2][9] (V rows, then
 * gradient rows; entry s: bound with s slices for samples |f| < 1).  With
 * out == NULL only *count is written.
 */
int bx_table_copy(const bx_ctx *ctx, int which, double *out, int64_t cap, int64_t *count);

/*
 * Split contexts: tolerance of the int8 slicing of the near tables.  The slice
 * count of each level (V rows and gradient rows separately) is the smallest
 * whose rigorous error bound (table and sample residuals and dropped slice
 * pairs, summed over all 33 configurations) is below tol * ||f||_inf * W^2 for
 * V and tol * ||f||_inf * W for grad V (W = root width).  Levels that would
 * need more than 6 slices (42 bits) evaluate their near field in FP64.  Takes
 * effect for trees uploaded after the call; default 1e-11.
 * Errors: BX_E_ARG.
 */
int bx_split_tolerance(bx_ctx *ctx, double tol);

/*
 * Scheduling parameters of a tree's evaluation (none changes any result: every
 * output is summed in the same order whatever they are):
 *   tune[0] heavy-tile threshold: a near tile whose cost exceeds this multiple
 *           of the balanced per-block share is split by rows (default 1.0,
 *           split contexts 1.5);
 *   tune[1] split contexts: cost of one FP64 slot of the near kernel, in int8
 *           slice pairs, for that balance (default 16);
 *   tune[2] persistent M2L blocks (default 4096);
 *   tune[3] M2M and L2L run two levels per launch where the middle level has
 *           at most this many internal boxes (default 0: never).
 * bx_tree_tuning sets them (tune[0..2] <= 0 or tune[3] = -1 keeps the current
 * value), rebuilds the work lists on the device (allocates; synchronizes
 * `stream`) and drops captured evaluation graphs.  bx_tree_tuning_get copies
 * the current ones.
 * Errors: BX_E_ARG (NULL, tune[2] not an integer in [1, 65535], tune[3] not an
 * integer >= -1), BX_E_HIP, BX_E_OOM.
 */
int bx_tree_tuning(bx_ctx *ctx, bx_tree *tree, const double tune[4], bx_stream_t stream);
int bx_tree_tuning_get(const bx_tree *tree, double tune[4]);

/*
 * Autotune a tree's scheduling parameters for one evaluation shape: runs
 * bx_volume_eval_grad(f_dev, n_rhs, V_dev, G_dev) for candidate settings, one
 * parameter at a time (M2L blocks, heavy threshold, FP64 slot weight,
 * two-level threshold), each
 * timed with device events as the median of 3 batches of `reps` evaluations,
 * and keeps the fastest.  V_dev and G_dev hold that evaluation's result on
 * return.  best (may be NULL) receives the chosen tune[0..3] and, in best[4],
 * the median milliseconds per evaluation with them.  Synchronizes `stream`;
 * not for use while other work on the tree is in flight.
 * Errors: as bx_volume_eval_grad and bx_tree_tuning; BX_E_ARG if reps < 1.
 */
int bx_autotune(bx_ctx *ctx, bx_tree *tree, const double *f_dev, int n_rhs, double *V_dev, double *G_dev,
                int reps, double best[5], bx_stream_t stream);

/*
 * The piecewise polynomial v~ of section 3.1 (the interpolant, on each leaf, of
 * values computed at its collocation nodes) and likewise of the gradient, at
 * arbitrary points.  Each target (x, y) is located in the tree (the leaf whose
 * closed-open square [x0, x0 + h) x [y0, y0 + h) holds it; the root's right and
 * top edges belong to the last leaves) and the tensor Chebyshev interpolant of
 * that leaf's n x n values is evaluated (barycentric form, first-kind nodes).
 *   V, G:    device, as written by bx_volume_eval_grad for n_rhs right-hand
 *            sides; either may be NULL to skip it (not both).
 *   xy:      device [n_targets][2] (x, y) in the tree's coordinates.
 *   v_out:   device [n_rhs][n_targets] (needed iff V != NULL);
 *   g_out:   device [n_rhs][n_targets][2] (needed iff G != NULL); caller-owned.
 * Targets outside the root box get NaN.  Stream-ordered; no allocation.
 * Errors: BX_E_ARG, BX_E_HIP.
 */
int bx_interpolate(const bx_ctx *ctx, const bx_tree *tree, const double *V, const double *G, int n_rhs,
                   const double *xy, int64_t n_targets, double *v_out, double *g_out, bx_stream_t stream);

/*
 * Per-phase timing with HIP events recorded on the evaluation stream.
 * bx_profile(ctx, 1) makes later evaluations record an event pair around each
 * phase; bx_profile_read waits for the recorded events, adds their elapsed
 * times to ms[phase] (BX_N_PHASES entries, caller-owned), writes the number of
 * timed evaluations to *n_evals and clears the record.  Recording adds a few
 * microseconds per phase.  Errors: BX_E_ARG, BX_E_HIP.
 */
/*
 * Copy one box's expansion from the last evaluation to the host (synchronizes
 * `stream`).  which 0: the multipole phi(z) = a_0 log(z - c) + sum_k a_k
 * (z - c)^-k of the sources in the box (the far field of section 3.1, a_0 = the
 * integral of f~ over the box); 1: the local expansion psi(z) = sum_l b_l
 * (z - c)^l of the sources far from it; V = Re(phi or psi) / 2 pi; c the box
 * centre, z = x1 + i x2.  out[2k], out[2k+1] = Re, Im of a_k (or b_k), k = 0..p,
 * unscaled (the library stores them scaled by powers of the box width).  box:
 * the library's box index (0 .. n_trees - 1 are the roots); rhs < the n_rhs
 * of the last evaluation.
 * Errors: BX_E_ARG (bad box, rhs, which or NULL), BX_E_UNSUPPORTED (no
 * evaluation yet), BX_E_HIP.
 */
int bx_expansion_read(const bx_ctx *ctx, const bx_tree *tree, int which, int64_t box, int rhs, double *out_host,
                      bx_stream_t stream);
int bx_profile(bx_ctx *ctx, int enable);
int bx_profile_read(bx_ctx *ctx, double *ms, int *n_evals);

void bx_tree_destroy(bx_tree *tree);
void bx_destroy(bx_ctx *ctx);
const char *bx_last_error(void);

/* ------------------------------------------------------------------------
 * Learned refinement (the adaptive refinement of section 3.1 proposed by a
 * small network; the plain tail criterion still checks every leaf).
 *
 * A perceptron 288 -> 128 -> 128 -> 1 (ReLU) proposes whether a quadtree box
 * is split.  Its inputs are features of the box (bx_mlp_features); its
 * output is a logit, split proposed when positive.  Matrix products run on
 * BF16 operands with FP32 sums; parameters, gradients and Adam moments are
 * FP32.  Parameter vector (flat, BX_MLP_NPARAMS floats): W1[128][288],
 * b1[128], W2[128][128], b2[128], w3[128], b3.
 * ---------------------------------------------------------------------- */
typedef struct bx_mlp bx_mlp;
#define BX_MLP_IN 288
#define BX_MLP_NPARAMS 53633

/*
 * Features of n_boxes boxes: samples_dev[n_boxes][16][16] (FP64, the source
 * at the 16 x 16 first-kind Chebyshev points of each box, x index fastest)
 * and level_dev[n_boxes] (int8) -> x_dev[n_boxes][288] BF16 (raw uint16):
 * x[k] = s_k / max|s| (k < 256; 0 if all samples are 0), x[256] = level/16,
 * x[257] = clip((log10 max|s| + 10) / 10, -1, 2) and x[258] =
 * max(log10 max|s|, -320) / 320 (both -1 if all are 0), then zeros.  All device pointers, x_dev 16-byte aligned; stream-ordered.
 * Errors: BX_E_ARG (NULL, n_boxes < 0, misaligned), BX_E_HIP.
 */
int bx_mlp_features(const double *samples_dev, const int8_t *level_dev, int64_t n_boxes, uint16_t *x_dev,
                    bx_stream_t stream);

/*
 * Create a network on the current device with parameters params_host
 * (BX_MLP_NPARAMS floats, copied; NULL: all zero) and zero Adam state.
 * bx_mlp_set_params replaces the parameters and resets the Adam state.
 * Both synchronize `stream`.  Errors: BX_E_ARG, BX_E_HIP, BX_E_OOM.
 */
int bx_mlp_create(bx_mlp **out, const float *params_host, bx_stream_t stream);
int bx_mlp_set_params(bx_mlp *net, const float *params_host, bx_stream_t stream);

/*
 * Logits of n boxes: x_dev[n][288] BF16 (16-byte aligned) -> logit_dev[n]
 * FP32.  Stream-ordered.  Errors: BX_E_ARG, BX_E_HIP.
 */
int bx_mlp_forward(const bx_mlp *net, const uint16_t *x_dev, int64_t n, float *logit_dev, bx_stream_t stream);

/*
 * Gradient of the mean binary cross-entropy of sigmoid(logit) against
 * labels y_dev[n] (FP32, 0 or 1) over the n boxes x_dev, held in the
 * network (read with bx_mlp_read); the mean loss likewise.  The products
 * round h1 and the back-propagated dL/dz2 and dL/dz1 to BF16 as operands;
 * sums over boxes use FP32 atomics, so their order (and the last bits)
 * varies from call to call.  Stream-ordered.  Errors: BX_E_ARG, BX_E_HIP.
 */
int bx_mlp_grad(bx_mlp *net, const uint16_t *x_dev, const float *y_dev, int64_t n, bx_stream_t stream);

/*
 * One Adam step (Kingma and Ba) with the held gradient: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),
 * t counting the calls since the parameters were set.  Stream-ordered.
 * Errors: BX_E_ARG (lr < 0, betas outside [0, 1), eps <= 0).
 */
int bx_mlp_adam(bx_mlp *net, float lr, float beta1, float beta2, float eps, bx_stream_t stream);

/*
 * Copy network state to the host (synchronizes `stream`): which 0 parameters,
 * 1 gradient, 2 Adam m, 3 Adam v (BX_MLP_NPARAMS floats each), 4 the mean
 * loss of the last bx_mlp_grad (1 float).  Errors: BX_E_ARG (cap too small).
 */
int bx_mlp_read(const bx_mlp *net, int which, float *out_host, int64_t cap, bx_stream_t stream);
void bx_mlp_destroy(bx_mlp *net);

#ifdef __cplusplus
}
#endif
#endif /* BOXFMM_H */
