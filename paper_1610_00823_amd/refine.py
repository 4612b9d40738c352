"""Learned refinement of the box-code quadtree (section 3.1's adaptive
refinement, with the network as a proposer).

The plain method refines top-down: a box splits while the tail of the
Chebyshev coefficients of its n x n interpolant exceeds tol (the tail
criterion).  For a general source the criterion only sees the n x n samples,
so a feature narrower than the node spacing is invisible and the box stops
too early (for the synthetic Gaussian sums the seed rule, which knows the
centres and widths, covers this; a general f offers no such knowledge).

Here a small network (bx_mlp_*, BF16 kernels) reads the source on a finer
16 x 16 first-kind grid of each box, plus the box level, and proposes split
or no split.  It is trained on the decisions of the plain criterion with the
seed rule.  The plain tail criterion then checks every proposed leaf: a leaf
that fails it is refined further by the plain method (the fallback), so every
leaf of the final tree passes the criterion, as in the plain method.

Sampling f, the tail criterion and the 2:1 balance run on the host (the tree
is an input of the box code); features, inference and training run in the
library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import boxfmm as B
from . import inputs as I

GRID = 16   # samples per side of the network's view of a box


def grid_samples(fun, level, bx, by, cx=0.0, cy=0.0, width=1.0) -> np.ndarray:
    """f on the 16 x 16 first-kind grid of each box: [B, 16, 16] float64."""
    X, Y = I.box_grid(level, bx, by, GRID, cx, cy, width)
    return np.ascontiguousarray(np.asarray(fun(X, Y), np.float64))


def _label_job(args):
    fun, n, tol, cap, cx, cy, width, seeds, widths = args
    rec = []
    I.adaptive_tree(fun, n, tol, cap, cx=cx, cy=cy, width=width, seed_points=seeds, seed_widths=widths, record=rec)
    lv = np.concatenate([r[0] for r in rec])
    bx = np.concatenate([r[1] for r in rec])
    by = np.concatenate([r[2] for r in rec])
    y = np.concatenate([r[3] for r in rec])
    return grid_samples(fun, lv, bx, by, cx, cy, width), lv.astype(np.int8), y.astype(np.float32)


def labelled_boxes(jobs, workers: int = 16):
    """Training boxes: for each job (fun, n, tol, cap, cx, cy, width, seed
    points, seed widths) every box the plain criterion visits, with its 16 x 16
    samples, level and decision.  Returns (samples [N,16,16], level [N] int8, y [N])."""
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            out = pool.map(_label_job, jobs)
    else:
        out = [_label_job(j) for j in jobs]
    return (np.concatenate([o[0] for o in out]), np.concatenate([o[1] for o in out]),
            np.concatenate([o[2] for o in out]))


def source_jobs(seeds, kinds=("gauss20",), n=8, tol=1e-10, cap=12):
    """Label jobs for seeded synthetic sources: 'gauss20' (20 Gaussians), 'gaussK'
    (1 to 40 Gaussians, count drawn from the seed), 'kink' (the C0 kink source)."""
    jobs = []
    for s in seeds:
        for kind in kinds:
            if kind == "kink":
                jobs.append((I.kink_source, n, tol, cap, 0.0, 0.0, 1.0, None, None))
                continue
            K = 20 if kind == "gauss20" else int(np.random.default_rng([s, 7]).integers(1, 41))
            src = I.random_gaussians(s, K)
            jobs.append((src, n, tol, cap, 0.0, 0.0, 1.0, src.c, src.sigma))
    return jobs


@dataclass
class BuildStats:
    net_boxes: int = 0          # boxes the network decided
    net_f_evals: int = 0        # f samples it read (16 x 16 per box)
    proposed_leaves: int = 0
    verify_f_evals: int = 0     # n x n samples of the plain check of every proposed leaf
    failed_leaves: int = 0      # proposed leaves the plain criterion refined further
    fallback_f_evals: int = 0
    leaves: int = 0             # after the 2:1 balance
    seconds: dict = field(default_factory=dict)

    @property
    def f_evals(self):
        return self.net_f_evals + self.verify_f_evals + self.fallback_f_evals


class LearnedRefiner:
    """Trains the refinement network and builds trees with it (one GPU)."""

    def __init__(self, params=None, seed: int = 0):
        self.net = B.RefineNet(I.refine_net_init(seed) if params is None else params)

    # --------------------------------------------------------------- training
    def features(self, samples: np.ndarray, level: np.ndarray):
        import torch
        s = torch.from_numpy(np.ascontiguousarray(samples, np.float64)).cuda()
        lv = torch.from_numpy(np.ascontiguousarray(level, np.int8)).cuda()
        return B.mlp_features(s, lv)

    def train(self, x, y, epochs: int = 4, batch: int = 1024, lr: float = 2e-3, seed: int = 0, log=None):
        """Adam on the mean binary cross-entropy over minibatches of the
        features x [N, 288] (GPU, bfloat16) and labels y [N] (0/1); the box
        order of each epoch is a seeded permutation.  Returns the mean loss per epoch."""
        import torch
        yt = torch.as_tensor(np.asarray(y, np.float32)).cuda() if not torch.is_tensor(y) else y
        N = x.shape[0]
        rng = np.random.default_rng(seed)
        losses = []
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(N)).cuda()
            for s0 in range(0, N, batch):
                idx = perm[s0:s0 + batch]
                xb = x.index_select(0, idx).contiguous()
                yb = yt.index_select(0, idx).contiguous()
                self.net.grad(xb, yb)
                self.net.adam(lr)
            # mean loss over the whole set with the epoch's final parameters
            losses.append(self.loss(x, yt))
            if log:
                log(f"epoch {ep}: loss {losses[-1]:.4f}")
        return losses

    def loss(self, x, y):
        import torch
        z = self.net.forward(x).double()
        yy = y.double()
        return float((torch.clamp(z, min=0) - z * yy + torch.log1p(torch.exp(-z.abs()))).mean())

    def predict(self, x):
        return (self.net.forward(x) > 0).cpu().numpy()

    # --------------------------------------------------------------- building
    def propose(self, samples: np.ndarray, level: np.ndarray, batch: int = 1 << 16) -> np.ndarray:
        """The network's split proposals for boxes with 16 x 16 samples and levels."""
        out = np.zeros(len(level), bool)
        for a in range(0, len(level), batch):
            out[a:a + batch] = self.predict(self.features(samples[a:a + batch], level[a:a + batch]))
        return out

    def build(self, funs, n: int = 8, tol: float = 1e-10, cap: int = 12, cx=0.0, cy=0.0, width=1.0):
        return build_trees(funs, self.propose, n, tol, cap, cx, cy, width)


def build_trees(funs, propose, n: int = 8, tol: float = 1e-10, cap: int = 12, cx=0.0, cy=0.0, width=1.0):
    """Trees for the sources `funs` (one per source): `propose(samples [B,16,16],
    level [B] int8) -> split [B]` decides the refinement level by level for all
    sources at once, the plain tail criterion checks each proposed leaf and
    refines the failures, then each tree is 2:1 balanced.  Returns (trees, BuildStats)."""
    st = BuildStats()
    t_all = time.perf_counter()
    T = {"sample": 0.0, "propose": 0.0, "verify": 0.0, "fallback": 0.0, "balance": 0.0}
    S = len(funs)
    src = np.arange(S)
    lv = np.zeros(S, np.int64)
    bx = np.zeros(S, np.int64)
    by = np.zeros(S, np.int64)
    prop = [[] for _ in range(S)]
    cxx = np.array([0, 1, 0, 1])
    cyy = np.array([0, 0, 1, 1])
    while len(lv):
        t0 = time.perf_counter()
        samples = np.empty((len(lv), GRID, GRID))
        for s in np.unique(src):
            sel = np.flatnonzero(src == s)
            samples[sel] = grid_samples(funs[s], lv[sel], bx[sel], by[sel], cx, cy, width)
        T["sample"] += time.perf_counter() - t0
        t0 = time.perf_counter()
        split = np.asarray(propose(samples, lv.astype(np.int8)), bool) & (lv < cap)
        T["propose"] += time.perf_counter() - t0
        st.net_boxes += len(lv)
        st.net_f_evals += samples.size
        for s in np.unique(src[~split]):
            sel = np.flatnonzero((src == s) & ~split)
            prop[s].append((lv[sel], bx[sel], by[sel]))
        k = np.flatnonzero(split)
        src = np.repeat(src[k], 4)
        bx, by = (2 * bx[k][:, None] + cxx).ravel(), (2 * by[k][:, None] + cyy).ravel()
        lv = np.repeat(lv[k] + 1, 4)
    trees = []
    for s in range(S):
        pl = [np.concatenate([p[k] for p in prop[s]]) for k in range(3)]
        st.proposed_leaves += len(pl[0])
        t0 = time.perf_counter()
        bad, ne = I.split_decision(funs[s], pl[0], pl[1], pl[2], n, tol, cap, cx=cx, cy=cy, width=width)
        T["verify"] += time.perf_counter() - t0
        st.verify_f_evals += ne
        st.failed_leaves += int(bad.sum())     # the plain criterion splits these further
        keep = [a[~bad] for a in pl]
        if bad.any():
            # the check already decided that these leaves split: the plain method
            # continues from their children
            t0 = time.perf_counter()
            kids = (np.repeat(pl[0][bad] + 1, 4), (2 * pl[1][bad][:, None] + cxx).ravel(),
                    (2 * pl[2][bad][:, None] + cyy).ravel())
            fb = I.adaptive_tree(funs[s], n, tol, cap, cx=cx, cy=cy, width=width, roots=kids)
            T["fallback"] += time.perf_counter() - t0
            st.fallback_f_evals += fb.meta["f_evals"]
            keep = [np.concatenate([k_, f_]) for k_, f_ in zip(keep, fb.meta["leaves"])]
        t0 = time.perf_counter()
        lvb, xs, ys = I.balance(*keep)
        T["balance"] += time.perf_counter() - t0
        trees.append(I.Tree(lvb, xs, ys, cx, cy, width, {"kind": "learned", "tol": tol, "max_level": cap, "n": n,
                                                          "leaves_unbalanced": tuple(keep)}))
        st.leaves += len(lvb)
    T["total"] = time.perf_counter() - t_all
    st.seconds = T
    return trees, st


def plain_trees(funs, n=8, tol=1e-10, cap=12, cx=0.0, cy=0.0, width=1.0):
    """The plain method on the same sources (tail criterion only), with its f evaluations."""
    out, ev = [], 0
    for f in funs:
        t = I.adaptive_tree(f, n, tol, cap, cx=cx, cy=cy, width=width)
        ev += t.meta["f_evals"]
        out.append(t)
    return out, ev


def resolution_error(tree, fun, n: int = 8, m: int = 12, points=None) -> float:
    """max |f - f~| / max |f| over an m x m grid in every leaf plus `points`
    (e.g. the centres of narrow bumps), f~ the leaf's n x n interpolant."""
    xi = I.cheb1_nodes(n)
    # Lagrange basis of the n first-kind points at local coordinates t
    def lag(t):
        t = np.asarray(t, np.float64)
        L = np.ones(t.shape + (n,))
        for j in range(n):
            for k in range(n):
                if k != j:
                    L[..., j] *= (t - xi[k]) / (xi[j] - xi[k])
        return L
    f = I.sample(tree, fun, n)                      # [N_L, n, n] (y, x)
    tu = (np.arange(m) + 0.5) / m * 2 - 1
    Lu = lag(tu)                                    # [m, n]
    ft = np.einsum("aj,ljk,bk->lab", Lu, f, Lu)     # [N_L, m(y), m(x)]
    h = tree.width * np.ldexp(1.0, -tree.level.astype(np.int64))
    x0 = tree.cx - 0.5 * tree.width + tree.ix * h
    y0 = tree.cy - 0.5 * tree.width + tree.iy * h
    X = (x0 + 0.5 * h)[:, None, None] + 0.5 * h[:, None, None] * tu[None, None, :]
    Y = (y0 + 0.5 * h)[:, None, None] + 0.5 * h[:, None, None] * tu[None, :, None]
    X, Y = np.broadcast_to(X, ft.shape), np.broadcast_to(Y, ft.shape)
    fx = np.asarray(fun(X, Y), np.float64)
    err = np.abs(fx - ft).max()
    scale = np.abs(fx).max()
    if points is not None and len(points):
        pts = np.asarray(points, np.float64).reshape(-1, 2)
        key = {(int(l), int(x), int(y)): i for i, (l, x, y) in enumerate(zip(tree.level, tree.ix, tree.iy))}
        for px, py in pts:
            for l in range(int(tree.level.max()) + 1):
                hh = tree.width / (1 << l)
                ix = int(np.floor((px - tree.cx + 0.5 * tree.width) / hh))
                iy = int(np.floor((py - tree.cy + 0.5 * tree.width) / hh))
                i = key.get((l, ix, iy))
                if i is None:
                    continue
                tx = (px - (x0[i] + 0.5 * h[i])) / (0.5 * h[i])
                ty = (py - (y0[i] + 0.5 * h[i])) / (0.5 * h[i])
                v = lag(ty) @ f[i] @ lag(tx)
                fv = float(fun(np.array(px), np.array(py)))
                err = max(err, abs(fv - v))
                scale = max(scale, abs(fv))
                break
    return float(err / scale) if scale > 0 else 0.0
