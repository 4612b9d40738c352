"""Seeded synthetic inputs for the box-code volume potential.

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds no arithmetic of the volume potential itself: it only
draws source functions, builds level-restricted quadtrees (the tree is an
input to the box code, built before it runs, as in the paper's section 3.1
and section 6.1), and samples the source at each leaf's collocation nodes.

Conventions
-----------
* Root box: centre (cx, cy), width ``width``; a box at level l has width
  ``width * 2**-l`` and integer position (ix, iy), 0 <= ix, iy < 2**l, counted
  from the lower-left corner of the root.
* Collocation nodes: first-kind Chebyshev points on [-1, 1],
  xi_j = -cos((2j+1) pi / (2n)), j = 0..n-1 (increasing), scaled to the box.
  Samples are stored f[leaf, j2, j1] with the x index (j1) fastest.
* Refinement (section 3.1 and section 6.1): a box is split while the tail of
  its Chebyshev coefficients exceeds ``tol`` and its level is below
  ``max_level``; the tail is the largest |c_ab| with max(a, b) >= n - 2.  For
  sums of narrow Gaussians a box containing a centre is also split while its
  width exceeds 4 sigma (a coarse sampling can miss a narrow bump entirely).
  The tree is then made level-restricted (adjacent leaves, corners included,
  differ by at most one level).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Tree:
    """A leaf set of a level-restricted quadtree on a square root box."""
    level: np.ndarray          # int8  [N_L]
    ix: np.ndarray             # int32 [N_L]
    iy: np.ndarray             # int32 [N_L]
    cx: float = 0.0
    cy: float = 0.0
    width: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n_leaves(self) -> int:
        return int(self.level.shape[0])

    def box_width(self) -> np.ndarray:
        return self.width * np.ldexp(1.0, -self.level.astype(np.int64))

    def box_centre(self):
        h = self.box_width()
        x = self.cx - 0.5 * self.width + (self.ix + 0.5) * h
        y = self.cy - 0.5 * self.width + (self.iy + 0.5) * h
        return x, y


def cheb1_nodes(n: int) -> np.ndarray:
    """First-kind Chebyshev points on [-1, 1], increasing."""
    j = np.arange(n, dtype=np.float64)
    return -np.cos((2.0 * j + 1.0) * np.pi / (2.0 * n))


def node_coords(tree: Tree, n: int):
    """Physical coordinates of every collocation node, shape [N_L, n, n] (x index fastest)."""
    xi = cheb1_nodes(n)
    xc, yc = tree.box_centre()
    h = tree.box_width()
    X = xc[:, None, None] + 0.5 * h[:, None, None] * xi[None, None, :]
    Y = yc[:, None, None] + 0.5 * h[:, None, None] * xi[None, :, None]
    X = np.broadcast_to(X, (tree.n_leaves, n, n)).copy()
    Y = np.broadcast_to(Y, (tree.n_leaves, n, n)).copy()
    return X, Y


def sample(tree: Tree, fun: Callable, n: int) -> np.ndarray:
    """f sampled at every leaf's collocation nodes, float64 [N_L, n, n]."""
    X, Y = node_coords(tree, n)
    return np.ascontiguousarray(fun(X, Y), dtype=np.float64)


# ---------------------------------------------------------------- sources
@dataclass
class GaussianSum:
    """f(x) = sum_i a_i exp(-|x - c_i|^2 / sigma_i^2)."""
    a: np.ndarray
    sigma: np.ndarray
    c: np.ndarray              # [K, 2]

    def __call__(self, x, y):
        out = np.zeros(np.broadcast(x, y).shape)
        for a, s, (c1, c2) in zip(self.a, self.sigma, self.c):
            out += a * np.exp(-((x - c1) ** 2 + (y - c2) ** 2) / (s * s))
        return out


def centred_gaussian(sigma: float = 0.1) -> GaussianSum:
    """The single centred Gaussian exp(-|x|^2 / sigma^2)."""
    return GaussianSum(np.array([1.0]), np.array([sigma]), np.zeros((1, 2)))


def random_gaussians(seed: int, K: int = 20, amp=(-1.0, 1.0), log_sigma=(1e-3, 1e-1),
                     centre=(-0.4, 0.4)) -> GaussianSum:
    """K Gaussians: amplitudes U(amp), widths log-uniform in log_sigma, centres U(centre)^2.

    Draw order (numpy default_rng(seed), PCG64): a, then sigma, then c.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(amp[0], amp[1], K)
    s = np.exp(rng.uniform(np.log(log_sigma[0]), np.log(log_sigma[1]), K))
    c = rng.uniform(centre[0], centre[1], (K, 2))
    return GaussianSum(a, s, c)


def kink_source(x, y):
    """C^0 source with a kink across the curve r = 0.3 + 0.05 cos(5 theta).

    phi = r - (0.3 + 0.05 cos 5 theta); f = sin(4 pi x) cos(4 pi y) inside
    (phi < 0) and the same times exp(-20 phi) outside: continuous, kinked.
    """
    r = np.hypot(x, y)
    th = np.arctan2(y, x)
    phi = r - (0.3 + 0.05 * np.cos(5.0 * th))
    base = np.sin(4.0 * np.pi * x) * np.cos(4.0 * np.pi * y)
    return np.where(phi < 0.0, base, base * np.exp(-20.0 * np.minimum(np.maximum(phi, 0.0), 50.0)))


# ---------------------------------------------------------------- trees
def uniform_tree(depth: int, cx=0.0, cy=0.0, width=1.0) -> Tree:
    m = 1 << depth
    iy, ix = np.meshgrid(np.arange(m, dtype=np.int32), np.arange(m, dtype=np.int32), indexing="ij")
    # Morton order is not required: any leaf order is accepted by the library.
    return Tree(np.full(m * m, depth, np.int8), ix.ravel().copy(), iy.ravel().copy(), cx, cy, width,
                {"kind": "uniform", "depth": depth})


def _cheb_tail(vals: np.ndarray, n: int) -> np.ndarray:
    """Largest |c_ab| with max(a,b) >= n-2 of the tensor interpolants of vals[B, n, n]."""
    j = np.arange(n)
    theta = (2.0 * (n - 1 - j) + 1.0) * np.pi / (2.0 * n)     # xi_j = cos(theta_j)
    a = np.arange(n)
    T = np.cos(a[:, None] * theta[None, :])                    # T[a, j] = T_a(xi_j)
    wgt = np.where(a == 0, 1.0, 2.0) / n
    Tm = T * wgt[:, None]
    C = np.einsum("aj,bk,ikj->iba", Tm, Tm, vals, optimize=True)   # C[i, b, a]: b along y, a along x
    mask = np.zeros((n, n), bool)
    mask[n - 2:, :] = True
    mask[:, n - 2:] = True
    return np.abs(C[:, mask]).max(axis=1) if vals.shape[0] else np.zeros(0)


def balance(level, ix, iy):
    """Make a leaf set level-restricted (corner adjacency) by splitting coarse leaves."""
    leaves = {(int(l), int(x), int(y)) for l, x, y in zip(level, ix, iy)}
    boxes = set()
    for (l, x, y) in leaves:
        while True:
            boxes.add((l, x, y))
            if l == 0:
                break
            l, x, y = l - 1, x >> 1, y >> 1
    maxl = max(l for l, _, _ in leaves)
    by_level = {l: [] for l in range(maxl + 1)}
    for b in leaves:
        by_level[b[0]].append(b)

    def split(b):
        l, x, y = b
        leaves.discard(b)
        for cy in (0, 1):
            for cx in (0, 1):
                c = (l + 1, 2 * x + cx, 2 * y + cy)
                leaves.add(c)
                boxes.add(c)
                by_level[l + 1].append(c)

    for l in range(maxl, 1, -1):
        m = 1 << l
        for b in list(by_level[l]):
            if b not in leaves:
                continue
            _, x, y = b
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    nx, ny = x + dx, y + dy
                    if (dx == 0 and dy == 0) or not (0 <= nx < m and 0 <= ny < m):
                        continue
                    target = (l - 1, nx >> 1, ny >> 1)
                    # split the covering leaf until the level l-1 box exists
                    while target not in boxes:
                        tl, tx, ty = target
                        k = 1
                        anc = (tl - k, tx >> k, ty >> k)
                        while anc not in boxes:
                            k += 1
                            anc = (tl - k, tx >> k, ty >> k)
                        assert anc in leaves
                        split(anc)
    out = sorted(leaves)
    lv = np.array([b[0] for b in out], np.int8)
    xs = np.array([b[1] for b in out], np.int32)
    ys = np.array([b[2] for b in out], np.int32)
    return lv, xs, ys


def box_grid(level, bx, by, m: int, cx=0.0, cy=0.0, width=1.0):
    """Coordinates X, Y [B, m, m] (x index fastest) of the m x m first-kind
    Chebyshev points of boxes (level, bx, by)."""
    xi = cheb1_nodes(m)
    lv = np.asarray(level, np.int64)
    h = width * np.ldexp(1.0, -lv)
    x0 = cx - 0.5 * width + np.asarray(bx, np.int64) * h
    y0 = cy - 0.5 * width + np.asarray(by, np.int64) * h
    X = (x0 + 0.5 * h)[:, None, None] + 0.5 * h[:, None, None] * xi[None, None, :]
    Y = (y0 + 0.5 * h)[:, None, None] + 0.5 * h[:, None, None] * xi[None, :, None]
    B = len(lv)
    return np.broadcast_to(X, (B, m, m)), np.broadcast_to(Y, (B, m, m))


def split_decision(fun: Callable, level, bx, by, n: int, tol: float, max_level: int, min_level: int = 0,
                   cx=0.0, cy=0.0, width=1.0, seed_points=None, seed_widths=None, weight: str = "none"):
    """The plain criterion's decision for boxes (level, bx, by): split when the
    tail of the n x n interpolant exceeds tol (weighted by h^2 or h with
    weight='area' / 'side'), below min_level, or (seed rule) when the box holds
    a seed point and is wider than 4 of its widths; never at max_level.
    Returns (split [B] bool, f evaluations used)."""
    lv = np.asarray(level, np.int64)
    if len(lv) == 0:
        return np.zeros(0, bool), 0
    X, Y = box_grid(lv, bx, by, n, cx, cy, width)
    vals = np.asarray(fun(X, Y), np.float64)
    h = width * np.ldexp(1.0, -lv)
    tail = _cheb_tail(vals, n)
    if weight == "area":
        tail = tail * h * h
    elif weight == "side":
        tail = tail * h
    split = (tail > tol) | (lv < min_level)
    if seed_points is not None:
        x0 = cx - 0.5 * width + np.asarray(bx, np.int64) * h
        y0 = cy - 0.5 * width + np.asarray(by, np.int64) * h
        for (px, py), sg in zip(seed_points, seed_widths):
            inside = (px >= x0) & (px < x0 + h) & (py >= y0) & (py < y0 + h)
            split |= inside & (h > 4.0 * sg)
    split &= lv < max_level
    return split, vals.size


def adaptive_tree(fun: Callable, n: int, tol: float = 1e-10, max_level: int = 14,
                  min_level: int = 0, cx=0.0, cy=0.0, width=1.0,
                  seed_points: Optional[np.ndarray] = None, seed_widths: Optional[np.ndarray] = None,
                  weight: str = "none", record: Optional[list] = None, roots=None) -> Tree:
    """Top-down refinement with the tail criterion, then 2:1 balance.

    weight='none' compares the tail itself with tol; weight='area' multiplies it
    by the box area (h^2) and 'side' by the side length, the weighted variants of
    section 6.1.  With `record` (a list) every visited box is appended as
    arrays (level, bx, by, split) per level.  `roots` (level, bx, by arrays)
    starts the refinement from those boxes instead of the root; their
    refinement is returned unbalanced (meta 'leaves').
    """
    if roots is None:
        todo = (np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(1, np.int64))
    else:
        todo = tuple(np.asarray(a, np.int64) for a in roots)
    leaves = [[], [], []]
    n_evals = 0
    while len(todo[0]):
        lv, bx, by = todo
        split, ne = split_decision(fun, lv, bx, by, n, tol, max_level, min_level, cx, cy, width, seed_points,
                                   seed_widths, weight)
        n_evals += ne
        if record is not None:
            record.append((lv, bx, by, split))
        keep = ~split
        for k, a in enumerate((lv, bx, by)):
            leaves[k].append(a[keep])
        sl, sx, sy = lv[split], bx[split], by[split]
        cxx = np.array([0, 1, 0, 1])
        cyy = np.array([0, 0, 1, 1])
        todo = (np.repeat(sl + 1, 4), (2 * sx[:, None] + cxx).ravel(), (2 * sy[:, None] + cyy).ravel())
    lv, xs, ys = (np.concatenate(a) for a in leaves)
    meta = {"kind": "adaptive", "tol": tol, "max_level": max_level, "n": n, "leaves_before_balance": len(lv),
            "f_evals": n_evals}
    if roots is not None:
        meta["leaves"] = (lv, xs, ys)
        return Tree(lv.astype(np.int8), xs.astype(np.int32), ys.astype(np.int32), cx, cy, width, meta)
    lv, xs, ys = balance(lv, xs, ys)
    return Tree(lv, xs, ys, cx, cy, width, meta)


def gaussian_tree(src: GaussianSum, n: int, tol=1e-10, max_level=14) -> Tree:
    """Adaptive tree for a Gaussian sum, with the narrow-feature seed rule."""
    return adaptive_tree(src, n, tol, max_level, seed_points=src.c, seed_widths=src.sigma)


def point_refined_tree(points, depths, cx=0.0, cy=0.0, width=1.0) -> Tree:
    """Graded tree: boxes containing points[i] are split down to level depths[i], then balanced."""
    pts = np.asarray(points, float).reshape(-1, 2)
    sig = width * np.ldexp(1.0, -np.asarray(depths, np.int64)) / 4.0 * 1.0000001
    zero = lambda x, y: np.zeros(np.broadcast(x, y).shape)
    t = adaptive_tree(zero, 2, 1.0, int(max(depths)), cx=cx, cy=cy, width=width,
                      seed_points=pts, seed_widths=sig)
    t.meta = {"kind": "graded", "points": pts.tolist(), "depths": list(map(int, depths))}
    return t


def is_balanced(tree: Tree) -> bool:
    lv, xs, ys = balance(tree.level, tree.ix, tree.iy)
    return len(lv) == tree.n_leaves


def _forest_tree(args):
    k, seed, n, with_samples = args
    r = np.random.default_rng([seed, k])
    K, cap = int(r.integers(1, 41)), int(r.integers(6, 13))
    src = random_gaussians(100000 * seed + k, K)
    t = gaussian_tree(src, n, 1e-10, cap)
    return t, src, (sample(t, src, n) if with_samples else None)


def forest(count: int, seed: int = 0, n: int = 8, workers: int = 16, samples: bool = False):
    """`count` trees of uneven depth: tree k draws its Gaussian count in [1, 40] and
    its depth cap in [6, 12] from a generator seeded by (seed, k), and its sources
    like the 20-Gaussian workload (seed 100000 seed + k); built in a process pool.
    Returns (trees, sources), or with samples=True (trees, sources, samples of each
    tree at its n x n nodes), the sampling done in the same pool."""
    import multiprocessing as mp
    jobs = [(k, seed, n, samples) for k in range(count)]
    if workers > 1 and count > 1:
        with mp.get_context("fork").Pool(min(workers, count)) as pool:
            out = pool.map(_forest_tree, jobs)
    else:
        out = [_forest_tree(j) for j in jobs]
    if samples:
        return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out]
    return [o[0] for o in out], [o[1] for o in out]


def _polar_curve(theta, c0, cos_terms, sin_terms):
    r = np.full_like(theta, c0)
    for j, c in cos_terms.items():
        r = r + c * np.cos(j * theta)
    for j, d in sin_terms.items():
        r = r + d * np.sin(j * theta)
    return r


def paper_domain(x, y):
    """Indicator of the multiply connected domain of the paper's section 6: the
    region between two polar curves r(theta) = c0 + sum_j (c_j cos j theta +
    d_j sin j theta), the outer with c0 = 0.25, d3 = c6 = c8 = c10 = 0.01,
    c5 = 0.02, the inner with c0 = 0.05, c2 = d3 = c5 = c7 = 0.005."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    r, th = np.hypot(x, y), np.arctan2(y, x)
    outer = _polar_curve(th, 0.25, {5: 0.02, 6: 0.01, 8: 0.01, 10: 0.01}, {3: 0.01})
    inner = _polar_curve(th, 0.05, {2: 0.005, 5: 0.005, 7: 0.005}, {3: 0.005})
    return (r < outer) & (r > inner)


def paper_example_rhs(example: int):
    """f = Laplacian of the exact solutions of the paper's Examples 1 and 2
    (u = sin(10(x1 + x2)) + x1^2 - 3 x2 + 8, plus exp(-500 x1^2) in Example 2)
    inside the domain, extended by zero outside it."""
    def f(x, y):
        x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
        v = -200.0 * np.sin(10.0 * (x + y)) + 2.0
        if example == 2:
            v = v + (1e6 * x * x - 1000.0) * np.exp(-500.0 * x * x)
        return np.where(paper_domain(x, y), v, 0.0)
    return f


def refine_net_init(seed: int) -> np.ndarray:
    """Initial parameters of the refinement network (flat: W1[128][288], b1[128],
    W2[128][128], b2[128], w3[128], b3[1]): He-uniform weights (bound
    sqrt(6 / fan_in), fan_in 258 for the 258 live inputs of W1), zero biases,
    drawn from default_rng(seed) in that order and rounded to FP32."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (128, 288)) * np.sqrt(6.0 / 258.0)
    W2 = rng.uniform(-1, 1, (128, 128)) * np.sqrt(6.0 / 128.0)
    w3 = rng.uniform(-1, 1, 128) * np.sqrt(6.0 / 128.0)
    z = np.zeros(128)
    theta = np.concatenate([W1.ravel(), z, W2.ravel(), z, w3, np.zeros(1)])
    return theta.astype(np.float32).astype(np.float64)


def workload(name: str, n: int = 8):
    """The named synthetic workloads: returns (tree, source function), or for a
    forest (forest<count>_s<seed>) (list of trees, list of sources).  The
    paper<d>_ex<k> workloads are the uniform depth-d trees of the paper's box-code
    tables with Example k's right-hand side extended by zero (use n = 4 for the
    paper's node count)."""
    if name.startswith("forest"):
        body = name[len("forest"):]
        count, seed = (int(body.split("_s")[0]), int(body.split("_s")[1])) if "_s" in body else (int(body), 0)
        return forest(count, seed, n)
    if name.startswith("gauss20_cap"):                # the 20-Gaussian source, seed 0, another depth cap
        src = random_gaussians(0, 20)
        return gaussian_tree(src, n, 1e-10, int(name[len("gauss20_cap"):])), src
    if name.startswith("uniform") and name.endswith("_gauss"):   # uniform<depth>_gauss
        return uniform_tree(int(name[len("uniform"):-len("_gauss")])), centred_gaussian(0.1)
    if name.startswith("gauss20"):
        seed = int(name.split("_s")[1]) if "_s" in name else 0
        src = random_gaussians(seed, 20)
        return gaussian_tree(src, n, 1e-10, 14), src
    if name.startswith("kink"):
        cap = int(name.split("_cap")[1]) if "_cap" in name else 16
        return adaptive_tree(kink_source, n, 1e-10, cap), kink_source
    if name.startswith("paper"):                     # paper<depth>_ex<1|2>: the paper's uniform-tree rows
        depth, ex = name[len("paper"):].split("_ex")
        return uniform_tree(int(depth)), paper_example_rhs(int(ex))
    raise KeyError(name)
