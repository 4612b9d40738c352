"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU.

Error metric E(psi) = max|psi - psi_oracle| / max|psi_oracle| over the
evaluated nodes (section 6's relative L-infinity error); the FP64 path must
reach 1e-12 for V and for each gradient component.
"""
import numpy as np
import pytest

import oracle
from paper_1610_00823_amd import boxfmm as B
from paper_1610_00823_amd import inputs as I
from tests import closed_forms as CF

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


@pytest.fixture(scope="module")
def ctx8():
    _torch()
    return B.Context(8, 30, B.BX_FP64)


def gpu_eval(ctx, tree, f, nrhs=None):
    torch = _torch()
    tr = B.Tree.from_inputs(ctx, tree)
    fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    V, G = B.volume_eval_grad(ctx, tr, fd)
    torch.cuda.synchronize()
    return V.cpu().numpy(), G.cpu().numpy(), tr


def E(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def check_vs_oracle(tree, f, V, G, leaves=None, tol=TOL):
    n = f.shape[-1]
    Vo, Gxo, Gyo = oracle.volume_at_nodes(tree.level, tree.ix, tree.iy, f, leaves=leaves, cx=tree.cx,
                                          cy=tree.cy, width=tree.width)
    sel = slice(None) if leaves is None else leaves
    ev, ex, ey = E(V[sel], Vo), E(G[sel, 0], Gxo), E(G[sel, 1], Gyo)
    print(f"E(V)={ev:.2e} E(dV/dx1)={ex:.2e} E(dV/dx2)={ey:.2e}")
    assert ev < tol and ex < tol and ey < tol
    return ev, ex, ey


def test_constant_source_closed_form(ctx8):
    # f = 1 is exact on any tree: the whole pipeline against the rectangle formula.
    for t in (I.uniform_tree(3), I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4]], [5, 4])):
        f = np.ones((t.n_leaves, 8, 8))
        V, G, _ = gpu_eval(ctx8, t, f)
        X, Y = oracle.leaf_nodes(t.level, t.ix, t.iy, 8)
        Ve, gxe, gye = CF.const_rect(X, Y, -0.5, 0.5, -0.5, 0.5)
        assert E(V[0], Ve) < TOL and E(G[0, :, 0], gxe) < TOL and E(G[0, :, 1], gye) < TOL


def test_single_leaf_and_two_levels(ctx8):
    rng = np.random.default_rng(11)
    for depth in (0, 1, 2):
        t = I.uniform_tree(depth)
        f = rng.standard_normal((t.n_leaves, 8, 8))
        V, G, _ = gpu_eval(ctx8, t, f)
        check_vs_oracle(t, f, V[0], G[0])


def test_uniform_depth4_gaussian_all_nodes(ctx8):
    # 256 leaves, 8x8 nodes, p = 30, f = exp(-|x|^2 / 0.1^2): every node.
    t, src = I.workload("uniform4_gauss")
    f = I.sample(t, src, 8)
    V, G, _ = gpu_eval(ctx8, t, f)
    check_vs_oracle(t, f, V[0], G[0])
    # and against the closed form within the discretisation bound
    X, Y = oracle.leaf_nodes(t.level, t.ix, t.iy, 8)
    Ve, gxe, gye = CF.radial_gaussian(X, Y, 0.1)
    assert np.abs(V[0] - Ve).max() < 1e-8


def test_graded_tree_random_source_all_nodes(ctx8):
    # Every near (same, coarse, fine), W, X and V configuration occurs here.
    t = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4], [0.45, -0.45], [-0.1, 0.33]], [5, 4, 6, 3])
    rng = np.random.default_rng(5)
    f = rng.standard_normal((t.n_leaves, 8, 8))
    V, G, tr = gpu_eval(ctx8, t, f)
    assert tr.query("w_pairs") > 0 and tr.query("x_pairs") > 0
    check_vs_oracle(t, f, V[0], G[0])


def test_multi_rhs_equals_single(ctx8):
    torch = _torch()
    t = I.point_refined_tree([[0.2, -0.3]], [4])
    rng = np.random.default_rng(9)
    f = rng.standard_normal((3, t.n_leaves, 8, 8))
    tr = B.Tree.from_inputs(ctx8, t)
    V3, G3 = B.volume_eval_grad(ctx8, tr, torch.from_numpy(f).cuda())
    for r in range(3):
        V1, G1 = B.volume_eval_grad(ctx8, tr, torch.from_numpy(f[r].copy()).cuda())
        assert torch.equal(V1[0], V3[r]) and torch.equal(G1[0], G3[r])


def test_eval_and_grad_entry_points_agree(ctx8):
    torch = _torch()
    t = I.uniform_tree(3)
    f = torch.from_numpy(np.random.default_rng(3).standard_normal((t.n_leaves, 8, 8))).cuda()
    tr = B.Tree.from_inputs(ctx8, t)
    V, G = B.volume_eval_grad(ctx8, tr, f)
    assert torch.equal(B.volume_eval(ctx8, tr, f), V)
    assert torch.equal(B.volume_grad(ctx8, tr, f), G)


def test_adaptive_gaussians_sampled_targets(ctx8):
    # 20 Gaussians, tail tolerance 1e-10, depth <= 14: about 42k leaves.  The
    # oracle checks a seeded sample of leaves stratified by level.
    t, src = I.workload("gauss20_s0")
    f = I.sample(t, src, 8)
    V, G, _ = gpu_eval(ctx8, t, f)
    rng = np.random.default_rng(0)
    sel = []
    for l in np.unique(t.level):
        idx = np.flatnonzero(t.level == l)
        sel += list(rng.choice(idx, min(len(idx), 6), replace=False))
    sel = np.array(sorted(sel))
    Vo, Gxo, Gyo = oracle.volume_at_nodes(t.level, t.ix, t.iy, f, leaves=sel)
    # normalise by the maxima over all nodes (the oracle's sample maxima are a lower bound)
    ev = np.abs(V[0][sel] - Vo).max() / np.abs(V[0]).max()
    ex = np.abs(G[0][sel, 0] - Gxo).max() / np.abs(G[0][:, 0]).max()
    ey = np.abs(G[0][sel, 1] - Gyo).max() / np.abs(G[0][:, 1]).max()
    print(f"sampled {len(sel)} leaves: E(V)={ev:.2e} E(dV/dx1)={ex:.2e} E(dV/dx2)={ey:.2e}")
    assert ev < TOL and ex < TOL and ey < TOL


# Other node counts and expansion orders (the K chunking of the leaf GEMM and
# the expansion operators depend on them).  A graded tree with W and X lists,
# random samples, a seeded sample of leaves per level against the oracle.  The
# tolerance is the far-field truncation of order p (measured errors are well
# below it), and at p = 40 the FP64 bar.
ORDERS = [(4, 16, B.BX_FP64, 1e-6), (8, 16, B.BX_FP64, 1e-6), (8, 40, B.BX_FP64, TOL),
          (16, 20, B.BX_FP64, 1e-7), (8, 16, B.BX_SPLIT_INT8, 1e-6), (16, 20, B.BX_SPLIT_INT8, 1e-7)]


@pytest.mark.parametrize("n,p,flags,tol", ORDERS, ids=[f"n{o[0]}_p{o[1]}_{'split' if o[2] else 'fp64'}" for o in ORDERS])
def test_other_orders_sampled(n, p, flags, tol):
    _torch()
    ctx = B.Context(n, p, flags)
    t = I.point_refined_tree([[0.31, 0.22], [-0.4, -0.35]], [5, 3])
    rng = np.random.default_rng(100 + n + p)
    f = rng.standard_normal((t.n_leaves, n, n))
    V, G, _ = gpu_eval(ctx, t, f)
    sel = []
    for l in np.unique(t.level):
        idx = np.flatnonzero(t.level == l)
        sel += list(rng.choice(idx, min(len(idx), 3), replace=False))
    sel = np.array(sorted(sel))
    Vo, Gxo, Gyo = oracle.volume_at_nodes(t.level, t.ix, t.iy, f, leaves=sel)
    ev = np.abs(V[0][sel] - Vo).max() / np.abs(V[0]).max()
    ex = np.abs(G[0][sel, 0] - Gxo).max() / np.abs(G[0][:, 0]).max()
    ey = np.abs(G[0][sel, 1] - Gyo).max() / np.abs(G[0][:, 1]).max()
    print(f"n={n} p={p} flags={flags}: {len(sel)} leaves E(V)={ev:.2e} E(dV/dx1)={ex:.2e} E(dV/dx2)={ey:.2e}")
    assert ev < tol and ex < tol and ey < tol


def test_graph_replays_match_eager(ctx8):
    # The evaluation is captured once into a hipGraph and replayed; each replay,
    # with unrelated eager torch work and synchronisations in between and new
    # data in the same buffers, must equal the eager (one launch per kernel) result.
    torch = _torch()
    t = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4]], [5, 4])
    tr = B.Tree.from_inputs(ctx8, t)
    rng = np.random.default_rng(21)
    f = torch.from_numpy(rng.standard_normal((1, t.n_leaves, 8, 8))).cuda()
    V = torch.empty_like(f)
    G = torch.empty((1, t.n_leaves, 2, 8, 8), dtype=torch.float64, device="cuda")
    for rep in range(4):
        f.copy_(torch.from_numpy(rng.standard_normal((1, t.n_leaves, 8, 8))))
        ctx8.profile(True)                      # eager: one launch per kernel
        Ve, Ge = B.volume_eval_grad(ctx8, tr, f)
        torch.cuda.synchronize()
        ctx8.profile(False)
        ctx8.profile_read()
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
        B.volume_eval_grad(ctx8, tr, f, V, G)   # captured on the first pass, replayed after
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(V, Ve) and torch.equal(G, Ge), f"replay {rep} differs"


# ---------------------------------------------------------------- split BF16
SPLIT_TOL = 1e-10


@pytest.fixture(scope="module")
def ctx8s():
    _torch()
    return B.Context(8, 30, B.BX_SPLIT_INT8)


@pytest.mark.parametrize("case", ["uniform4_gauss", "graded_random"])
def test_split_precision_all_nodes(ctx8s, case):
    # Near tables as exact BF16 slice products (FP32 accumulation, FP64
    # recombination): every result within 1e-10 of the oracle (relative L-inf).
    if case == "uniform4_gauss":
        t, src = I.workload("uniform4_gauss")
        f = I.sample(t, src, 8)
    else:
        t = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4], [0.45, -0.45], [-0.1, 0.33]], [5, 4, 6, 3])
        f = np.random.default_rng(5).standard_normal((t.n_leaves, 8, 8))
    V, G, tr = gpu_eval(ctx8s, t, f)
    assert tr.query("split_products") > 0
    check_vs_oracle(t, f, V[0], G[0], tol=SPLIT_TOL)


def test_split_precision_adaptive_sampled(ctx8s):
    t, src = I.workload("gauss20_s0")
    f = I.sample(t, src, 8)
    V, G, _ = gpu_eval(ctx8s, t, f)
    rng = np.random.default_rng(1)
    sel = []
    for l in np.unique(t.level):
        idx = np.flatnonzero(t.level == l)
        sel += list(rng.choice(idx, min(len(idx), 6), replace=False))
    sel = np.array(sorted(sel))
    Vo, Gxo, Gyo = oracle.volume_at_nodes(t.level, t.ix, t.iy, f, leaves=sel)
    ev = np.abs(V[0][sel] - Vo).max() / np.abs(V[0]).max()
    ex = np.abs(G[0][sel, 0] - Gxo).max() / np.abs(G[0][:, 0]).max()
    ey = np.abs(G[0][sel, 1] - Gyo).max() / np.abs(G[0][:, 1]).max()
    print(f"split, sampled {len(sel)} leaves: E(V)={ev:.2e} E(dV/dx1)={ex:.2e} E(dV/dx2)={ey:.2e}")
    assert ev < SPLIT_TOL and ex < SPLIT_TOL and ey < SPLIT_TOL


def test_split_multi_rhs_equals_single(ctx8s):
    torch = _torch()
    t = I.point_refined_tree([[0.2, -0.3]], [4])
    f = np.random.default_rng(19).standard_normal((2, t.n_leaves, 8, 8))
    tr = B.Tree.from_inputs(ctx8s, t)
    V2, G2 = B.volume_eval_grad(ctx8s, tr, torch.from_numpy(f).cuda())
    for r in range(2):
        V1, G1 = B.volume_eval_grad(ctx8s, tr, torch.from_numpy(f[r].copy()).cuda())
        assert torch.equal(V1[0], V2[r]) and torch.equal(G1[0], G2[r])


# ------------------------------------------------ interpolation at points
def _locate(tree, x, y):
    """Leaf holding (x, y) and its local coordinates in [-1, 1] (host reference)."""
    ux, uy = (x - tree.cx) / tree.width + 0.5, (y - tree.cy) / tree.width + 0.5
    for i in range(tree.n_leaves):
        h = 0.5 ** tree.level[i]
        x0, y0 = tree.ix[i] * h, tree.iy[i] * h
        if x0 <= ux < x0 + h and y0 <= uy < y0 + h:
            return i, 2 * (ux - x0) / h - 1, 2 * (uy - y0) / h - 1
    raise AssertionError("point outside the tree")


def test_interpolate_reproduces_nodes_and_numpy_chebyshev(ctx8):
    # At the collocation nodes the interpolant returns the computed values; at
    # random points it equals numpy's Chebyshev interpolant of the same values.
    torch = _torch()
    t = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4]], [5, 4])
    rng = np.random.default_rng(31)
    f = rng.standard_normal((t.n_leaves, 8, 8))
    V, G, tr = gpu_eval(ctx8, t, f)
    X, Y = oracle.leaf_nodes(t.level, t.ix, t.iy, 8)
    sel = rng.choice(t.n_leaves, 20, replace=False)
    xy = np.stack([X[sel].ravel(), Y[sel].ravel()], 1)
    Vd, Gd = torch.from_numpy(V).cuda(), torch.from_numpy(G).cuda()
    v, g = B.interpolate(ctx8, tr, torch.from_numpy(xy).cuda(), Vd, Gd)
    v, g = v.cpu().numpy()[0], g.cpu().numpy()[0]
    assert np.abs(v - V[0][sel].ravel()).max() < 1e-13 * np.abs(V).max()
    assert np.abs(g[:, 0] - G[0][sel, 0].ravel()).max() < 1e-13 * np.abs(G).max()
    assert np.abs(g[:, 1] - G[0][sel, 1].ravel()).max() < 1e-13 * np.abs(G).max()
    pts = rng.uniform(-0.5, 0.5, size=(300, 2))
    v, g = B.interpolate(ctx8, tr, torch.from_numpy(pts).cuda(), Vd, Gd)
    v, g = v.cpu().numpy()[0], g.cpu().numpy()[0]
    nodes = -np.cos((2 * np.arange(8) + 1) * np.pi / 16)
    C = np.polynomial.chebyshev
    for k, (x, y) in enumerate(pts):
        leaf, lx, ly = _locate(t, x, y)
        for vals, got in ((V[0][leaf], v[k]), (G[0][leaf, 0], g[k, 0]), (G[0][leaf, 1], g[k, 1])):
            cx = C.chebfit(nodes, vals.T, 7)            # fit along x (columns), per y row
            rows = C.chebval(lx, cx)                    # values at lx on each y node
            ref = C.chebval(ly, C.chebfit(nodes, rows, 7))
            assert abs(got - ref) < 1e-12 * max(1.0, np.abs(vals).max()), (k, got, ref)
    out, _ = B.interpolate(ctx8, tr, torch.tensor([[0.7, 0.0], [0.0, -0.51]], dtype=torch.float64).cuda(), Vd)
    assert torch.isnan(out).all()


def test_interpolant_vs_oracle_off_node():
    # v~ at points other than the nodes (section 3.1) against the oracle's V f~
    # there.  The difference is the interpolation error of the smooth potential;
    # its reference is the same interpolation applied to the exact radial
    # Gaussian potential (closed form) at the nodes, compared with the closed
    # form at the points.
    torch = _torch()
    ctx = B.Context(8, 30, B.BX_FP64)
    t, src = I.workload("uniform4_gauss")
    f = I.sample(t, src, 8)
    V, G, tr = gpu_eval(ctx, t, f)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-0.5, 0.5, size=(200, 2))
    pd = torch.from_numpy(pts).cuda()
    v, g = B.interpolate(ctx, tr, pd, torch.from_numpy(V).cuda(), torch.from_numpy(G).cuda())
    Vo, Gxo, Gyo = oracle.volume(t.level, t.ix, t.iy, f, pts[:, 0], pts[:, 1])
    ev = np.abs(v.cpu().numpy()[0] - Vo).max() / np.abs(V).max()
    eg = np.abs(g.cpu().numpy()[0, :, 0] - Gxo).max() / np.abs(G[:, :, 0]).max()
    X, Y = oracle.leaf_nodes(t.level, t.ix, t.iy, 8)
    Ve, gxe, gye = CF.radial_gaussian(X, Y, 0.1)
    Gn = np.stack([gxe, gye], 1)[None]
    vi, gi = B.interpolate(ctx, tr, pd, torch.from_numpy(np.ascontiguousarray(Ve[None])).cuda(),
                           torch.from_numpy(np.ascontiguousarray(Gn)).cuda())
    Vc, gxc, _ = CF.radial_gaussian(pts[:, 0], pts[:, 1], 0.1)
    iv = np.abs(vi.cpu().numpy()[0] - Vc).max() / np.abs(Ve).max()
    ig = np.abs(gi.cpu().numpy()[0, :, 0] - gxc).max() / np.abs(gxe).max()
    print(f"off-node: E(v~)={ev:.2e} E(g~_1)={eg:.2e}; interpolation of the exact potential: {iv:.2e} {ig:.2e}")
    assert ev < 2 * iv + 1e-12 and eg < 2 * ig + 1e-12


# ----------------------------------------------------------------- forests
def _forest_inputs(n, seed):
    trees = [I.point_refined_tree([[0.3, 0.2]], [5]), I.uniform_tree(3),
             I.point_refined_tree([[-0.3, 0.4], [0.1, -0.2]], [4, 6]), I.uniform_tree(1)]
    rng = np.random.default_rng(seed)
    fs = [rng.standard_normal((2, t.n_leaves, n, n)) for t in trees]
    return trees, fs


@pytest.mark.parametrize("flags", [B.BX_FP64, B.BX_SPLIT_INT8], ids=["fp64", "split"])
def test_forest_equals_separate_trees(ctx8, flags):
    # Four trees of uneven depth and two right-hand sides as one forest (one
    # upload, one captured evaluation) against each tree evaluated alone in FP64.
    torch = _torch()
    trees, fs = _forest_inputs(8, 41)
    ctx = ctx8 if flags == B.BX_FP64 else B.Context(8, 30, flags)
    forest = B.Tree.forest(ctx, trees)
    f = np.concatenate(fs, axis=1)
    V, G = B.volume_eval_grad(ctx, forest, torch.from_numpy(f).cuda())
    V, G = V.cpu().numpy(), G.cpu().numpy()
    off = 0
    for t, ft in zip(trees, fs):
        tr = B.Tree.from_inputs(ctx8, t)
        Vs, Gs = B.volume_eval_grad(ctx8, tr, torch.from_numpy(ft).cuda())
        Vs, Gs = Vs.cpu().numpy(), Gs.cpu().numpy()
        sl = slice(off, off + t.n_leaves)
        ev, eg = E(V[:, sl], Vs), E(G[:, sl], Gs)
        tol = 1e-13 if flags == B.BX_FP64 else 1e-10
        print(f"tree with {t.n_leaves} leaves: E(V)={ev:.2e} E(G)={eg:.2e}")
        assert ev < tol and eg < tol
        off += t.n_leaves


# ------------------------------------------------------ schedule tuning
@pytest.mark.parametrize("flags", [B.BX_FP64, B.BX_SPLIT_INT8], ids=["fp64", "split"])
def test_tuning_changes_no_result(ctx8, flags):
    # The scheduling parameters only move work between blocks and launches:
    # every output is summed in the same order, so results are bitwise equal
    # for any setting, including the extremes (every tile split by rows, none
    # split, one M2L block, every level alone or two levels per launch).
    torch = _torch()
    ctx = ctx8 if flags == B.BX_FP64 else B.Context(8, 30, flags)
    t, src = I.workload("gauss20_s0")
    f = torch.from_numpy(I.sample(t, src, 8)).cuda()
    tr = B.Tree.from_inputs(ctx, t)
    assert tr.tuning() == (1.5 if flags == B.BX_SPLIT_INT8 else 1.0, 16.0, 4096, 0)
    V0, G0 = B.volume_eval_grad(ctx, tr, f)
    for heavy, w, blocks, fuse in [(1e-3, 1.0, 1, 0), (1e30, 16.0, 7, 100000), (0.5, 0.25, 4096, 300)]:
        tr.set_tuning(heavy, w, blocks, fuse)
        assert tr.tuning() == (heavy, w, blocks, fuse)
        V, G = B.volume_eval_grad(ctx, tr, f)
        assert torch.equal(V, V0) and torch.equal(G, G0), (heavy, w, blocks, fuse)
    V, G, best = B.autotune(ctx, tr, f, reps=2)
    print("autotune:", best)
    assert torch.equal(V, V0) and torch.equal(G, G0)
    assert tr.tuning() == best[:4] and best[4] > 0
    V, G = B.volume_eval_grad(ctx, tr, f)
    assert torch.equal(V, V0) and torch.equal(G, G0)


# ------------------------------------------- the paper's own right-hand sides
@pytest.mark.parametrize("example", [1, 2])
def test_paper_examples_zero_extension_n4(example):
    # The paper's node count (4 x 4) on a uniform tree, with Example 1 or 2's
    # f = Laplacian(u) inside its multiply connected domain and zero outside
    # (a discontinuous source: the box code integrates the piecewise
    # polynomial f~ whatever f is), against the oracle on sampled leaves.
    torch = _torch()
    t, src = I.workload(f"paper4_ex{example}", 4)
    f = I.sample(t, src, 4)
    ctx = B.Context(4, 30, B.BX_FP64)
    tr = B.Tree.from_inputs(ctx, t)
    V, G = B.volume_eval_grad(ctx, tr, torch.from_numpy(f).cuda())
    V, G = V.cpu().numpy()[0], G.cpu().numpy()[0]
    sel = np.sort(np.random.default_rng(example).choice(t.n_leaves, 24, replace=False))
    Vo, Gxo, Gyo = oracle.volume_at_nodes(t.level, t.ix, t.iy, f, leaves=sel)
    ev = np.abs(V[sel] - Vo).max() / np.abs(V).max()
    ex = np.abs(G[sel, 0] - Gxo).max() / np.abs(G[:, 0]).max()
    ey = np.abs(G[sel, 1] - Gyo).max() / np.abs(G[:, 1]).max()
    print(f"example {example}, n = 4, 24 of {t.n_leaves} leaves: E(V)={ev:.2e} E(dV/dx1)={ex:.2e} E(dV/dx2)={ey:.2e}")
    assert ev < TOL and ex < TOL and ey < TOL


# ------------------------------------------- full-size workloads, sampled
def _sampled_check(t, f, V, G, sel, tol, label):
    Vo, Gxo, Gyo = oracle.volume_at_nodes(t.level, t.ix, t.iy, f, leaves=sel, cx=t.cx, cy=t.cy, width=t.width)
    ev = np.abs(V[sel] - Vo).max() / np.abs(V).max()
    ex = np.abs(G[sel, 0] - Gxo).max() / np.abs(G[:, 0]).max()
    ey = np.abs(G[sel, 1] - Gyo).max() / np.abs(G[:, 1]).max()
    print(f"{label}: {len(sel)} of {t.n_leaves} leaves: E(V)={ev:.2e} E(dV/dx1)={ex:.2e} E(dV/dx2)={ey:.2e}")
    assert ev < tol and ex < tol and ey < tol


@pytest.mark.parametrize("name,n", [("kink_cap16", 8), ("kink_cap12", 16)])
def test_kink_source_full_size_sampled(name, n):
    # Configuration 3 at its full size (the C0 kink source, refinement to the
    # cap along the curve), both precisions in the launch configuration the
    # benchmark times, on leaves the oracle evaluates one by one: the deepest
    # leaf nearest the kink, the coarsest leaf, and two at random.
    torch = _torch()
    t, src = I.workload(name, n)
    f = I.sample(t, src, n)
    deep = np.flatnonzero(t.level == t.level.max())
    rng = np.random.default_rng(3)
    sel = np.unique(np.concatenate([deep[:1], [int(np.argmin(t.level))], rng.choice(t.n_leaves, 2, replace=False)]))
    fd = torch.from_numpy(f).cuda()
    for flags, tol in ((B.BX_FP64, TOL), (B.BX_SPLIT_INT8, SPLIT_TOL)):
        ctx = B.Context(n, 30, flags)
        tr = B.Tree.from_inputs(ctx, t)
        V, G = B.volume_eval_grad(ctx, tr, fd)
        V, G = V.cpu().numpy()[0], G.cpu().numpy()[0]
        _sampled_check(t, f, V, G, sel, tol, f"{name} n={n} {'split' if flags else 'fp64'}")
        del V, G, tr, ctx


def test_forest256_full_size_sampled():
    # Configuration 4's forest at its full size (256 trees, 1-40 Gaussians,
    # depth caps 6-12) as one structure, mixed precision; trees do not
    # interact, so sampled leaves of a few trees are checked against the
    # oracle on their own tree.
    torch = _torch()
    trees, srcs, fs = I.forest(256, 0, 8, workers=8, samples=True)   # host processes (no GPU use)
    ctx = B.Context(8, 30, B.BX_SPLIT_INT8)
    forest = B.Tree.forest(ctx, trees)
    V, G = B.volume_eval_grad(ctx, forest, torch.from_numpy(np.concatenate(fs)).cuda())
    V, G = V.cpu().numpy()[0], G.cpu().numpy()[0]
    off = np.concatenate([[0], np.cumsum([t.n_leaves for t in trees])])
    depth = [int(t.level.max()) for t in trees]
    rng = np.random.default_rng(11)
    for k in sorted({int(np.argmax(depth)), int(np.argmin(depth)), int(rng.integers(len(trees)))}):
        t, sl = trees[k], slice(off[k], off[k + 1])
        sel = np.unique(np.concatenate([np.flatnonzero(t.level == t.level.max())[:1],
                                        rng.choice(t.n_leaves, min(2, t.n_leaves), replace=False)]))
        _sampled_check(t, fs[k], V[sl], G[sl], sel, SPLIT_TOL, f"forest256 tree {k} (depth {depth[k]})")


# ------------------------------------------------------------ edge cases
@pytest.mark.parametrize("flags", [B.BX_FP64, B.BX_SPLIT_INT8], ids=["fp64", "split"])
def test_zero_and_single_leaf_sources(ctx8, flags):
    # f = 0 gives exactly zero (the mixed path's scales come from max|f|); a
    # source on one leaf of a graded tree matches the oracle, which sums that
    # leaf alone: FP64 relative to the largest value, the mixed path within its
    # slice tolerance, which is relative to ||f||_inf W^2 (V) and ||f||_inf W
    # (grad V), W = 1 (one deep leaf makes max|V| far smaller than that).
    torch = _torch()
    ctx = ctx8 if flags == B.BX_FP64 else B.Context(8, 30, flags)
    t = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4]], [5, 3])
    tr = B.Tree.from_inputs(ctx, t)
    V, G = B.volume_eval_grad(ctx, tr, torch.zeros((1, t.n_leaves, 8, 8), dtype=torch.float64, device="cuda"))
    assert torch.count_nonzero(V).item() == 0 and torch.count_nonzero(G).item() == 0
    f = np.zeros((t.n_leaves, 8, 8))
    k = int(np.argmax(t.level))
    f[k] = np.random.default_rng(8).standard_normal((8, 8))
    V, G = B.volume_eval_grad(ctx, tr, torch.from_numpy(f).cuda())
    V, G = V.cpu().numpy()[0], G.cpu().numpy()[0]
    assert np.all(np.isfinite(V)) and np.all(np.isfinite(G))
    sel = np.array([0, k, t.n_leaves - 1])
    if flags == B.BX_FP64:
        check_vs_oracle(t, f, V, G, leaves=sel)
    else:
        Vo, Gxo, Gyo = oracle.volume_at_nodes(t.level, t.ix, t.iy, f, leaves=sel)
        fm = np.abs(f).max()
        ev = np.abs(V[sel] - Vo).max() / fm
        eg = max(np.abs(G[sel, 0] - Gxo).max(), np.abs(G[sel, 1] - Gyo).max()) / fm
        print(f"single-leaf source, mixed: |dV| / ||f|| = {ev:.2e}, |dG| / ||f|| = {eg:.2e}")
        assert ev < SPLIT_TOL and eg < SPLIT_TOL


@pytest.mark.parametrize("flags", [B.BX_FP64, B.BX_SPLIT_INT8], ids=["fp64", "split"])
def test_power_of_two_scaling_is_exact(ctx8, flags):
    # Every operation is linear in f and every scale the mixed path chooses is
    # a power of two taken from max|f|, so 2^k f gives exactly 2^k V and 2^k grad V.
    torch = _torch()
    ctx = ctx8 if flags == B.BX_FP64 else B.Context(8, 30, flags)
    t, src = I.workload("uniform4_gauss")
    f = I.sample(t, src, 8)
    tr = B.Tree.from_inputs(ctx, t)
    V0, G0 = B.volume_eval_grad(ctx, tr, torch.from_numpy(f).cuda())
    for k in (-300, -7, 9, 250):
        V, G = B.volume_eval_grad(ctx, tr, torch.from_numpy(np.ldexp(f, k)).cuda())
        assert torch.equal(V, V0 * 2.0 ** k), k          # 2.0 ** k is exact
        assert torch.equal(G, G0 * 2.0 ** k), k


# ------------------------------------------------ expansions: Gauss law
@pytest.mark.parametrize("flags", [B.BX_FP64, B.BX_SPLIT_INT8], ids=["fp64", "split"])
def test_root_multipole_gauss_law_and_exterior(ctx8, flags):
    # P2M and M2M on the GPU end to end: the root's a_0 is the total source
    # integral of f~ (the oracle's exact per-leaf integrals), and the root
    # multipole reproduces the oracle's potential on circles of radius 2 and
    # 5 about the root centre (truncation (0.71 / R)^31, below 1e-13 there).
    torch = _torch()
    ctx = ctx8 if flags == B.BX_FP64 else B.Context(8, 30, flags)
    t = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4], [0.1, 0.35]], [6, 4, 5])
    f = I.sample(t, I.random_gaussians(12, 6, log_sigma=(0.02, 0.2)), 8)
    tr = B.Tree.from_inputs(ctx, t)
    B.volume_eval_grad(ctx, tr, torch.from_numpy(f).cuda())
    a = tr.expansion("multipole", 0)
    Q = oracle.leaf_mass(t.level, f, t.width).sum()
    print(f"a_0 = {a[0].real:.15e}, integral of f~ = {Q:.15e}")
    assert abs(a[0] - Q) <= 1e-13 * np.abs(f).max() * t.width ** 2
    th = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    for R in (2.0, 5.0):
        zt = t.cx + 1j * t.cy + R * np.exp(1j * th)
        w = zt - (t.cx + 1j * t.cy)
        phi = a[0] * np.log(w) + sum(a[k] * w ** (-k) for k in range(1, len(a)))
        Vo, _, _ = oracle.volume(t.level, t.ix, t.iy, f, zt.real, zt.imag)
        e = np.abs(phi.real / (2 * np.pi) - Vo).max() / np.abs(Vo).max()
        print(f"R = {R}: multipole vs oracle {e:.2e}")
        assert e < 1e-12


# ------------------------------------------- root boxes away from the origin
@pytest.mark.parametrize("flags", [B.BX_FP64, B.BX_SPLIT_INT8], ids=["fp64", "split"])
@pytest.mark.parametrize("cx,cy,width", [(2.5, -1.75, 0.3), (-40.0, 13.0, 7.0)])
def test_translated_and_scaled_root(ctx8, flags, cx, cy, width):
    # The same leaves and samples on a root box of centre (cx, cy) and width w:
    # against the oracle at every node, and against the unit box's result by the
    # change of variables y = c + w y' (G(w r) = G(r) + log(w) / 2 pi):
    # V_w = w^2 (V_1 + log(w) Q_1 / 2 pi), grad V_w = w grad V_1, Q_1 = the
    # integral of f~ over the unit box.
    import dataclasses
    torch = _torch()
    ctx = ctx8 if flags == B.BX_FP64 else B.Context(8, 30, flags)
    tol = TOL if flags == B.BX_FP64 else SPLIT_TOL
    t1 = I.point_refined_tree([[0.3, 0.2], [-0.26, -0.4], [0.45, -0.45]], [5, 4, 3])
    tw = dataclasses.replace(t1, cx=cx, cy=cy, width=width)
    f = np.random.default_rng(int(width * 10)).standard_normal((t1.n_leaves, 8, 8))
    Vw, Gw, _ = gpu_eval(ctx, tw, f)
    V1, G1, _ = gpu_eval(ctx, t1, f)
    check_vs_oracle(tw, f, Vw[0], Gw[0], tol=tol)
    Q1 = oracle.leaf_mass(t1.level, f, 1.0).sum()
    Vlaw = width ** 2 * (V1[0] + np.log(width) * Q1 / (2 * np.pi))
    ev, eg = E(Vw[0], Vlaw), E(Gw[0], width * G1[0])
    print(f"root ({cx}, {cy}) width {width}: change of variables E(V)={ev:.2e} E(G)={eg:.2e}")
    assert ev < tol and eg < tol
