"""Host logic of the learned-refinement tree builder, with stub proposers in
place of the network (no GPU): verification and fallback by the plain tail
criterion, and the 16 x 16 sample grids."""
import numpy as np

from paper_1610_00823_amd import inputs as I
from paper_1610_00823_amd import refine as R


def _funs():
    return [I.random_gaussians(500 + s, K) for s, K in [(2, 1), (3, 1), (2, 3), (5, 4)]]


def _covered(fine, coarse):
    leaves = set(zip(fine.level.tolist(), fine.ix.tolist(), fine.iy.tolist()))
    for l, x, y in zip(coarse.level.tolist(), coarse.ix.tolist(), coarse.iy.tolist()):
        for k in range(1, l + 1):
            if (l - k, x >> k, y >> k) in leaves:
                return False
    return True


def test_never_split_proposer_gives_the_plain_trees():
    # every proposed leaf is the root; the plain criterion refines it, so the
    # result is the plain method's tree exactly, and costs its f evaluations
    # plus the network's 256 samples of the root
    funs = _funs()
    trees, st = R.build_trees(funs, lambda s, l: np.zeros(len(l), bool), cap=8)
    plain, ev = R.plain_trees(funs, cap=8)
    for a, b in zip(trees, plain):
        assert a.n_leaves == b.n_leaves
        ka = sorted(zip(a.level.tolist(), a.ix.tolist(), a.iy.tolist()))
        kb = sorted(zip(b.level.tolist(), b.ix.tolist(), b.iy.tolist()))
        assert ka == kb
    assert st.net_boxes == len(funs) and st.verify_f_evals + st.fallback_f_evals == ev
    assert st.net_f_evals == 256 * len(funs)


def test_every_leaf_passes_the_criterion_and_refines_the_plain_tree():
    # a proposer that over-refines coarse boxes and one that splits boxes with
    # large samples: either way each unbalanced leaf passes the plain tail
    # criterion and the tree is at least as fine as the plain one
    funs = _funs()
    plain, _ = R.plain_trees(funs, cap=8)
    for prop in (lambda s, l: l < 3, lambda s, l: (l < 6) & (np.abs(s).max((1, 2)) > 1e-3)):
        trees, st = R.build_trees(funs, prop, cap=8)
        for f, t, p in zip(funs, trees, plain):
            lv, xs, ys = t.meta["leaves_unbalanced"]
            bad, _ = I.split_decision(f, lv, xs, ys, 8, 1e-10, 8)
            assert not bad.any()
            assert _covered(t, p)
            assert I.is_balanced(t)
        assert st.leaves == sum(t.n_leaves for t in trees)


def test_grid_samples_are_the_16x16_first_kind_points():
    # samples of x + 2y on the grid of box (level 2, 1, 3) of the unit root
    s = R.grid_samples(lambda x, y: x + 2 * y, np.array([2]), np.array([1]), np.array([3]))
    xi = I.cheb1_nodes(16)
    h = 0.25
    x = -0.5 + 1 * h + 0.5 * h * (1 + xi)
    y = -0.5 + 3 * h + 0.5 * h * (1 + xi)
    assert s.shape == (1, 16, 16)
    assert np.allclose(s[0], x[None, :] + 2 * y[:, None], rtol=0, atol=1e-15)
