"""Pins of the synthetic input recipes against facts they do not compute
themselves: the leaf sets tile the root box and are level-restricted (checked
cell by cell on the finest grid), the paper's domain has the area its polar
curves fix in closed form, and the paper's right-hand sides are the Laplacians
of the exact solutions (checked by finite differences)."""
import numpy as np
import pytest

from paper_1610_00823_amd import inputs as I


def _finest_grid(t):
    """Level of the leaf covering each cell of the finest level, and the number
    of leaves covering it (every cell must be covered exactly once)."""
    D = int(t.level.max())
    m = 1 << D
    lev = np.full((m, m), -1, np.int64)
    cover = np.zeros((m, m), np.int64)
    for l, x, y in zip(t.level.tolist(), t.ix.tolist(), t.iy.tolist()):
        s = 1 << (D - l)
        lev[y * s:(y + 1) * s, x * s:(x + 1) * s] = l
        cover[y * s:(y + 1) * s, x * s:(x + 1) * s] += 1
    return lev, cover


def _max_neighbour_jump(lev):
    """Largest level difference between the leaves of two cells that share an
    edge or a corner."""
    jump = 0
    for dy, dx in ((0, 1), (1, 0), (1, 1), (1, -1)):
        a = lev[max(0, -dy):lev.shape[0] - max(0, dy), max(0, -dx):lev.shape[1] - max(0, dx)]
        b = lev[max(0, dy):, max(0, dx):][:a.shape[0], :a.shape[1]]
        jump = max(jump, int(np.abs(a - b).max()))
    return jump


@pytest.mark.parametrize("case", ["graded", "gauss", "kink"])
def test_trees_tile_the_box_and_are_level_restricted(case):
    if case == "graded":
        t = I.point_refined_tree([(0.31, -0.22), (-0.4, 0.45), (0.0, 0.0)], [8, 6, 7])
    elif case == "gauss":
        t = I.adaptive_tree(I.random_gaussians(5, 6), 8, 1e-8, max_level=8)
    else:
        t = I.adaptive_tree(I.kink_source, 8, 1e-6, max_level=7)
    lev, cover = _finest_grid(t)
    assert np.all(cover == 1)                                   # a partition of the root box
    assert np.isclose(np.sum(np.ldexp(1.0, -2 * t.level.astype(np.int64))), 1.0, rtol=0, atol=1e-15)
    assert _max_neighbour_jump(lev) <= 1
    assert I.is_balanced(t)


def test_balance_only_splits():
    # An unbalanced leaf set (three level-1 leaves beside a quarter cut
    # straight to level 4): the balanced set refines it (each input leaf is a
    # union of output leaves), tiles the box, and balancing it again changes
    # nothing.
    lv, xs, ys = [1, 1, 1], [1, 0, 1], [0, 1, 1]
    for y in range(8):
        for x in range(8):
            lv.append(4)
            xs.append(x)
            ys.append(y)
    t0 = I.Tree(np.array(lv, np.int8), np.array(xs, np.int32), np.array(ys, np.int32))
    assert _max_neighbour_jump(_finest_grid(t0)[0]) > 1
    bl, bx, by = I.balance(t0.level, t0.ix, t0.iy)
    t1 = I.Tree(np.asarray(bl, np.int8), np.asarray(bx, np.int32), np.asarray(by, np.int32))
    lev0, _ = _finest_grid(t0)
    lev1, cover = _finest_grid(t1)
    assert np.all(cover == 1) and _max_neighbour_jump(lev1) <= 1
    assert np.all(lev1 >= lev0)                                 # nothing coarsened
    again = I.balance(t1.level, t1.ix, t1.iy)
    assert sorted(zip(*again)) == sorted(zip(bl, bx, by))


def test_paper_domain_area_matches_the_polar_curves():
    # The area inside r(theta) = c0 + sum (c_j cos j theta + d_j sin j theta)
    # is pi c0^2 + (pi / 2) sum (c_j^2 + d_j^2); the domain is the outer
    # curve's region minus the inner one's.  Midpoint counting on a 2000^2 grid
    # errs only in boundary cells, whose errors largely cancel (measured
    # 2.6e-6); the smallest coefficient, 0.005, moves the area by
    # (pi / 2) 0.005^2 = 3.9e-5, so a dropped or mistyped term fails.
    outer = np.pi * 0.25 ** 2 + np.pi / 2 * (0.02 ** 2 + 3 * 0.01 ** 2 + 0.01 ** 2)
    inner = np.pi * 0.05 ** 2 + np.pi / 2 * (4 * 0.005 ** 2)
    m = 2000
    c = (np.arange(m) + 0.5) / m - 0.5
    X, Y = np.meshgrid(c, c)
    area = I.paper_domain(X, Y).sum() / m ** 2
    assert abs(area - (outer - inner)) < 2e-5
    assert not I.paper_domain(0.0, 0.0) and not I.paper_domain(0.45, 0.45)   # the hole and the exterior
    assert I.paper_domain(0.15, 0.0) and I.paper_domain(0.0, -0.15)


@pytest.mark.parametrize("example", [1, 2])
def test_paper_rhs_is_the_laplacian_of_the_exact_solution(example):
    # The exact solutions of Examples 1 and 2, written here independently of
    # the recipe; the 4th-order five-point Laplacian of u with step 1e-3 agrees
    # with f inside the domain, and f is zero outside it.
    def u(x, y):
        v = np.sin(10 * (x + y)) + x * x - 3 * y + 8
        return v + (np.exp(-500 * x * x) if example == 2 else 0.0)

    rng = np.random.default_rng(example)
    x, y = rng.uniform(-0.5, 0.5, (2, 4000))
    h = 1e-3
    lap = 0.0
    for ex, ey in ((1, 0), (0, 1)):
        lap = lap + (-u(x + 2 * h * ex, y + 2 * h * ey) + 16 * u(x + h * ex, y + h * ey) - 30 * u(x, y)
                     + 16 * u(x - h * ex, y - h * ey) - u(x - 2 * h * ex, y - 2 * h * ey)) / (12 * h * h)
    f = I.paper_example_rhs(example)(x, y)
    inside = I.paper_domain(x, y)
    assert inside.sum() > 500 and (~inside).sum() > 500
    scale = np.abs(lap[inside]).max()
    assert np.abs(f[inside] - lap[inside]).max() <= 1e-5 * scale
    assert np.all(f[~inside] == 0.0)
