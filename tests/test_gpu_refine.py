"""The refinement network's kernels against the CPU oracle (on the GPU), and
what the trained network gains over the plain tail criterion."""
import numpy as np
import pytest

from oracle import refine_net as O
from paper_1610_00823_amd import boxfmm as B
from paper_1610_00823_amd import inputs as I
from paper_1610_00823_amd import refine as R

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


def _boxes(seed, Bn):
    """Samples of assorted magnitudes (an all-zero box, tiny and huge ones) and levels."""
    rng = np.random.default_rng(seed)
    s = rng.standard_normal((Bn, 16, 16)) * np.exp(rng.uniform(-40, 3, Bn))[:, None, None]
    s[0] = 0.0
    s[1] *= 1e-300
    s[2] = 1e30
    return s, rng.integers(0, 17, Bn).astype(np.int8)


def _params(seed):
    th = I.refine_net_init(seed)
    rng = np.random.default_rng(seed + 1)
    k = 0
    for name, shp in O.SHAPES:                       # nonzero biases: some units on, some off
        size = int(np.prod(shp))
        if name.startswith("b"):
            th[k:k + size] = rng.uniform(-0.3, 0.3, size)
        k += size
    return th.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("Bn", [1, 3, 67, 1000])
def test_features_match_oracle(Bn):
    # BF16 features bit for bit (both sides divide in FP64, round to FP32,
    # then to BF16); the two log10 features may differ by one BF16 step when
    # the two log10 implementations round differently.
    torch = _torch()
    s, lv = _boxes(Bn, max(Bn, 3))
    s, lv = s[:Bn], lv[:Bn]
    x = B.mlp_features(torch.from_numpy(s).cuda(), torch.from_numpy(lv).cuda())
    got = x.float().cpu().numpy().astype(np.float64)
    ref = O.features(s, lv)
    assert np.array_equal(np.delete(got, [257, 258], axis=1), np.delete(ref, [257, 258], axis=1))
    lg = slice(257, 259)
    assert np.all(np.abs(got[:, lg] - ref[:, lg]) <= 2.0 ** -7 * np.maximum(np.abs(ref[:, lg]), 2.0 ** -126))


@pytest.mark.parametrize("Bn", [1, 63, 64, 65, 777])
def test_forward_matches_oracle(Bn):
    # FP32 sums of BF16 products against the oracle's FP64 sums of the same
    # BF16 operands: agreement to ~1e-5 of the logit scale, except where an
    # h1 value rounds to the other BF16 neighbour (a 2^-8 relative step on one
    # of 128 terms), bounded by 1e-3 of the scale.
    torch = _torch()
    s, lv = _boxes(100 + Bn, max(Bn, 3))
    s, lv = s[:Bn], lv[:Bn]
    th = _params(3)
    net = B.RefineNet(th)
    x = B.mlp_features(torch.from_numpy(s).cuda(), torch.from_numpy(lv).cuda())
    z = net.forward(x).cpu().numpy().astype(np.float64)
    xr = x.float().cpu().numpy().astype(np.float64)
    ref = O.forward(th, xr, emulate=True)
    scale = np.abs(ref).max()
    err = np.abs(z - ref).max() / scale
    print(f"B={Bn}: max |dlogit| / max |logit| = {err:.2e} (vs unrounded FP64: "
          f"{np.abs(z - O.forward(th, xr, emulate=False)).max() / scale:.2e})")
    assert err < 1e-3


@pytest.mark.parametrize("Bn", [5, 64, 300, 2048])
def test_gradient_matches_oracle(Bn):
    # Every parameter block of the gradient against the oracle's back-propagation
    # with the same BF16 roundings, relative to the block's largest entry.
    torch = _torch()
    s, lv = _boxes(200 + Bn, max(Bn, 3))
    s, lv = s[:Bn], lv[:Bn]
    y = (np.random.default_rng(Bn).random(Bn) < 0.4).astype(np.float32)
    th = _params(4)
    net = B.RefineNet(th)
    x = B.mlp_features(torch.from_numpy(s).cuda(), torch.from_numpy(lv).cuda())
    net.grad(x, torch.from_numpy(y).cuda())
    g = net.read("grad").astype(np.float64)
    loss = float(net.read("loss")[0])
    xr = x.float().cpu().numpy().astype(np.float64)
    L, gr = O.loss_and_grad(th, xr, y.astype(np.float64), emulate=True)
    assert abs(loss - L) <= 1e-5 * abs(L)
    G, Gr = O.unpack(g), O.unpack(gr)
    for name, _ in O.SHAPES:
        e = np.abs(G[name] - Gr[name]).max() / max(np.abs(Gr[name]).max(), 1e-30)
        print(f"B={Bn} {name}: {e:.2e}")
        assert e < 3e-3, name


def test_adam_matches_oracle():
    # Two Adam steps on two batches: the kernel's FP32 update against the
    # oracle's FP64 update from the same gradients (read back after each grad)
    # and the same hyper-parameters, which the kernel takes as FP32 values
    # (0.999 as FP32 moves 1 - beta2 by 1.3e-5 relative).
    torch = _torch()
    lr, b1, b2, eps = (float(np.float32(v_)) for v_ in (1e-3, 0.9, 0.999, 1e-8))
    th = _params(5)
    net = B.RefineNet(th)
    m = v = mb = np.zeros(O.N_PARAMS)
    w = th.copy()
    for t, seed in ((1, 11), (2, 12)):
        s, lv = _boxes(seed, 200)
        y = (np.random.default_rng(seed).random(200) < 0.5).astype(np.float32)
        x = B.mlp_features(torch.from_numpy(s).cuda(), torch.from_numpy(lv).cuda())
        net.grad(x, torch.from_numpy(y).cuda())
        g = net.read("grad").astype(np.float64)
        net.adam(lr, b1, b2, eps)
        w, m, v = O.adam_step(w, g, m, v, t, lr, b1, b2, eps)
        got = net.read("params").astype(np.float64)
        # a step is at most lr: the FP32 update (some ten roundings) lies
        # within 8 single-precision ulps of |w| + lr
        assert np.all(np.abs(got - w) <= 8 * 2.0 ** -24 * (np.abs(w) + lr)), t
        # m can cancel (beta1 m and (1 - beta1) g of opposite signs): its error
        # is bounded by ulps of the terms' magnitudes, mb; v has no cancellation
        mb = b1 * mb + (1 - b1) * np.abs(g)
        # (2^-126, the smallest normal single, covers squares that underflow)
        assert np.all(np.abs(net.read("adam_m") - m) <= 4 * 2.0 ** -24 * mb + 2.0 ** -126), t
        assert np.all(np.abs(net.read("adam_v") - v) <= 8 * 2.0 ** -24 * v + 2.0 ** -126), t


CAP = 9


@pytest.fixture(scope="module")
def trained():
    """A network trained on the plain criterion's decisions (with the seed rule)
    over every box it visits for 48 seeded sums of 1 to 40 Gaussians, 12 of
    20 Gaussians and the kink source, depth cap 9 (about 1.1e6 boxes)."""
    _torch()
    jobs = (R.source_jobs(range(300, 348), kinds=("gaussK",), cap=CAP)
            + R.source_jobs(range(400, 412), kinds=("gauss20",), cap=CAP)
            + R.source_jobs([0], kinds=("kink",), cap=CAP))
    s, lv, y = R.labelled_boxes(jobs, workers=8)
    ref = R.LearnedRefiner(seed=0)
    x = ref.features(s, lv)
    del s
    torch = _torch()
    loss0 = ref.loss(x, torch.from_numpy(y).cuda())            # the untrained network
    losses = ref.train(x, y, epochs=8, batch=1024, lr=2e-3, seed=0, log=print)
    return ref, [loss0] + losses, x, y, lv


def test_training_reduces_the_loss(trained):
    ref, losses, x, y, lv = trained
    # (the sums of the gradient use FP32 atomics, so the losses vary a little
    # from run to run)
    print("loss before training and per epoch:", [round(l_, 4) for l_ in losses])
    assert min(losses[1:]) < 0.5 * losses[0]
    pred = ref.predict(x)
    live = lv < CAP                                  # cap-level boxes are never split
    acc = (pred[live] == (y[live] > 0.5)).mean()
    base = max(y[live].mean(), 1 - y[live].mean())
    print(f"training accuracy below the cap: {acc:.4f} (majority class {base:.4f})")
    assert acc > base + 0.1


def _covered(fine, coarse):
    """Every leaf of `coarse` is a leaf of `fine` or is split in it."""
    leaves = set(zip(fine.level.tolist(), fine.ix.tolist(), fine.iy.tolist()))
    for l, x, y in zip(coarse.level.tolist(), coarse.ix.tolist(), coarse.iy.tolist()):
        for k in range(1, l + 1):
            if (l - k, x >> k, y >> k) in leaves:
                return False
    return True


def test_learned_tree_resolves_what_the_tail_criterion_misses(trained):
    # 32 fresh sources of 1 to 8 Gaussians, some narrower than the coarse node
    # spacing.  Without the seed rule (which needs the source's centres) the
    # plain criterion can stop before it ever sees a bump; the network reads
    # finer samples and learned where the seeded criterion refines.
    # * every leaf of the learned tree passes the plain tail criterion, and the
    #   learned tree refines the plain one (a proposed leaf the plain method
    #   would split fails the check and is refined by the plain method);
    # * the gain: the resolution error max |f - f~| / max |f| (over every leaf
    #   and at the bump centres) where the plain criterion missed a bump;
    # * the cost: f evaluations (16 x 16 per box the network decides) and leaves.
    ref = trained[0]
    funs = [I.random_gaussians(10000 + i, int(np.random.default_rng([10000 + i, 7]).integers(1, 9)))
            for i in range(32)]
    trees, st = ref.build(funs, cap=CAP)
    plain, plain_ev = R.plain_trees(funs, cap=CAP)
    e_l, e_p = [], []
    for f, t, p in zip(funs, trees, plain):
        lv, xs, ys = t.meta["leaves_unbalanced"]
        bad, _ = I.split_decision(f, lv, xs, ys, 8, 1e-10, CAP)
        assert not bad.any()
        assert _covered(t, p)
        e_l.append(R.resolution_error(t, f, points=f.c))
        e_p.append(R.resolution_error(p, f, points=f.c))
    missed = [i for i in range(len(funs)) if e_p[i] > 1e-3]
    fixed = [i for i in missed if e_l[i] < 1e-3]
    print("resolution error, learned:", " ".join(f"{e:.0e}" for e in e_l))
    print("resolution error, plain:  ", " ".join(f"{e:.0e}" for e in e_p))
    print(f"plain criterion missed a bump in {len(missed)} of {len(funs)} sources; the learned tree resolved "
          f"{len(fixed)} of them")
    print(f"leaves learned {st.leaves} plain {sum(p.n_leaves for p in plain)}; f evaluations learned {st.f_evals} "
          f"plain {plain_ev}; proposed leaves refined by the fallback {st.failed_leaves}/{st.proposed_leaves}")
    assert all(el <= 2 * ep + 1e-12 for el, ep in zip(e_l, e_p))   # never coarser (check points differ)
    assert len(missed) >= 5 and len(fixed) >= len(missed) // 3
