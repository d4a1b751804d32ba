"""Pins of the learned-count oracle: BF16 rounding, the MLP gradient against
finite differences of the forward, Adam against its closed form on a
constant gradient, the features against hand-computed geometry, and the
first-round width rule."""
import math

import numpy as np
import pytest

from oracle import learned as OL
from oracle.tree import Tree


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is half-way between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e-3, 65504.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, -2.5, 197 / 128 * 2.0 ** -9, 65536.0])
    assert np.array_equal(OL.bf16_round(x), want)
    r = OL.bf16_round(np.random.Generator(np.random.PCG64(1)).standard_normal(1000))
    # at most 8 significant bits
    m, _ = np.frexp(r)
    assert np.all(np.abs(m * 256 - np.round(m * 256)) == 0)


def test_mlp_gradient_matches_finite_differences():
    W = OL.init_weights(3)
    g = np.random.Generator(np.random.PCG64(4))
    X = g.standard_normal((7, OL.NFEAT))
    t = g.standard_normal(7)
    y, cache = OL.forward(W, X, round_weights=False)
    loss, grads = OL.backward(cache, y, t)
    h = 1e-6
    for k in OL.PARAMS:
        base = W[k].astype(np.float64)
        for idx in [(0,) * base.ndim, tuple(s - 1 for s in base.shape)]:
            Wp = {q: v.astype(np.float64) for q, v in W.items()}
            Wm = {q: v.astype(np.float64) for q, v in W.items()}
            Wp[k][idx] += h
            Wm[k][idx] -= h
            lp = np.mean((OL.forward(Wp, X, False)[0] - t) ** 2)
            lm = np.mean((OL.forward(Wm, X, False)[0] - t) ** 2)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_mlp_planted_mistake_caught():
    """A dropped ReLU mask in the backward breaks the finite-difference pin."""
    W = OL.init_weights(5)
    X = np.random.Generator(np.random.PCG64(6)).standard_normal((9, OL.NFEAT))
    t = np.zeros(9)
    y, cache = OL.forward(W, X, round_weights=False)
    cache_bad = dict(cache)
    cache_bad["z1"] = np.abs(cache["z1"]) + 1.0     # every unit active
    _, gbad = OL.backward(cache_bad, y, t)
    _, good = OL.backward(cache, y, t)
    assert not np.allclose(gbad["W1"], good["W1"])


def test_adam_closed_form_constant_gradient():
    """With a constant gradient g, bias-corrected Adam moves each weight by
    lr * g / (|g| + eps) per step."""
    W = {k: np.zeros_like(v) for k, v in OL.init_weights(1).items()}
    m = {k: np.zeros_like(v) for k, v in W.items()}
    v = {k: np.zeros_like(v_) for k, v_ in W.items()}
    g = {k: np.full(W[k].shape, 0.25) for k in W}
    for t in range(1, 6):
        W, m, v = OL.adam_step(W, g, m, v, t, lr=0.01)
    for k in W:
        assert np.allclose(W[k], -5 * 0.01 * 0.25 / (0.25 + 1e-8), rtol=1e-5)


def test_pair_features_geometry():
    pts = np.stack(np.meshgrid((np.arange(16) + 0.5) / 16, (np.arange(8) + 0.5) / 16,
                               indexing="xy"), -1).reshape(-1, 2)
    T = Tree(pts, 16, 0.7)
    f = OL.pair_features(T, 1, 0, 1e-4, [], 0)
    assert f[0] == pytest.approx(1 / T.L)
    assert f[1] == pytest.approx(math.log2(64) / 16)
    # root box 15/16 x 7/16; level-1 split along x: the right half is 7/16 x 7/16
    assert f[2] == pytest.approx((7 / 16) / (15 / 16)) and f[3] == pytest.approx((7 / 16) / (15 / 16))
    assert f[5] == pytest.approx(0.0, abs=1e-9)
    assert f[6] == pytest.approx(2 / 3) and f[7] == pytest.approx(-0.4) and f[15] == -1.0
    g = OL.pair_features(T, 2, 1, 1e-4, [4.0, 2.0, 1.0, 0.5, 0.25], 3)
    assert g[8] == pytest.approx(math.log10(0.5) / 16)       # sigma_2 / sigma_1
    assert g[9] == pytest.approx(math.log10(0.125) / 16)     # sigma_4 / sigma_1
    assert g[10] == -1.0 and g[15] == pytest.approx(2 / 10)


def test_first_round_width_rule():
    assert OL.first_round_width(np.log1p([3.0, 40.2, 7.0]), 10, 34) == 51
    assert OL.first_round_width(np.log1p([3.0]), 10, 34) == 34
    assert OL.first_round_width(np.log1p([5000.0]), 10, 34) == 990
    assert OL.first_round_width(np.array([]), 10, 34) == 34


def test_first_round_width_keeps_accuracy():
    """A wider first round (as a prediction would set it) reaches the same
    tolerance with no more rounds; the plain width reproduces plain peeling."""
    from oracle.hessians import KernelHessian, tree_order
    from oracle.ns import build, power_norm
    import seeded_inputs as si
    pts = si.points_grid_cell_centres(24, 20)
    K = KernelHessian(pts, 0.1, 1e-3)
    T = Tree(pts, 32, 0.7)
    A = tree_order(K.apply, T.perm)
    nu, _ = power_norm(A, T.n, 1)
    Dn = A(np.eye(T.n))
    H0, p0 = build(A, T, 1e-6, nu, 24, 10, adaptive=True, seed=5)
    Hs, ps = build(A, T, 1e-6, nu, 24, 10, adaptive=True, seed=5,
                   first_cols={l: 34 for l in range(1, T.L + 1)})
    assert np.array_equal(H0.dense_tree(), Hs.dense_tree())
    H1, p1 = build(A, T, 1e-6, nu, 24, 10, adaptive=True, seed=5,
                   first_cols={l: 100 for l in range(1, T.L + 1)})
    for H in (H0, H1):
        assert np.linalg.norm(H.dense_tree() - Dn, 2) <= 1e-6 * nu
    assert sum(p1.rounds.values()) <= sum(p0.rounds.values())
    assert p1.first_cols[1] == 100 and p0.first_cols[1] == 34
