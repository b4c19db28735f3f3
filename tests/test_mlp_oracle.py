"""Pins of the FP64 MLP reference (no GPU): finite differences, closed forms, Adam."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

DIMS = (3, 4, 2, 2)  # in, hidden, depth, out (tiny, so every parameter is checked)


def _rand(seed, dims=DIMS, batch=5):
    rng = np.random.default_rng(seed)
    n = M.num_params(*dims)
    return rng.standard_normal(n) * 0.7, rng.standard_normal((batch, dims[0])), rng.standard_normal((batch, dims[3]))


def test_num_params_and_packing():
    assert M.num_params(16, 128, 3, 5) == (16 * 128 + 128) + 2 * (128 * 128 + 128) + (128 * 5 + 5)
    p = np.arange(M.num_params(*DIMS), dtype=float)
    layers = M.unpack(p, *DIMS)
    assert [W.shape for W, _ in layers] == [(4, 3), (4, 4), (2, 4)]
    # first weight of every layer follows the previous layer's bias
    assert layers[1][0][0, 0] == layers[0][1][-1] + 1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    p, X, T = _rand(seed)
    loss, g = M.loss_and_grad(p, X, T, *DIMS)
    h = 1e-6
    num = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        num[k] = (M.loss_and_grad(p + e, X, T, *DIMS)[0] - M.loss_and_grad(p - e, X, T, *DIMS)[0]) / (2 * h)
    assert np.abs(num - g).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_only_output_bias_gives_constant_output():
    # all weights zero: every hidden unit is ReLU(bias); with zero hidden biases the output is
    # exactly the output bias, and the loss gradient of that bias is 2 mean_b (bias - t_b) / out
    p = np.zeros(M.num_params(*DIMS))
    layers = M.unpack(p, *DIMS)
    layers[-1][1][:] = [0.5, -1.5]
    X = np.random.default_rng(3).standard_normal((6, 3))
    T = np.random.default_rng(4).standard_normal((6, 2))
    y, _, _ = M.forward(p, X, *DIMS)
    assert np.array_equal(y, np.tile([0.5, -1.5], (6, 1)))
    loss, g = M.loss_and_grad(p, X, T, *DIMS)
    gb = M.unpack(g, *DIMS)[-1][1]
    assert np.allclose(gb, 2.0 * (np.array([0.5, -1.5]) - T).sum(axis=0) / (6 * 2))
    assert np.isclose(loss, ((np.array([0.5, -1.5]) - T) ** 2).mean())


def test_linear_net_gradient_is_least_squares_gradient():
    # depth 0: a single dense layer, y = X W^T + b, whose MSE gradient has a closed form
    dims = (3, 4, 0, 2)
    rng = np.random.default_rng(5)
    p = rng.standard_normal(M.num_params(*dims))
    X = rng.standard_normal((7, 3))
    T = rng.standard_normal((7, 2))
    (W, b), = M.unpack(p, *dims)
    R = X @ W.T + b - T
    loss, g = M.loss_and_grad(p, X, T, *dims)
    gW, gb = M.unpack(g, *dims)[0]
    assert np.allclose(gW, 2 * R.T @ X / 14) and np.allclose(gb, 2 * R.sum(0) / 14)
    assert np.isclose(loss, (R ** 2).sum() / 14)


def test_relu_blocks_gradient_of_inactive_units():
    # a hidden unit with a large negative bias never activates: its incoming weights get
    # no gradient
    p, X, T = _rand(7)
    layers = M.unpack(p, *DIMS)
    layers[0][1][2] = -1e3
    _, g = M.loss_and_grad(p, X, T, *DIMS)
    gW0, gb0 = M.unpack(g, *DIMS)[0]
    assert np.all(gW0[2] == 0.0) and gb0[2] == 0.0


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p0 = np.ones(4)
    p1, m, v = M.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias-corrected first moments equal g and second moments g^2, so the step is
    # lr * g / (|g| + eps)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_reduces_a_quadratic():
    # Adam on f(p) = |p - c|^2 approaches c
    c = np.array([1.0, -2.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for k in range(1, 2001):
        p, m, v = M.adam_step(p, 2 * (p - c), m, v, k, lr=0.01)
    assert np.abs(p - c).max() < 1e-3


def test_features_of_a_perfectly_blocked_grid():
    # a 7-point grid with 3 unknowns per node: every row of a node has the same pattern
    # (one class per node), interior rows hold 7 blocks of 3 entries
    from paper_1508_02219_amd import synth
    s = synth.grid_system(4, 4, 4, ell=3, stencil="7pt", seed=1)
    f = M.matrix_features(s.n, s.rowptr, s.col, s.val)
    assert np.isclose(f[0], np.log10(192))
    assert np.isclose(f[6], 1.0 / 3.0)
    interior = [3 * (x + 4 * (y + 4 * z)) for x in (1, 2) for y in (1, 2) for z in (1, 2)]
    assert all(s.rowptr[r + 1] - s.rowptr[r] == 21 for r in interior)
    assert 0.0 < f[4] <= f[3] < 1.0
    # perturbation scales entries by 1e-6 (and removes some): more tiny entries, and rows
    # of one node no longer share one pattern
    q = synth.grid_system(4, 4, 4, ell=3, stencil="7pt", perturb=0.2, seed=1)
    g = M.matrix_features(q.n, q.rowptr, q.col, q.val)
    assert g[5] > f[5] + 0.02 and g[6] > f[6]


def test_features_small_matrix_by_hand():
    # rows: [10, 0.005, 1], [_, 4, 0.003], [1, 1, 1] (columns 0..2)
    rowptr = np.array([0, 3, 5, 8])
    col = np.array([0, 1, 2, 1, 2, 0, 1, 2], dtype=np.int32)
    val = np.array([10.0, 0.005, 1.0, 4.0, 0.003, 1.0, 1.0, -1.0])
    f = M.matrix_features(3, rowptr, col, val)
    dom = [10 / 11.005, 4 / 4.003, 1 / 3]
    coup = [1.005 / (2 * 10), 0.003 / (1 * 4), 2 / 2]
    lens = np.array([3, 2, 3])
    assert np.allclose(f, [np.log10(3), lens.mean() / 100, lens.std() / lens.mean(), np.mean(dom), min(dom),
                           2 / 8, 2 / 3, np.mean(coup)])


def test_features_diagonal_matrix():
    n = 10
    rowptr = np.arange(n + 1)
    col = np.arange(n, dtype=np.int32)
    val = np.linspace(1.0, 2.0, n)
    f = M.matrix_features(n, rowptr, col, val)
    assert np.allclose(f, [1.0, 0.01, 0.0, 1.0, 1.0, 0.0, 1.0, 0.0])
