"""FP64 reference of the parameter-prediction MLP -- TEST INFRASTRUCTURE ONLY.

A plain NumPy restatement of the small multilayer perceptron that predicts the
compression threshold tau and the per-level drop tolerances from matrix features.
Only the test suite and the benchmark's CPU-baseline leg may use it.  It shares no code
with the GPU kernels.

Network: x (in_dim) -> [dense + ReLU] x depth (width `hidden`) -> dense (out_dim).
Parameters are packed layer by layer as W_l (out x in, row-major) followed by b_l (out).
Loss: mean squared error over the batch and the outputs, L = sum (y - t)^2 / (B * out_dim).
Optimizer: Adam with bias correction (Kingma and Ba, 2015).
"""
from __future__ import annotations

import numpy as np


def layer_dims(in_dim: int, hidden: int, depth: int, out_dim: int):
    """[(n_in, n_out)] of every dense layer."""
    dims = [in_dim] + [hidden] * depth + [out_dim]
    return list(zip(dims[:-1], dims[1:]))


def num_params(in_dim, hidden, depth, out_dim) -> int:
    return sum(o * i + o for i, o in layer_dims(in_dim, hidden, depth, out_dim))


def unpack(params: np.ndarray, in_dim, hidden, depth, out_dim):
    """Views (W, b) of every layer inside the packed vector."""
    out, off = [], 0
    for i, o in layer_dims(in_dim, hidden, depth, out_dim):
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    assert off == params.size
    return out


def forward(params, X, in_dim, hidden, depth, out_dim):
    """Returns (output, [pre-activations], [layer inputs])."""
    layers = unpack(np.asarray(params, dtype=np.float64), in_dim, hidden, depth, out_dim)
    a = np.asarray(X, dtype=np.float64)
    zs, ins = [], []
    for li, (W, b) in enumerate(layers):
        ins.append(a)
        z = a @ W.T + b
        zs.append(z)
        a = np.maximum(z, 0.0) if li < len(layers) - 1 else z
    return a, zs, ins


def loss_and_grad(params, X, T, in_dim, hidden, depth, out_dim):
    """MSE loss and its gradient with respect to the packed parameters (backpropagation)."""
    y, zs, ins = forward(params, X, in_dim, hidden, depth, out_dim)
    T = np.asarray(T, dtype=np.float64)
    B = y.shape[0]
    scale = 1.0 / (B * out_dim)
    loss = float(np.sum((y - T) ** 2) * scale)
    layers = unpack(np.asarray(params, dtype=np.float64), in_dim, hidden, depth, out_dim)
    grads = []
    dz = 2.0 * (y - T) * scale            # dL/dz of the output layer (linear)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        gW = dz.T @ ins[li]                # sum over the batch of dz_o * input_i
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            da = dz @ W                    # back through the dense layer
            dz = da * (zs[li - 1] > 0.0)   # ReLU derivative of the layer below
    grads.reverse()
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def matrix_features(n, rowptr, col, val):
    """The eight matrix features, in FP64, from their definitions:
    0 log10 n; 1 mean row length / 100; 2 std / mean of row lengths; 3 mean and 4 smallest
    |a_ii| / sum_j |a_ij| (0 for an empty row); 5 share of entries below 1e-3 of their row's
    largest magnitude; 6 identical-pattern classes per row (every empty row its own class);
    7 mean over rows of (sum_{j != i} |a_ij|) / ((len - 1) |a_ii|) (0 without a diagonal or
    off-diagonal entry)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col)
    a = np.abs(np.asarray(val, dtype=np.float64))
    rl = np.diff(rowptr)
    rows = np.repeat(np.arange(n), rl)
    rowsum = np.bincount(rows, a, n)
    rowmax = np.zeros(n)
    np.maximum.at(rowmax, rows, a)
    diag = np.zeros(n)
    d = col == rows
    diag[rows[d]] = a[d]
    dom = np.where(rowsum > 0, diag / np.where(rowsum > 0, rowsum, 1.0), 0.0)
    tiny = np.count_nonzero(a < 1e-3 * rowmax[rows])
    off = rowsum - diag
    with np.errstate(divide="ignore", invalid="ignore"):
        coup = np.where((diag > 0) & (rl > 1), off / ((rl - 1) * np.where(diag > 0, diag, 1.0)), 0.0)
    patterns = set()
    empty = 0
    for i in range(n):
        if rl[i] == 0:
            empty += 1
        else:
            patterns.add(col[rowptr[i]:rowptr[i + 1]].tobytes())
    mean_len = rl.mean()
    return np.array([np.log10(n), mean_len / 100.0, rl.std() / mean_len if mean_len > 0 else 0.0, dom.mean(),
                     dom.min(), tiny / max(1, len(col)), (len(patterns) + empty) / n, coup.mean()])
