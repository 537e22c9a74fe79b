"""FP64 reference of the warm-start network's loss and gradient (test infrastructure only).

Not part of the paper: the learned warm start is a project addition.  The network is
x (n_in) -> tanh(W1 x + b1) -> tanh(W2 . + b2) -> W3 . + b3, with inputs standardised by
(x - mean) / stdv, and the loss is the mean squared error over all outputs of the batch.  The
parameter vector is W1 [n_in][H], b1 [H], W2 [H][H], b2 [H], W3 [H][n_out], b3 [n_out], row-major.

parity pin: the gradient agrees with central finite differences of the loss
(tests/test_oracle_warmstart.py).
"""
import numpy as np


def unpack(theta, n_in, H, n_out):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    out = []
    for shape in [(n_in, H), (H,), (H, H), (H,), (H, n_out), (n_out,)]:
        size = int(np.prod(shape))
        out.append(theta[o:o + size].reshape(shape))
        o += size
    assert o == theta.size
    return out


def forward(theta, x, n_in, H, n_out, mean=None, stdv=None):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    x = np.asarray(x, dtype=np.float64)
    mean = np.zeros(n_in) if mean is None else np.asarray(mean, dtype=np.float64)
    stdv = np.ones(n_in) if stdv is None else np.asarray(stdv, dtype=np.float64)
    xs = (x - mean) / stdv
    a1 = np.tanh(xs @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    return xs, a1, a2, a2 @ W3 + b3


def loss_grad(theta, x, t, n_in, H, n_out, mean=None, stdv=None):
    """Mean squared error of the batch and its gradient with respect to theta (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    xs, a1, a2, y = forward(theta, x, n_in, H, n_out, mean, stdv)
    t = np.asarray(t, dtype=np.float64)
    cnt = y.size
    d = y - t
    loss = np.sum(d * d) / cnt
    dy = 2.0 * d / cnt
    gW3 = a2.T @ dy
    gb3 = dy.sum(0)
    d2 = (dy @ W3.T) * (1.0 - a2 * a2)
    gW2 = a1.T @ d2
    gb2 = d2.sum(0)
    d1 = (d2 @ W2.T) * (1.0 - a1 * a1)
    gW1 = xs.T @ d1
    gb1 = d1.sum(0)
    return loss, np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def loss_only(theta, x, t, n_in, H, n_out, mean=None, stdv=None):
    y = forward(theta, x, n_in, H, n_out, mean, stdv)[3]
    d = y - np.asarray(t, dtype=np.float64)
    return np.sum(d * d) / d.size
