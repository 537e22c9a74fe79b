"""Pin of the warm-start network oracle: backpropagation equals central finite differences."""
import numpy as np

from oracle import warmstart as ws


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_in, H, n_out, B = 4, 7, 5, 6
    npar = n_in * H + H + H * H + H + H * n_out + n_out
    theta = rng.normal(scale=0.5, size=npar)
    x = rng.normal(size=(B, n_in))
    t = rng.normal(size=(B, n_out))
    mean, stdv = rng.normal(size=n_in), rng.uniform(0.5, 2.0, size=n_in)
    loss, g = ws.loss_grad(theta, x, t, n_in, H, n_out, mean, stdv)
    assert abs(loss - ws.loss_only(theta, x, t, n_in, H, n_out, mean, stdv)) < 1e-14
    eps = 1e-6
    fd = np.empty(npar)
    for i in range(npar):
        e = np.zeros(npar)
        e[i] = eps
        fd[i] = (ws.loss_only(theta + e, x, t, n_in, H, n_out, mean, stdv)
                 - ws.loss_only(theta - e, x, t, n_in, H, n_out, mean, stdv)) / (2 * eps)
    assert np.max(np.abs(fd - g)) < 1e-8 * max(1.0, np.max(np.abs(g)))
