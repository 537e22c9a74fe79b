"""Helpers for the GPU parity tests (device transfer, error metric, sampled oracle sums)."""
import numpy as np

from oracle import potential as op

TOL = {0: 1e-10, 1: 1e-6}   # relative max-norm parity, FP64 / FP32 path


def torch_mod():
    import torch
    return torch


def to_dev(a, prec):
    torch = torch_mod()
    dt = torch.float64 if prec == 0 else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host_input(a, prec):
    """The exact values the GPU sees, in FP64 for the oracle."""
    return np.asarray(a, dtype=np.float64 if prec == 0 else np.float32).astype(np.float64)


def rel_err(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def oracle_u_at(points, c, k, n, L, kernel, rho=None, sigma=None):
    """u at selected grid points (index tuples) from node coefficients c over the FULL node set:
    Re sum_m c_m e^{i k_m . x_j}, plus the analytic u1 term for the Laplace kernel."""
    xs, h = op.grid_axes(n, L)
    out = []
    m0 = m1 = None
    if kernel == op.LAPLACE2D:
        m0, m1 = op.moments(rho, n, L)
    for pt in points:
        x = np.array([xs[i][pt[i]] for i in range(len(n))])
        v = float(np.real(np.sum(c * np.exp(1j * (k @ x)))))
        if kernel == op.LAPLACE2D:
            X = np.array([[x[0]]])
            Y = np.array([[x[1]]])
            ax, ay = op.u12(X, Y, sigma)
            v += m0 * float(op.u11(X, Y, sigma)[0, 0]) - (m1[0] * ax[0, 0] + m1[1] * ay[0, 0])
        out.append(v)
    return np.array(out)
