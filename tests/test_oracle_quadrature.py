"""Pins for the oracle's quadrature (Sec. 2.1, Eq. 'ifft'): exactness and geometry."""
import numpy as np
import pytest

from oracle import quadrature as q


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33])
def test_gauss_legendre_exact_to_degree_2n_minus_1(n):
    t, w = q.gauss_legendre(n)
    for deg in range(2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * t ** deg) - exact) < 1e-13
    # degree 2n is NOT integrated exactly: pins the node count (the Gauss error for t^{2n}
    # shrinks like 4^-n, so this is only visible above rounding for small n)
    if n <= 16:
        deg = 2 * n
        exact = 2.0 / (deg + 1)
        assert abs(np.sum(w * t ** deg) - exact) > 1e-11


def test_radial_rule_on_0_P():
    P = 7.3
    r, w = q.radial_rule(P, 12)
    assert np.all((r > 0) & (r < P))
    for deg in range(24):
        assert abs(np.sum(w * r ** deg) - P ** (deg + 1) / (deg + 1)) < 1e-12 * P ** (deg + 1)


def test_ball_2d_measure_and_symmetry():
    P = 5.0
    k, w, kmag = q.ball_nodes(2, P, 16, 32)
    assert k.shape == (16 * 32, 2)
    # int dr dphi = 2 pi P ; with the Jacobian r: area of the disk
    assert abs(w.sum() - 2 * np.pi * P) < 1e-12
    assert abs(np.sum(w * kmag) - np.pi * P * P) < 1e-11
    # k -> -k maps the node set onto itself (even n_phi)
    s = {tuple(np.round(v, 12)) for v in k}
    assert all(tuple(np.round(-v, 12)) in s for v in k)
    assert np.allclose(np.linalg.norm(k, axis=1), kmag)


def test_ball_3d_measure_moments_symmetry():
    P = 3.0
    k, w, kmag = q.ball_nodes(3, P, 8, 16, n_theta=8)
    assert k.shape == (8 * 8 * 16, 3)
    # int dr dmu dphi = 4 pi P ; with r^2: volume of the ball
    assert abs(w.sum() - 4 * np.pi * P) < 1e-12
    assert abs(np.sum(w * kmag ** 2) - 4.0 / 3.0 * np.pi * P ** 3) < 1e-10
    # second angular moments of the unit vector: int k_i^2/r^2 dOmega = 4 pi / 3 for each axis
    for i in range(3):
        assert abs(np.sum(w * (k[:, i] / kmag) ** 2) / P - 4 * np.pi / 3) < 1e-12
    s = {tuple(np.round(v, 12)) for v in k}
    assert all(tuple(np.round(-v, 12)) in s for v in k)
