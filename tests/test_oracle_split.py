"""Pins for the oracle's split evaluation of the 3D Coulomb potential (Eq. '3.9'): each part
against a closed form it must reproduce, the sum against Example 2.1's closed form, and the
independence of the sum from the partition's width."""
import numpy as np
import pytest
from scipy.special import erf

from oracle import closed_forms as cf
from oracle import potential as op
from oracle import split as sp


def _gauss(n, L, sigma):
    xs, _ = op.grid_axes(n, L)
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    R = np.sqrt(X * X + Y * Y + Z * Z)
    return R, np.exp(-R * R / (sigma * sigma))


def _i2_closed(R, sigma, a):
    """I2 = U2 * rho with U2 = erf(sqrt(a) r / 2) / (4 pi r), the Coulomb potential of the unit
    Gaussian of width s = 2 / sqrt(a); for rho = exp(-r^2/sigma^2) = (pi sigma^2)^{3/2} times the
    unit Gaussian of width sigma, the two Gaussians convolve to width S = sqrt(sigma^2 + s^2):
    I2 = sqrt(pi) sigma^3 erf(r/S) / (4 r), sigma^3 / (2 S) at r = 0."""
    S = np.sqrt(sigma * sigma + 4.0 / a)
    out = np.empty_like(R)
    nz = R > 0
    out[nz] = np.sqrt(np.pi) * sigma ** 3 * erf(R[nz] / S) / (4.0 * R[nz])
    out[~nz] = sigma ** 3 / (2.0 * S)
    return out


def test_split_parts_and_sum_closed_forms():
    """rho = exp(-|x|^2/1.5^2) on a 32^3 grid of [-8,8]^3 (Example 2.1's setting): I2 is the
    potential of the Gaussian blurred by the partition's width, I1 the remainder, and the sum is
    Example 2.1's sigma^3 sqrt(pi) erf(r/sigma) / (4 r) with no ball-truncation floor (the plain
    ball quadrature stops at erfc(sigma P / 2) ~ 2.6e-11 here)."""
    n, L, sigma = (32,) * 3, (8.0,) * 3, 1.5
    R, rho = _gauss(n, L, sigma)
    u, parts = sp.split_potential(rho, n, L, return_parts=True)
    ue = cf.coulomb3d_gauss(R, sigma)
    i2 = _i2_closed(R, sigma, parts["a"])
    scale = ue.max()
    assert np.max(np.abs(parts["I2"] - i2)) < 1e-12 * scale
    assert np.max(np.abs(parts["I1"] - (ue - i2))) < 1e-12 * scale
    assert np.max(np.abs(u - ue)) < 1e-12 * scale
    # the partition puts a visible share in each part
    assert 0.1 < parts["I2"].max() / scale < 0.9


def test_split_sum_independent_of_partition_width():
    """Changing a moves weight between I1 and I2 but not their sum (an off-centre density, so
    that the first moments are nonzero)."""
    n, L = (32,) * 3, (8.0,) * 3
    xs, _ = op.grid_axes(n, L)
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    rho = np.exp(-((X - 1.5) ** 2 + (Y + 1.0) ** 2 + 2.0 * Z ** 2) / 2.0)
    a0 = sp.split_params(n, L)["a"]
    u0, p0 = sp.split_potential(rho, n, L, return_parts=True)
    u1, p1 = sp.split_potential(rho, n, L, a=0.8 * a0, return_parts=True)
    assert np.max(np.abs(u0 - u1)) < 1e-11 * np.max(np.abs(u0))
    assert np.max(np.abs(p0["I1"] - p1["I1"])) > 1e-3 * np.max(np.abs(u0))


def test_split_rejects_coarse_grid():
    with pytest.raises(ValueError):
        sp.split_params((16,) * 3, (8.0,) * 3)


def test_split_ball_rule_converged_on_corner_densities():
    """The default ball rule resolves the largest phases across the box: with Gaussians near
    three corners of [-8,8]^3 (separations up to ~19 across the box), I2 by the default rule
    equals I2 by a rule of 80 radial and polar and 160 azimuthal nodes to rounding."""
    n, L = (32,) * 3, (8.0,) * 3
    xs, _ = op.grid_axes(n, L)
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    cs = [(5.5, 5.0, 5.5), (-5.5, -5.5, -5.0), (5.0, -5.5, 5.5)]
    rho = sum(np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)) for c in cs)
    prm = sp.split_params(n, L)
    assert prm["n_r"] < 60
    u2 = sp.i2_ball(rho, n, L, prm["a"], prm["P2"], prm["n_r"], prm["n_theta"], prm["n_phi"])
    ref = sp.i2_ball(rho, n, L, prm["a"], prm["P2"], 80, 80, 160)
    assert np.max(np.abs(u2 - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.slow
def test_split_reaches_example_21_printed_cell():
    """Example 2.1, Table 'tab:exmp1': rho = exp(-|x|^2/sigma^2), sigma = 1.1, on [-8,8]^3 with
    h = 1/4 (64^3), where the paper prints e_h = 2.367e-14 against the closed form.  The oracle's
    split evaluation must reach that level: <= 3e-14 relative max-norm error over the whole grid."""
    n, L, sigma = (64,) * 3, (8.0,) * 3, 1.1
    R, rho = _gauss(n, L, sigma)
    u = sp.split_potential(rho, n, L)
    ue = cf.coulomb3d_gauss(R, sigma)
    assert np.max(np.abs(u - ue)) / np.max(np.abs(ue)) <= 3e-14


@pytest.mark.slow
def test_split_anisotropic_gaussian_example_21():
    """Example 2.1's gamma != 1 branch: rho = exp(-(x^2 + y^2 + gamma^2 z^2)/sigma^2), gamma = 2,
    sigma = 1.1, on [-8,8]^3 with h = 1/4 across and h_z = h / gamma along z (64 x 64 x 128; the
    paper's h_z: with h_z = 1/4 the density's spectrum is still 7e-6 at the grid's Nyquist and the
    grid alone errs by 3e-9).  The oracle's split evaluation (pinned to the isotropic closed form
    above) and the 1D integral of the closed form (coulomb3d_gauss_aniso) are independent
    evaluations; they agree to the isotropic cell's 3e-14 at points on the axes, the diagonals and
    scattered over the central box."""
    n, L, sigma, gamma = (64, 64, 128), (8.0,) * 3, 1.1, 2.0
    xs, _ = op.grid_axes(n, L)
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    rho = np.exp(-(X * X + Y * Y + gamma * gamma * Z * Z) / (sigma * sigma))
    u = sp.split_potential(rho, n, L)
    c, cz = 32, 64                               # the origin's indices
    idx = [(c, c, cz), (c + 4, c, cz), (c, c + 4, cz), (c, c, cz + 8), (c + 6, c + 6, cz + 12),
           (c - 8, c + 3, cz - 10), (0, 0, 0), (c + 12, c, cz - 24)]
    rng = np.random.default_rng(5)
    idx += [(int(rng.integers(16, 48)), int(rng.integers(16, 48)), int(rng.integers(32, 96))) for _ in range(16)]
    got = np.array([u[i] for i in idx])
    want = np.array([float(cf.coulomb3d_gauss_aniso(X[i], Y[i], Z[i], sigma, gamma)) for i in idx])
    assert np.max(np.abs(got - want)) / abs(want[0]) <= 3e-14
