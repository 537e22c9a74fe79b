"""Pins for the oracle's potential: closed forms, Fourier-transform values, operator
identities.  Each test names what fixes the expected value."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import potential as op
from paper_1410_3584_amd import inputs
from conftest import load_table


def _grid(n, L):
    xs, h = op.grid_axes(n, L)
    return np.meshgrid(*xs, indexing="ij"), h


@pytest.mark.parametrize("dim", [2, 3])
def test_type2_equals_fourier_transform_of_shifted_gaussian(dim):
    """rho = exp(-|x-c|^2/s^2) has rhohat(k) = (pi s^2)^{d/2} e^{-s^2|k|^2/4} e^{-i k.c};
    the trapezoid sum on a fine grid reproduces it to rounding (fixes sign, scale, index)."""
    n = (64,) * dim if dim == 2 else (40,) * 3
    L = (9.0,) * dim
    c = np.array([0.7, -1.1, 0.4][:dim])
    s = 1.3 if dim == 2 else 1.6
    X, h = _grid(n, L)
    rho = np.exp(-sum((x - ci) ** 2 for x, ci in zip(X, c)) / s ** 2)
    rng = np.random.default_rng(3)
    k = rng.uniform(-2.0, 2.0, size=(40, dim))
    got = op.type2_direct(rho, n, L, k)
    want = (np.pi * s * s) ** (dim / 2) * np.exp(-s * s * np.sum(k * k, 1) / 4) * np.exp(-1j * k @ c)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("dim", [2, 3])
def test_type1_is_adjoint_of_type2(dim):
    """h^d <v, type1(c)> = Re sum_m c_m conj(type2(v)_m) for any real v, complex c."""
    n = (12, 10) if dim == 2 else (6, 8, 10)
    L = (3.0, 2.5) if dim == 2 else (2.0, 3.0, 4.0)
    rng = np.random.default_rng(7)
    k = rng.uniform(-3, 3, size=(37, dim))
    c = rng.normal(size=37) + 1j * rng.normal(size=37)
    v = rng.normal(size=n)
    _, h = op.grid_axes(n, L)
    lhs = np.prod(h) * np.sum(v * op.type1_direct(c, n, L, k))
    rhs = np.real(np.sum(c * np.conj(op.type2_direct(v, n, L, k))))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_coulomb2d_closed_form_example_2_2():
    """Example 2.2, gamma = 1, sigma^2 = 1.2, L = 8, h = 1/4: the paper prints e_h = 3.202e-15."""
    rows = load_table("potential_errors.txt")
    s2, Lb, hh, e_paper = rows[0][2], rows[0][3], rows[0][4], rows[0][5]
    n = (int(2 * Lb / hh),) * 2
    L = (Lb, Lb)
    (X, Y), _ = _grid(n, L)
    u = op.potential(np.exp(-(X * X + Y * Y) / s2), n, L, op.COULOMB2D)
    ue = cf.coulomb2d_gauss(np.sqrt(X * X + Y * Y), np.sqrt(s2))
    e = np.max(np.abs(u - ue)) / np.max(np.abs(ue))
    assert e < 10 * e_paper


def test_laplace2d_closed_form_example_2_3():
    """Example 2.3, sigma^2 = 1.3, L = 8, h = 1/4: the paper prints e_h = 4.936e-14."""
    rows = load_table("potential_errors.txt")
    s2, Lb, hh, e_paper = rows[1][2], rows[1][3], rows[1][4], rows[1][5]
    n = (int(2 * Lb / hh),) * 2
    L = (Lb, Lb)
    (X, Y), _ = _grid(n, L)
    u, parts = op.potential(np.exp(-(X * X + Y * Y) / s2), n, L, op.LAPLACE2D, return_parts=True)
    ue = cf.laplace2d_gauss(np.sqrt(X * X + Y * Y), np.sqrt(s2))
    e = np.max(np.abs(u - ue)) / np.max(np.abs(ue))
    assert e < 2 * e_paper
    assert np.max(np.abs(parts["imag"])) < 1e-14 * np.max(np.abs(u))


def test_coulomb2d_anisotropic_closed_form():
    """Example 2.2, gamma = 2, sigma = 2 (its gamma != 1 integral), L = 12, h = 1/4."""
    n, L = (96, 96), (12.0, 12.0)
    (X, Y), _ = _grid(n, L)
    u = op.potential(np.exp(-(X * X + 4 * Y * Y) / 4.0), n, L, op.COULOMB2D)
    idx = [(48, 48), (60, 50), (10, 80), (0, 0), (70, 20)]
    ue = np.array([cf.coulomb2d_gauss_aniso(X[i], Y[i], 2.0, 2.0) for i in idx])
    got = np.array([u[i] for i in idx])
    assert np.max(np.abs(got - ue)) < 1e-11 * np.max(np.abs(u))


def test_laplace2d_bumps_superposition():
    """The 2D workload's density (anisotropic Gaussian + seeded off-centre bumps) on a 128^2
    grid of [-16,16]^2 (the narrow y-width 1/2 limits the accuracy to ~1e-9): the potential equals the superposed closed forms.  Off-centre mass makes m1 != 0,
    so a dropped or mis-signed first-moment term of the subtraction fails here."""
    n, L = (128, 128), (16.0, 16.0)
    rho, bumps = inputs.density_2d_bumps(n, L, seed=5, n_bumps=3)
    (X, Y), _ = _grid(n, L)
    u = op.potential(rho, n, L, op.LAPLACE2D)
    idx = [(64, 64), (80, 60), (40, 100), (10, 120), (126, 0)]
    want = []
    for i in idx:
        v = float(cf.laplace2d_gauss_aniso(X[i], Y[i], 1.0, 0.5))
        for a, c, w in bumps:
            v += a * float(cf.laplace2d_gauss(np.hypot(X[i] - c[0], Y[i] - c[1]), w))
        want.append(v)
    got = np.array([u[i] for i in idx])
    assert np.max(np.abs(got - np.array(want))) < 2e-8 * np.max(np.abs(u))


def test_coulomb3d_closed_form_resolved():
    """Example 2.1, gamma = 1, sigma = 1.5 on [-8,8]^3, h = 1/2, P = 2 pi; with enough radial and
    angular nodes the error is set by the ball truncation alone: for a Gaussian the dropped
    part of the Fourier integral at the origin is exactly erfc(sigma P / 2) ~ 2.6e-11 of u(0)."""
    from scipy.special import erfc
    n, L = (32,) * 3, (8.0,) * 3
    (X, Y, Z), _ = _grid(n, L)
    R = np.sqrt(X * X + Y * Y + Z * Z)
    u = op.potential(np.exp(-R * R / 2.25), n, L, op.COULOMB3D, n_r=48, n_theta=64, n_phi=128)
    ue = cf.coulomb3d_gauss(R, 1.5)
    assert np.max(np.abs(u - ue)) / np.max(ue) < 5e-11
    e0 = abs(u[16, 16, 16] - ue[16, 16, 16]) / ue[16, 16, 16]
    assert abs(e0 / erfc(1.5 * np.pi) - 1.0) < 0.1


def test_coulomb3d_workload_floor():
    """The 3D check workload (rho = e^{-|x|^2}, 32^3 on [-8,8]^3, 32x32x64 nodes): at the
    origin the only error left is the ball truncation, which for a unit Gaussian is close to
    erfc(P/2) = erfc(pi) ~ 8.9e-6 (the trapezoid transform of the grid data shifts it by a
    few percent); over the grid the angular rule adds at most a few 1e-5 at the corners."""
    from scipy.special import erfc
    n, L, rho = inputs.coulomb3d_gauss_32()
    (X, Y, Z), _ = _grid(n, L)
    R = np.sqrt(X * X + Y * Y + Z * Z)
    u = op.potential(rho, n, L, op.COULOMB3D, n_r=32, n_theta=32, n_phi=64)
    ue = cf.coulomb3d_gauss(R, 1.0)
    e0 = abs(u[16, 16, 16] - ue[16, 16, 16]) / ue[16, 16, 16]
    assert 0.8 * erfc(np.pi) < e0 < 1.1 * erfc(np.pi)
    assert np.max(np.abs(u - ue)) / np.max(ue) < 5e-5


def test_coulomb_operator_symmetric_positive():
    """K (rho -> u) is symmetric and positive for the Coulomb kernels (its matrix is
    sum_m w_m cos(k_m . (x_i - x_j)) with positive weights)."""
    rng = np.random.default_rng(11)
    for n, L, ker in [((16, 12), (4.0, 3.0), op.COULOMB2D), ((8, 8, 8), (3.0, 3.0, 3.0), op.COULOMB3D)]:
        P = op.DirectPotential(n, L, ker)
        a, b = rng.normal(size=n), rng.normal(size=n)
        Ka, Kb = P(a), P(b)
        assert abs(np.sum(b * Ka) - np.sum(a * Kb)) < 1e-12 * np.sum(np.abs(a * Kb))
        assert np.sum(a * Ka) > 0


def test_rotation_equivariance_2d():
    """With n_phi divisible by 4 the node set is invariant under 90-degree rotation, so rotating
    the density rotates the potential exactly (catches a transposed or mis-ordered axis)."""
    n, L = (32, 32), (8.0, 8.0)
    rho, _ = inputs.density_2d_bumps(n, L, seed=2, n_bumps=2)
    for ker in (op.COULOMB2D, op.LAPLACE2D):
        u = op.potential(rho, n, L, ker)
        # rot90 about the grid centre: index j -> n - j maps x -> -x on the periodic grid.  The
        # free-space potential is not periodic, so row 0 of the rotated field (which needs u at
        # x = +L, off the grid) is not compared; the density is ~1e-28 there, so wrapping it is harmless.
        rot = np.roll(np.rot90(rho), 1, axis=0)
        ur = op.potential(rot, n, L, ker)
        want = np.roll(np.rot90(u), 1, axis=0)
        assert np.max(np.abs(ur[1:] - want[1:])) < 1e-12 * np.max(np.abs(u))


def test_laplace2d_sigma_invariance():
    """The subtracted Gaussian only moves work between u1 and u2 (Sec. 2.2); the sum does not
    depend on sigma beyond the dropped tail of the Gaussian outside the ball."""
    n, L = (48, 48), (8.0, 8.0)
    rho, _ = inputs.density_2d_bumps(n, L, seed=4, n_bumps=3)
    P = np.pi / (16.0 / 48)
    u1 = op.potential(rho, n, L, op.LAPLACE2D, sigma=6 * np.sqrt(2) / P)
    u2 = op.potential(rho, n, L, op.LAPLACE2D, sigma=1.2 * 6 * np.sqrt(2) / P)
    assert np.max(np.abs(u1 - u2)) < 1e-12 * np.max(np.abs(u1))
    # the printed sigma = 6/P leaves a Gaussian tail e^{-18} outside the ball: visible at 1e-9
    u3 = op.potential(rho, n, L, op.LAPLACE2D, sigma=6.0 / P)
    assert 1e-11 < np.max(np.abs(u1 - u3)) / np.max(np.abs(u1)) < 1e-6


# ---- confined Coulomb kernel (Sec. 2, Eq. 'Kernal124d'; Sec. 2.3, Eqs. 'ifft2d', '2Dw1') ----------

def test_confined_w1_quadrature_equals_erfcx_and_asymptotes():
    """The oracle's W1 (Gauss-Kronrod quadrature of Eq. '2Dw1') equals erfcx(eps |k| / sqrt 2),
    the closed form of that integral, is 1 at k = 0, and follows the paper's limits
    Uhat ~ 1/|k| (|k| -> 0) and Uhat ~ sqrt(2) / (sqrt(pi) eps |k|^2) (|k| -> inf)."""
    from scipy.special import erfcx
    eps = 0.3
    k = np.concatenate([[0.0, 1e-8, 1e-3], np.geomspace(0.01, 3e4, 40)])
    w1 = op.confined_w1(k, eps)
    want = erfcx(eps * k / np.sqrt(2.0))
    assert np.max(np.abs(w1 / want - 1.0)) < 1e-13
    assert w1[0] == 1.0 and abs(w1[1] - 1.0) < 1e-8
    big = k > 1e4
    asym = np.sqrt(2.0) / (np.sqrt(np.pi) * eps * k[big])     # |k| Uhat at large |k|
    assert np.max(np.abs(w1[big] / asym - 1.0)) < 1e-6


@pytest.mark.parametrize("sigma2,eps", [(1.2, 0.1), (1.2, 1.0), (2.0, 3.0)])
def test_confined2d_gaussian_closed_form(sigma2, eps):
    """rho = exp(-|x|^2/sigma^2) on [-8,8]^2, h = 1/4: the oracle's potential equals the Hankel
    integral of the Gaussian (erfcx and J0, independent of the oracle's quadrature W1) at
    sampled points, and at the origin the elementary closed form; both derivations of u(0)
    agree with each other."""
    n, L = (64, 64), (8.0, 8.0)
    sigma = np.sqrt(sigma2)
    (X, Y), _ = _grid(n, L)
    u = op.potential(np.exp(-(X * X + Y * Y) / sigma2), n, L, op.CONFINED2D, eps=eps)
    u0 = cf.confined2d_gauss_origin(sigma, eps)
    assert abs(float(cf.confined2d_gauss(0.0, sigma, eps)) - u0) < 1e-13 * u0
    assert abs(u[32, 32] - u0) < 1e-13 * u0
    idx = [(40, 32), (32, 50), (10, 20), (0, 0), (60, 5)]
    want = cf.confined2d_gauss(np.array([np.hypot(X[i], Y[i]) for i in idx]), sigma, eps)
    got = np.array([u[i] for i in idx])
    assert np.max(np.abs(got - want)) < 1e-12 * u0


def test_confined2d_small_eps_is_coulomb2d():
    """eps -> 0 takes U_Con^eps to the 2D Coulomb kernel (W1 -> 1): the two
    oracle potentials agree to rounding at eps = 1e-16 (W1 = 1 - O(eps |k|)), and at eps = 1e-3
    they differ by O(eps)."""
    n, L = (32, 32), (6.0, 6.0)
    rho, _ = inputs.density_2d_bumps(n, L, seed=3, n_bumps=3)
    uc = op.potential(rho, n, L, op.COULOMB2D)
    u0 = op.potential(rho, n, L, op.CONFINED2D, eps=1e-16)
    u3 = op.potential(rho, n, L, op.CONFINED2D, eps=1e-3)
    assert np.max(np.abs(u0 - uc)) < 1e-14 * np.max(np.abs(uc))
    d = np.max(np.abs(u3 - uc)) / np.max(np.abs(uc))
    assert 1e-5 < d < 1e-2


def test_anisotropic_closed_forms_reduce_to_isotropic():
    """The anisotropic closed forms at equal widths are the isotropic ones: Example 2.1's gamma != 1
    integral at gamma = 1 (erf formula) and the heat-semigroup 2D Laplace formula at a = b (the
    E1 formula of Example 2.3), at points along a skew direction."""
    for r in (0.0, 0.3, 1.0, 2.5, 4.0):
        x, y, z = 0.48 * r, 0.6 * r, 0.64 * r
        want = float(cf.coulomb3d_gauss(np.array(r), 1.3))
        got = float(cf.coulomb3d_gauss_aniso(x, y, z, 1.3, 1.0))
        assert abs(got - want) <= 1e-12 * abs(want)
        x2, y2 = 0.6 * r, 0.8 * r
        want2 = float(cf.laplace2d_gauss(np.array(r), 0.8))
        got2 = float(cf.laplace2d_gauss_aniso(x2, y2, 0.8, 0.8))
        assert abs(got2 - want2) <= 1e-11 * max(1.0, abs(want2))
