"""Fourier-space quadrature of the ball |k| <= P (oracle; test infrastructure only).

Sec. 2.1, Eq. 'ifft': after truncating the Fourier integral to the ball |k| <= P and
switching to spherical (3D) or polar (2D) coordinates, the Jacobian |k|^(d-1) cancels
the Coulomb symbol 1/|k|^(d-1), leaving a smooth integrand in (|k|, theta, phi) that a
high-order quadrature integrates.  The paper does not name the rules; the reading taken
here (stated in the design notes) is:

* radial:   n_r-point Gauss-Legendre on [0, P];
* polar:    n_theta-point Gauss-Legendre in mu = cos(theta) on [-1, 1] (absorbs sin(theta));
* azimuth:  n_phi-point trapezoid rule phi_c = 2 pi c / n_phi (exact for trigonometric
            polynomials, the natural rule for a periodic variable).

Node coordinates, axis convention: k = r (sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi, mu)
in 3D and k = r (cos phi, sin phi) in 2D, components ordered like the grid axes.

parity pin: Gauss-Legendre exactness on polynomials (tests/test_oracle_quadrature.py).
"""
import numpy as np
from numpy.polynomial.legendre import leggauss


def gauss_legendre(n):
    """n-point Gauss-Legendre nodes and weights on [-1, 1] (library routine)."""
    t, w = leggauss(int(n))
    return np.asarray(t, dtype=np.float64), np.asarray(w, dtype=np.float64)


def radial_rule(P, n_r):
    """Gauss-Legendre on [0, P]: r_a = P (t_a + 1) / 2, w_a = P omega_a / 2."""
    t, w = gauss_legendre(n_r)
    return 0.5 * P * (t + 1.0), 0.5 * P * w


def ball_nodes(dim, P, n_r, n_phi, n_theta=None):
    """All quadrature nodes of the ball of radius P, full (unsymmetrised) set.

    Returns (k, weight, kmag):
      k      (M, dim) node coordinates,
      weight (M,)     quadrature weight of the measure d|k| d(mu) d(phi) (3D) or
                      d|k| d(phi) (2D) -- i.e. WITHOUT the Jacobian, which the
                      Coulomb symbol cancels (Sec. 2.1, Eq. 'ifft'),
      kmag   (M,)     |k| = r_a.
    Node order: radial index slowest, then polar (3D), then azimuth fastest.
    """
    r, wr = radial_rule(P, n_r)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    wphi = 2.0 * np.pi / n_phi
    if dim == 2:
        R, PH = np.meshgrid(r, phi, indexing="ij")
        k = np.stack([R * np.cos(PH), R * np.sin(PH)], axis=-1).reshape(-1, 2)
        weight = np.repeat(wr * wphi, n_phi)
        return k, weight, R.reshape(-1)
    if dim == 3:
        if n_theta is None:
            raise ValueError("3D needs n_theta")
        mu, wmu = gauss_legendre(n_theta)
        R, MU, PH = np.meshgrid(r, mu, phi, indexing="ij")
        S = np.sqrt(1.0 - MU * MU)
        k = np.stack([R * S * np.cos(PH), R * S * np.sin(PH), R * MU], axis=-1).reshape(-1, 3)
        weight = (wr[:, None, None] * wmu[None, :, None] * wphi * np.ones((1, 1, n_phi))).reshape(-1)
        return k, weight, R.reshape(-1)
    raise ValueError("dim must be 2 or 3")
