"""Analytic potentials of Gaussian densities (test infrastructure only).

These pin the oracle to something other than itself: the continuum potential that the
quadrature sum approximates.  Each function states the density it belongs to.

* 3D Coulomb, rho = exp(-(x^2+y^2+gamma^2 z^2)/sigma^2)   -- Example 2.1, Eq. 'DensGaus'
* 2D Coulomb, rho = exp(-(x^2+gamma^2 y^2)/sigma^2)       -- Example 2.2, Eq. '2.5D-clb-exact'
* 2D Laplace, rho = exp(-|x|^2/sigma^2)                   -- Example 2.3, Eq. 'eg-2d-Exact'
* 2D confined Coulomb U_Con^eps (Sec. 2, Eq. 'Kernal124d'), rho = exp(-|x|^2/sigma^2) -- not in
  the paper; derived here.  With W1(k) = |k| Uhat = erfcx(eps |k| / sqrt 2) (Eq. '2Dw1' is
  (2/pi) int e^{-a^2 s^2}/(1+s^2) ds = erfcx(a), a standard integral) and
  rhohat = pi sigma^2 e^{-sigma^2 k^2 / 4}, the polar form of Eq. 'ifft2d' gives
      u(r) = (sigma^2 / 2) int_0^inf erfcx(eps k / sqrt 2) e^{-sigma^2 k^2 / 4} J0(k r) dk,
  and at r = 0, putting the integral of W1 back and integrating over k first,
      u(0) = sigma^2 / (2 sqrt pi) int_0^inf ds / ((1 + s^2) sqrt(c^2 + b^2 s^2)),
  c = sigma / 2, b = eps / sqrt 2, which is arccos(b/c)/q with q = sqrt(c^2 - b^2) for c > b
  (acosh(b/c)/q, q = sqrt(b^2 - c^2), for b > c; 1/c for b = c).  eps -> 0 gives the 2D
  Coulomb value sqrt(pi) sigma / 2.
* 2D Laplace, rho = exp(-x^2/a^2 - y^2/b^2)               -- not in the paper; derived from
  the heat-semigroup representation -Delta^{-1} = int_0^inf e^{t Delta} dt with the
  logarithmic far field of Sec. 2.2 (Eq. 'Poiff35a') fixing the constant:
      u = int_0^inf [ ab e^{-x^2/(a^2+4t) - y^2/(b^2+4t)} / sqrt((a^2+4t)(b^2+4t))
                      - ab e^{-1/(4t)} / (4t) ] dt,
  which reduces to the isotropic formula when a = b (checked in the tests).
"""
import numpy as np
from scipy.integrate import quad
from scipy.special import erf, erfcx, exp1, i0e, j0

EULER_GAMMA = 0.57721566490153286061


def coulomb3d_gauss(r, sigma):
    """sigma^3 sqrt(pi) erf(r/sigma) / (4 r); sigma^2/2 at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    nz = r > 0
    out[nz] = sigma ** 3 * np.sqrt(np.pi) * erf(r[nz] / sigma) / (4.0 * r[nz])
    out[~nz] = 0.5 * sigma * sigma
    return out


def coulomb3d_gauss_aniso(x, y, z, sigma, gamma):
    """Example 2.1, gamma != 1 branch: a 1D integral evaluated by adaptive quadrature (tested at
    gamma = 1 against the erf formula and at gamma = 2 against the split evaluation)."""
    g2 = gamma ** -2

    def one(xx, yy, zz):
        def f(t):
            return (np.exp(-(xx * xx + yy * yy) / (sigma * sigma * (t + 1.0)))
                    * np.exp(-zz * zz / (sigma * sigma * (t + g2)))
                    / ((t + 1.0) * np.sqrt(t + g2)))
        v1, _ = quad(f, 0.0, 1.0, epsabs=1e-16, epsrel=1e-13, limit=400)
        v2, _ = quad(f, 1.0, np.inf, epsabs=1e-16, epsrel=1e-13, limit=400)
        return sigma * sigma / (4.0 * gamma) * (v1 + v2)

    return np.vectorize(one)(x, y, z)


def coulomb2d_gauss(r, sigma):
    """(sqrt(pi) sigma / 2) I0(r^2/(2 sigma^2)) exp(-r^2/(2 sigma^2))."""
    r = np.asarray(r, dtype=np.float64)
    return 0.5 * np.sqrt(np.pi) * sigma * i0e(r * r / (2.0 * sigma * sigma))


def coulomb2d_gauss_aniso(x, y, sigma, gamma):
    """Example 2.2, gamma != 1 branch: (sigma/(gamma sqrt pi)) int_0^inf ... dt."""
    g2 = gamma ** -2

    def one(xx, yy):
        def f(t):
            t2 = t * t
            return (np.exp(-xx * xx / (sigma * sigma * (t2 + 1.0)))
                    * np.exp(-yy * yy / (sigma * sigma * (t2 + g2)))
                    / (np.sqrt(t2 + 1.0) * np.sqrt(t2 + g2)))
        v1, _ = quad(f, 0.0, 1.0, epsabs=1e-16, epsrel=1e-13, limit=400)
        # t in [1, inf) -> s = 1/t in (0, 1]: dt = ds / s^2
        v2, _ = quad(lambda s: f(1.0 / s) / (s * s) if s > 0 else 0.0, 0.0, 1.0,
                     epsabs=1e-16, epsrel=1e-13, limit=400)
        return sigma / (gamma * np.sqrt(np.pi)) * (v1 + v2)

    return np.vectorize(one)(x, y)


def laplace2d_gauss(r, sigma):
    """-(sigma^2/4) [E1(r^2/sigma^2) + 2 ln r]; (sigma^2/4)(gamma_e - 2 ln sigma) at r = 0.

    For small z = r^2/sigma^2 the cancellation in E1(z) + ln z is avoided with the
    series E1(z) + ln z = -gamma_e - sum_{n>=1} (-z)^n / (n n!).
    """
    r = np.asarray(r, dtype=np.float64)
    z = r * r / (sigma * sigma)
    out = np.empty_like(r)
    small = z < 0.5
    zs = z[small]
    ser = np.zeros_like(zs)
    term = np.ones_like(zs)
    for nn in range(1, 40):
        term = term * (-zs) / nn
        ser += term / nn
    e1_plus_lnz = -EULER_GAMMA - ser
    out[small] = -(sigma * sigma / 4.0) * (e1_plus_lnz + 2.0 * np.log(sigma))
    big = ~small
    out[big] = -(sigma * sigma / 4.0) * (exp1(z[big]) + 2.0 * np.log(r[big]))
    return out


def laplace2d_gauss_aniso(x, y, a, b):
    """2D Laplace potential of exp(-x^2/a^2 - y^2/b^2) (module docstring)."""

    def one(xx, yy):
        def f(t):
            A = a * a + 4.0 * t
            B = b * b + 4.0 * t
            g = a * b * np.exp(-xx * xx / A - yy * yy / B) / np.sqrt(A * B)
            s = a * b * np.exp(-1.0 / (4.0 * t)) / (4.0 * t) if t > 0 else 0.0
            return g - s
        v1, _ = quad(f, 0.0, 1.0, epsabs=1e-15, epsrel=1e-13, limit=400)
        v2, _ = quad(lambda s: f(1.0 / s) / (s * s) if s > 0 else 0.0, 0.0, 1.0,
                     epsabs=1e-15, epsrel=1e-13, limit=400)
        return v1 + v2

    return np.vectorize(one)(x, y)


def confined2d_gauss_origin(sigma, eps):
    """u(0) of the confined Coulomb kernel for rho = exp(-|x|^2/sigma^2) (module docstring)."""
    c, b = 0.5 * sigma, eps / np.sqrt(2.0)
    if abs(c - b) < 1e-12 * c:
        integral = 1.0 / c
    elif c > b:
        q = np.sqrt(c * c - b * b)
        integral = np.arccos(b / c) / q
    else:
        q = np.sqrt(b * b - c * c)
        integral = np.arccosh(b / c) / q
    return sigma * sigma / (2.0 * np.sqrt(np.pi)) * integral


def confined2d_gauss(r, sigma, eps):
    """u(r) of the confined Coulomb kernel for rho = exp(-|x|^2/sigma^2): the radial Hankel
    integral of the module docstring by adaptive quadrature (scipy's erfcx and J0)."""
    def one(rr):
        f = lambda k: erfcx(eps * k / np.sqrt(2.0)) * np.exp(-0.25 * sigma * sigma * k * k) * j0(k * rr)
        kmax = 2.0 * 40.0 ** 0.5 / sigma * 2.0          # e^{-sigma^2 k^2 / 4} < e^{-160} beyond
        v, _ = quad(f, 0.0, kmax, epsabs=1e-17, epsrel=1e-13, limit=2000)
        return 0.5 * sigma * sigma * v
    return np.vectorize(one)(np.asarray(r, dtype=np.float64))
