"""Split evaluation of the 3D Coulomb potential (test infrastructure only).

Sec. 2.1, Eq. '3.9' and Fig. 'fig3.1': a partition of unity p(k) divides the Fourier integral
of u = U * rho (Uhat = 1/|k|^2) into

    I1 = (2 pi)^-3 int_D  e^{ik.x} w(k) rhohat(k) dk,     w = (1 - p(k)) / |k|^2   (smooth),
    I2 = (2 pi)^-3 int_{|k| <= P2} e^{ik.x} p(k) rhohat(k) d|k| dmu dphi            (Jacobian cancelled),

with D = prod_i [-P_i, P_i), P_i = pi / h_i, the cube of the grid's frequencies, and p the
Gaussian e^{-|k|^2 / a} that the paper allows in 3D (w(0) = 1/a).  I1 is the trapezoid rule on
the frequency lattice k_l = l dk_i, dk_i = pi / (2 L_i), l_i in [-n_i, n_i): with rhohat from
the trapezoid sum of the grid data (reading c4) it is a cyclic convolution of the grid data,
zero-padded to 2 n_i per axis, computed here with numpy's FFT as a library step.  I2 is the
ball quadrature of the plain method (same rules as `oracle.quadrature`) on the small ball
|k| <= P2 with the weights multiplied by p(|k|), evaluated by the direct sums of
`oracle.potential`.

Parameters (the paper leaves them open; reading taken here, stated in the design notes):
    sqrt(a) = 5.5 / min_i L_i      I1's kernel erfc(sqrt(a) r / 2) / (4 pi r) has fallen to
                                   erfc(5.5) ~ 7e-15 at the nearest periodic image (2 L away);
    P2 = sqrt(34.5 a)              p(P2) = e^{-34.5} ~ 1e-15;
    n_r = n_theta = ceil(3 P2 D / 8) + 8, n_phi = 2 n_theta, D = 2 |L| the box diameter
                                   (the largest phase |k| |x - x_j| across the box is P2 D;
                                   on densities near opposite corners of the box the ball sum has
                                   converged to rounding from about 0.65 P2 D / 2 nodes on, and
                                   this rule keeps 0.75 of P2 D / 2 plus 8).
The split needs the grid's cube to hold the ball: P_i >= sqrt(34.5 a) on every axis.

parity pins (tests/test_oracle_split.py): I1 and I2 each against their closed forms for a
Gaussian density, their sum against the 3D Coulomb closed form of Example 2.1, the independence
of the sum from a, and the ball rule against a finer one on densities in the box's corners.
"""
import numpy as np

from .potential import type1_direct, type2_direct
from .quadrature import ball_nodes


def split_params(n, L, a=None, n_r=None, n_theta=None, n_phi=None):
    """The split's parameters for a grid (module docstring)."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in L)
    h = [2.0 * Li / ni for ni, Li in zip(n, L)]
    P = np.pi / max(h)
    if a is None:
        a = (5.5 / min(L)) ** 2
    P2 = np.sqrt(34.5 * a)
    if P2 > P:
        raise ValueError("grid too coarse for the split: pi / max(h) = %g < sqrt(34.5 a) = %g" % (P, P2))
    D = 2.0 * np.sqrt(sum(Li * Li for Li in L))
    nr = int(np.ceil(3.0 * P2 * D / 8.0)) + 8
    n_r = nr if n_r is None else int(n_r)
    n_theta = nr if n_theta is None else int(n_theta)
    n_phi = 2 * nr if n_phi is None else int(n_phi)
    return dict(a=float(a), P2=float(P2), n_r=n_r, n_theta=n_theta, n_phi=n_phi)


def w_smooth(kk, a):
    """w = (1 - e^{-|k|^2/a}) / |k|^2 from |k|^2, with w = 1/a at k = 0."""
    kk = np.asarray(kk, dtype=np.float64)
    out = np.full(kk.shape, 1.0 / a)
    nz = kk > 0
    out[nz] = -np.expm1(-kk[nz] / a) / kk[nz]
    return out


def i1_regular(rho, n, L, a):
    """I1 on the grid: (2 pi)^-3 dk^3 sum_l e^{ik_l.x_j'} w(k_l) rhohat(k_l), l_i in [-n_i, n_i).

    With x_j = -L + j h and rhohat(k_l) = h^3 sum_j rho_j e^{-ik_l.x_j}, the phases e^{-+ik_l L}
    cancel and the sum is the cyclic convolution of rho zero-padded to 2n_i per axis with the
    lattice transform of w, scaled by h^3 dk^3 / (2 pi)^3 = 1 / prod(2 n_i)."""
    n = tuple(int(v) for v in n)
    rho = np.asarray(rho, dtype=np.float64).reshape(n)
    pad = np.zeros(tuple(2 * v for v in n))
    pad[:n[0], :n[1], :n[2]] = rho
    ks = [2.0 * np.pi * np.fft.fftfreq(2 * ni, d=2.0 * float(Li) / ni) for ni, Li in zip(n, L)]
    K0, K1, K2 = np.meshgrid(*ks, indexing="ij")
    w = w_smooth(K0 * K0 + K1 * K1 + K2 * K2, a)
    out = np.fft.ifftn(w * np.fft.fftn(pad))     # ifftn includes the 1 / prod(2 n_i)
    return out.real[:n[0], :n[1], :n[2]]


def i2_ball(rho, n, L, a, P2, n_r, n_theta, n_phi):
    """I2 on the grid: the ball quadrature of radius P2 with weights times e^{-|k|^2/a}."""
    k, weight, kmag = ball_nodes(3, P2, n_r, n_phi, n_theta)
    rhohat = type2_direct(rho, n, L, k)
    c = (2.0 * np.pi) ** -3 * weight * np.exp(-kmag * kmag / a) * rhohat
    return type1_direct(c, n, L, k)


def split_potential(rho, n, L, a=None, n_r=None, n_theta=None, n_phi=None, return_parts=False):
    """u = I1 + I2 for the 3D Coulomb kernel (module docstring)."""
    prm = split_params(n, L, a, n_r, n_theta, n_phi)
    u1 = i1_regular(rho, n, L, prm["a"])
    u2 = i2_ball(rho, n, L, prm["a"], prm["P2"], prm["n_r"], prm["n_theta"], prm["n_phi"])
    if return_parts:
        return u1 + u2, dict(I1=u1, I2=u2, **prm)
    return u1 + u2
