"""Direct-summation oracle for the NUFFT potential (test infrastructure only).

What the GPU path approximates with a type-2 NUFFT, a symbol multiply and a type-1
NUFFT, this module computes *exactly* (to FP64 rounding) by direct nonuniform DFT
sums.  No FFT, no spreading, no blocking beyond chunking the node set:

    u(x_j) = Re sum_m c_m exp(+i k_m . x_j),
    c_m    = (2 pi)^-d  weight_m  S_m,
    S_m    = rhohat(k_m)                                   Coulomb 3D / 2D  (Sec. 2.1, Eq. 'ifft')
           = [rhohat(k_m) - (m0 - i k_m . m1) e^{-sigma^2 |k_m|^2 / 2}] / |k_m|
                                                           Laplace 2D        (Sec. 2.2, Eq. 'phi2fourier')
           = W1(|k_m|) rhohat(k_m)                         confined Coulomb 2D (Sec. 2.3, Eqs. 'ifft2d',
                                                           '2Dw1'), W1 by adaptive Gauss-Kronrod
                                                           quadrature of its defining integral
    rhohat(k) = (prod_i h_i) sum_j rho_j exp(-i k . x_j)   trapezoid rule for the Fourier
                                                           transform of grid data (Alg. 1, first step)

and, for the 2D Laplace kernel, u += m0 u11(x) - m1 . u12(x) (Sec. 2.2, Eqs. 'phi1_exct',
'phi12_ext'), with m0 = rhohat(0), m1 = (x rho)^(0), both by the same trapezoid rule.

The Fourier transform convention is fhat(k) = int f(x) exp(-i k.x) dx (Sec. 1, under Eq.
'Kernal').  The grid is x_j = -L_i + j h_i, h_i = 2 L_i / n_i, j = 0..n_i-1 (periodic
reading of the mesh Omega_h of Sec. 2.4).

parity pins: closed-form potentials of Gaussian densities (Examples 2.1-2.3), Fourier
transform of a shifted Gaussian, adjointness of the two sums, symmetry and positivity
of the operator (tests/test_oracle_potential.py).
"""
import numpy as np
from scipy.integrate import quad
from scipy.special import exp1

from .quadrature import ball_nodes

EULER_GAMMA = 0.57721566490153286061

COULOMB3D = 1   # U = 1/(4 pi |x|),   Uhat = 1/|k|^2   (Sec. 1, Eq. 'Kernal', d = 3)
COULOMB2D = 2   # U = 1/(2 pi |x|),   Uhat = 1/|k|     (Sec. 1, Eq. 'Kernal', d = 2)
LAPLACE2D = 3   # U = -ln|x| / (2 pi), Uhat = 1/|k|^2  (Sec. 1, Eq. 'Kernal21d', d = 2)
CONFINED2D = 4  # U_Con^eps, Uhat = (2/pi) int_0^inf e^{-eps^2 s^2/2} / (|k|^2 + s^2) ds
                #                                      (Sec. 2, Eq. 'Kernal124d', d = 2)

_CHUNK = 2048


def grid_axes(n, L):
    """Per-axis coordinates x_i[j] = -L_i + j h_i and spacings h_i."""
    h = [2.0 * float(Li) / int(ni) for ni, Li in zip(n, L)]
    xs = [-float(Li) + hi * np.arange(int(ni), dtype=np.float64) for ni, Li, hi in zip(n, L, h)]
    return xs, h


def type2_direct(rho, n, L, k):
    """rhohat_m = (prod h) sum_j rho_j exp(-i k_m . x_j), exact sum, chunked over nodes."""
    rho = np.asarray(rho, dtype=np.float64).reshape(tuple(n))
    xs, h = grid_axes(n, L)
    dim = len(n)
    M = k.shape[0]
    out = np.empty(M, dtype=np.complex128)
    for s in range(0, M, _CHUNK):
        kc = k[s:s + _CHUNK]
        E = [np.exp(-1j * np.outer(kc[:, i], xs[i])) for i in range(dim)]   # (m, n_i)
        if dim == 2:
            T = rho @ E[1].T                                  # (n0, m): sum over j1
            out[s:s + _CHUNK] = np.sum(E[0].T * T, axis=0)    # sum over j0
        else:
            n0, n1, n2 = n
            T1 = (rho.reshape(n0 * n1, n2) @ E[2].T).reshape(n0, n1, -1)   # sum over j2
            T2 = np.einsum("abm,mb->am", T1, E[1])                           # sum over j1
            out[s:s + _CHUNK] = np.sum(E[0].T * T2, axis=0)                  # sum over j0
    return np.prod(h) * out


def type1_direct(c, n, L, k, return_complex=False):
    """u_j = sum_m c_m exp(+i k_m . x_j) (real part unless return_complex)."""
    xs, _ = grid_axes(n, L)
    dim = len(n)
    M = k.shape[0]
    acc = np.zeros(tuple(n), dtype=np.complex128)
    for s in range(0, M, _CHUNK):
        kc = k[s:s + _CHUNK]
        cc = c[s:s + _CHUNK]
        E = [np.exp(1j * np.outer(kc[:, i], xs[i])) for i in range(dim)]    # (m, n_i)
        if dim == 2:
            acc += (E[0] * cc[:, None]).T @ E[1]
        else:
            n0, n1, n2 = n
            A = (cc[:, None, None] * E[0][:, :, None] * E[1][:, None, :]).reshape(-1, n0 * n1)
            acc += (A.T @ E[2]).reshape(n0, n1, n2)
    return acc if return_complex else acc.real


def moments(rho, n, L):
    """m0 = rhohat(0) = (prod h) sum rho_j, m1 = (x rho)^(0) = (prod h) sum x_j rho_j."""
    rho = np.asarray(rho, dtype=np.float64).reshape(tuple(n))
    xs, h = grid_axes(n, L)
    w = np.prod(h)
    m0 = w * rho.sum()
    m1 = []
    for i in range(len(n)):
        shape = [1] * len(n)
        shape[i] = -1
        m1.append(w * np.sum(rho * xs[i].reshape(shape)))
    return m0, np.array(m1)


def confined_w1(kmag, eps):
    """W1(|k|) = |k| Uhat_Con^eps(k) = (2/pi) int_0^inf e^{-eps^2 |k|^2 s^2 / 2} / (1 + s^2) ds,
    W1(0) = 1 (Sec. 2.3, Eq. '2Dw1'), by adaptive Gauss-Kronrod quadrature (QUADPACK, as the
    paper suggests) once per distinct |k|.  With a = eps |k| / sqrt 2 and t = a s the integral
    is (2/pi) int_0^inf e^{-t^2} a / (a^2 + t^2) dt; for a <= 1, where that integrand is a
    spike of width a, the same integral is taken as 1 - (2/pi) int_0^inf (1 - e^{-t^2}) a /
    (a^2 + t^2) dt (int_0^inf ds / (1 + s^2) = pi/2 subtracted), whose integrand is smooth."""
    kmag = np.asarray(kmag, dtype=np.float64)
    vals = {}
    for q in np.unique(kmag):
        a = eps * q / np.sqrt(2.0)
        if a == 0.0:
            vals[q] = 1.0
            continue
        if a <= 1.0:
            f = lambda t: -np.expm1(-t * t) * a / (a * a + t * t)
            v, _ = quad(f, 0.0, np.inf, epsabs=1e-17, epsrel=1e-13, limit=400)
            vals[q] = 1.0 - 2.0 / np.pi * v
        else:
            f = lambda t: np.exp(-t * t) * a / (a * a + t * t)
            v, _ = quad(f, 0.0, np.inf, epsabs=1e-17, epsrel=1e-13, limit=400)
            vals[q] = 2.0 / np.pi * v
    return np.vectorize(vals.__getitem__, otypes=[np.float64])(kmag)


def symbol_coeffs(kernel, k, weight, kmag, rhohat, m0=None, m1=None, sigma=None, w1=None):
    """c_m = (2 pi)^-d weight_m S_m with S_m per kernel (module docstring); w1: W1(|k_m|) of the
    confined kernel."""
    dim = k.shape[1]
    if kernel in (COULOMB3D, COULOMB2D):
        S = rhohat
    elif kernel == CONFINED2D:
        S = w1 * rhohat
    elif kernel == LAPLACE2D:
        kdotm1 = k @ m1
        G1hat = (m0 - 1j * kdotm1) * np.exp(-0.5 * sigma * sigma * kmag * kmag)
        S = (rhohat - G1hat) / kmag
    else:
        raise ValueError("unknown kernel")
    return (2.0 * np.pi) ** (-dim) * weight * S


def u11(X, Y, sigma):
    """u_{1,1} = U_Lap * G for the normalised 2D Gaussian of width sigma (Sec. 2.2, Eq. 'phi1_exct')."""
    r2 = X * X + Y * Y
    out = np.empty_like(r2)
    nz = r2 > 0
    out[nz] = -(exp1(r2[nz] / (2.0 * sigma * sigma)) + np.log(r2[nz])) / (4.0 * np.pi)
    out[~nz] = (EULER_GAMMA - np.log(2.0 * sigma * sigma)) / (4.0 * np.pi)
    return out


def u12(X, Y, sigma):
    """u_{1,2} = grad u_{1,1} (Sec. 2.2, Eq. 'phi12_ext'); returns the two components."""
    r2 = X * X + Y * Y
    fx = np.zeros_like(r2)
    fy = np.zeros_like(r2)
    nz = r2 > 0
    f = -(1.0 - np.exp(-r2[nz] / (2.0 * sigma * sigma))) / (2.0 * np.pi * r2[nz])
    fx[nz] = f * X[nz]
    fy[nz] = f * Y[nz]
    return fx, fy


def default_sigma(P):
    """Width of the subtracted Gaussian for the 2D Laplace kernel.

    Sec. 2.2 asks for the Gaussian e^{-sigma^2 |k|^2/2} to be 2e-16 at |k| = P; solving
    that gives sigma = 6 sqrt(2) / P (the printed 6/P only reaches e^-18).  Reading taken:
    6 sqrt(2) / P.
    """
    return 6.0 * np.sqrt(2.0) / P


class DirectPotential:
    """u = U * rho on one grid by the direct quadrature sum (module docstring).

    Holds the node set and, for small problems, the per-axis exponential tables so that
    repeated evaluations (inside the tiny solver oracles) do not rebuild them.  The sums
    themselves are those of `type2_direct` / `type1_direct`.

    Defaults follow the plan's reading: P = pi / max(h_i); (n_r, n_theta, n_phi) =
    (n_0, n_0, 2 n_0).
    """

    def __init__(self, n, L, kernel, P=None, n_r=None, n_theta=None, n_phi=None, sigma=None, eps=None):
        self.n = tuple(int(v) for v in n)
        self.L = tuple(float(v) for v in L)
        dim = len(self.n)
        if (kernel == COULOMB3D and dim != 3) or (kernel in (COULOMB2D, LAPLACE2D, CONFINED2D) and dim != 2):
            raise ValueError("kernel/dimension mismatch")
        if kernel == CONFINED2D and not (eps is not None and eps > 0):
            raise ValueError("the confined kernel needs eps > 0")
        self.dim, self.kernel = dim, kernel
        self.xs, self.h = grid_axes(self.n, self.L)
        self.P = np.pi / max(self.h) if P is None else float(P)
        self.n_r = self.n[0] if n_r is None else int(n_r)
        self.n_theta = self.n[0] if n_theta is None else int(n_theta)
        self.n_phi = 2 * self.n[0] if n_phi is None else int(n_phi)
        self.k, self.weight, self.kmag = ball_nodes(dim, self.P, self.n_r, self.n_phi,
                                                    self.n_theta if dim == 3 else None)
        self.sigma = None
        self.w1 = confined_w1(self.kmag, float(eps)) if kernel == CONFINED2D else None
        if kernel == LAPLACE2D:
            self.sigma = default_sigma(self.P) if sigma is None else float(sigma)
            X, Y = np.meshgrid(self.xs[0], self.xs[1], indexing="ij")
            self._u11 = u11(X, Y, self.sigma)
            self._u12 = u12(X, Y, self.sigma)

    def __call__(self, rho, return_parts=False, rhohat=None):
        """u for the density rho.  rhohat: the type-2 sum of this same rho on this node set
        (`type2_direct`), when a caller already has it (two kernels of one density share it)."""
        rho = np.asarray(rho, dtype=np.float64).reshape(self.n)
        if rhohat is None:
            rhohat = type2_direct(rho, self.n, self.L, self.k)
        m0 = m1 = None
        if self.kernel == LAPLACE2D:
            m0, m1 = moments(rho, self.n, self.L)
        c = symbol_coeffs(self.kernel, self.k, self.weight, self.kmag, rhohat, m0, m1, self.sigma, self.w1)
        uc = type1_direct(c, self.n, self.L, self.k, return_complex=True)
        u = uc.real.copy()
        if self.kernel == LAPLACE2D:
            u += m0 * self._u11 - (m1[0] * self._u12[0] + m1[1] * self._u12[1])
        if return_parts:
            return u, dict(k=self.k, weight=self.weight, kmag=self.kmag, rhohat=rhohat, c=c,
                           imag=uc.imag, m0=m0, m1=m1, sigma=self.sigma, P=self.P)
        return u


def potential(rho, n, L, kernel, P=None, n_r=None, n_theta=None, n_phi=None, sigma=None,
              return_parts=False, eps=None):
    """One-shot direct evaluation; see `DirectPotential`."""
    op = DirectPotential(n, L, kernel, P, n_r, n_theta, n_phi, sigma, eps)
    return op(rho, return_parts=return_parts)
