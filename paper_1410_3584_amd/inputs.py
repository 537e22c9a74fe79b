"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only *generates* inputs (grids of densities and wave functions, instance
parameters); it holds none of the method's arithmetic and imports neither the oracle nor
the HIP binding.  All random draws use numpy.random.default_rng(seed) in the order stated
in each function.

Workload shapes follow the paper's examples: analytic Gaussians on uniform grids of a
periodic box [-L, L]^d with x_j = -L + j h, h = 2L/n (Sec. 2.4).
"""
import numpy as np


def axes(n, L):
    return [-float(Li) + (2.0 * float(Li) / int(ni)) * np.arange(int(ni), dtype=np.float64)
            for ni, Li in zip(n, L)]


def mesh(n, L):
    return np.meshgrid(*axes(n, L), indexing="ij")


def gaussian(n, L, sigma=1.0, gamma=None, center=None):
    """exp(-sum_i gamma_i^2 (x_i - c_i)^2 / sigma^2) (Examples 2.1-2.3 densities)."""
    X = mesh(n, L)
    gamma = [1.0] * len(n) if gamma is None else gamma
    center = [0.0] * len(n) if center is None else center
    q = sum((gi * (x - ci)) ** 2 for x, gi, ci in zip(X, gamma, center))
    return np.exp(-q / (sigma * sigma))


# ---- the five workloads -------------------------------------------------------------

def coulomb3d_gauss_32():
    """3D Coulomb check: rho = exp(-|x|^2) on a 32^3 grid of [-8,8]^3."""
    n, L = (32, 32, 32), (8.0, 8.0, 8.0)
    return n, L, gaussian(n, L, 1.0)


def bumps_2d(seed, n_bumps=8):
    """Bump parameters for the 2D workload: per bump, in this order, amplitude a ~ U[0,0.5],
    centre c ~ U[-4,4]^2, width w ~ U[0.5,2]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_bumps):
        a = rng.uniform(0.0, 0.5)
        c = rng.uniform(-4.0, 4.0, size=2)
        w = rng.uniform(0.5, 2.0)
        out.append((float(a), (float(c[0]), float(c[1])), float(w)))
    return out


def density_2d_bumps(n, L, seed, n_bumps=8):
    """exp(-(x^2 + 4 y^2)) + sum_b a_b exp(-|x - c_b|^2 / w_b^2); returns (rho, bumps)."""
    X, Y = mesh(n, L)
    rho = np.exp(-(X * X + 4.0 * Y * Y))
    bumps = bumps_2d(seed, n_bumps)
    for a, c, w in bumps:
        rho += a * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (w * w))
    return rho, bumps


def potential_2d_512(seed=1):
    """2D workload: 512^2 grid of [-16,16]^2, anisotropic Gaussian plus 8 seeded bumps."""
    n, L = (512, 512), (16.0, 16.0)
    rho, bumps = density_2d_bumps(n, L, seed)
    return n, L, rho, bumps


def psi0_phase_modulated(n, L, seed, n_modes=8):
    """Normalised Gaussian exp(-|x|^2/2) times exp(i S(x)),
    S = sum_q a_q cos(k_q . x + theta_q); per mode, in this order: a_q ~ U[0,0.5],
    k_q uniform in the ball |k| <= 2 (direction ~ normal, radius 2 U^{1/d}), theta_q ~ U[0, 2 pi).
    Normalised so that h^d sum |psi|^2 = 1."""
    rng = np.random.default_rng(seed)
    d = len(n)
    X = mesh(n, L)
    S = np.zeros(tuple(n))
    for _ in range(n_modes):
        a = rng.uniform(0.0, 0.5)
        v = rng.normal(size=d)
        v /= np.linalg.norm(v)
        kq = 2.0 * rng.uniform() ** (1.0 / d) * v
        th = rng.uniform(0.0, 2.0 * np.pi)
        S += a * np.cos(sum(kq[i] * X[i] for i in range(d)) + th)
    r2 = sum(x * x for x in X)
    psi = np.exp(-0.5 * r2) * np.exp(1j * S)
    dv = np.prod([2.0 * Li / ni for ni, Li in zip(n, L)])
    return psi / np.sqrt(dv * np.sum(np.abs(psi) ** 2))


def honeycomb_2d(n, L):
    """The 2D Coulomb dynamics application (Sec. 'Applications'; beta = 5 on [-32,32]^2 with
    h = 1/16, tau = 1e-4): honeycomb external potential
    V = 10 [cos(b1 . x) + cos(b2 . x) + cos((b1 + b2) . x)], b1 = (pi/4)(sqrt 3, 1),
    b2 = (pi/4)(-sqrt 3, 1), and initial data psi0 = exp(-(x^2 + y^2)/2), not normalised (the
    paper states it so).  Returns (V, psi0) on the mesh of n, L; no random draws."""
    X, Y = mesh(n, L)
    q = np.pi / 4.0
    b1 = (q * np.sqrt(3.0), q)
    b2 = (-q * np.sqrt(3.0), q)
    V = 10.0 * (np.cos(b1[0] * X + b1[1] * Y) + np.cos(b2[0] * X + b2[1] * Y)
                + np.cos((b1[0] + b2[0]) * X + (b1[1] + b2[1]) * Y))
    psi0 = np.exp(-0.5 * (X * X + Y * Y)).astype(np.complex128)
    return V, psi0


def ground_state_batch_2d(seed, count=64, sizes=(64, 128, 256)):
    """Batched 2D ground-state instances: per instance, in this order, grid N1 uniform over
    `sizes`, beta ~ U[10,1000], gamma ~ U[0.5,2] (V = (x^2 + gamma^2 y^2)/2), box [-16,16]^2."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        N1 = int(sizes[rng.integers(len(sizes))])
        beta = float(rng.uniform(10.0, 1000.0))
        gam = float(rng.uniform(0.5, 2.0))
        out.append(dict(n=(N1, N1), L=(16.0, 16.0), beta=beta, gamma=(1.0, gam)))
    return out


def warmstart_instances_3d(seed, count):
    """Warm-start instances: beta ~ U[1,500], (gx, gy, gz) ~ U[0.5,2]^3, in this order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        beta = float(rng.uniform(1.0, 500.0))
        g = rng.uniform(0.5, 2.0, size=3)
        out.append(dict(beta=beta, gamma=tuple(float(v) for v in g)))
    return out


def warmstart_instances_2d(seed, count, beta_lo=1.0, beta_hi=50.0):
    """2D warm-start instances: beta log-uniform in [beta_lo, beta_hi], (gx, gy) ~ U[0.5,2]^2, in this order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        beta = float(np.exp(rng.uniform(np.log(beta_lo), np.log(beta_hi))))
        g = rng.uniform(0.5, 2.0, size=2)
        out.append(dict(beta=beta, gamma=tuple(float(v) for v in g)))
    return out
