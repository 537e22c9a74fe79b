"""Tiny-grid solver oracles (test infrastructure only).

* Ground state by the gradient flow with discrete normalization, backward Euler in time,
  Fourier pseudospectral in space, nonlocal potential lagged at phi^n
  (Sec. 3.1, Eqs. 'gf-eq2', 'gf-colb2', 'gffg33').  The backward-Euler step is read
  as fully implicit in the linear part: (1/tau - Delta/2 + V + beta varphi^n) phi1 =
  phi^n / tau (the paper omits the details).  Solved here by plain conjugate gradients
  with the spectral Laplacian; stopping rule max|phi^{n+1}-phi^n|/tau <= eps0 (Sec. 3.2).
* Energies, chemical potential and virial identity (Sec. 3.2).
* Time splitting: Strang splitting of the kinetic flow (exact in Fourier space) and the
  potential flow psi <- exp(-i (V + beta varphi^n) tau) psi, which is exact because |psi| is
  invariant during it (Sec. 4.1, Eqs. 'sps-eq65'-'sps-eq68').  Yoshida's fourth-order
  composition of Strang steps is offered as `order=4` (Sec. 4.1 names it).

The nonlocal potential is evaluated with `oracle.potential.DirectPotential` (direct sums);
the Laplacian with numpy's FFT.

parity pins: beta = 0 reduces to the harmonic oscillator (E = sum gamma_i / 2 exactly);
the paper's printed ground-state energies (Tables 'virial_2d_Coulomb', 'virial_2d_Poisson');
mu = E + E_int and the virial identity; unitarity of each split step (mass), time-transverse
invariance (Sec. 1) -- tests/test_oracle_solvers.py.
"""
import numpy as np

from .potential import DirectPotential, LAPLACE2D, grid_axes


def freq_squared(n, L):
    """|mu|^2 of the discrete Fourier modes mu_l = pi l / L_i on the periodic box."""
    h = [2.0 * Li / ni for ni, Li in zip(n, L)]
    mus = [2.0 * np.pi * np.fft.fftfreq(ni, d=hi) for ni, hi in zip(n, h)]
    grids = np.meshgrid(*mus, indexing="ij")
    return sum(g * g for g in grids)


def harmonic_trap(n, L, gamma):
    """V = (1/2) sum_i gamma_i^2 x_i^2 on the grid."""
    xs, _ = grid_axes(n, L)
    grids = np.meshgrid(*xs, indexing="ij")
    return 0.5 * sum((g * gi) ** 2 for g, gi in zip(grids, gamma))


def ho_gaussian(n, L, gamma):
    """Harmonic-oscillator ground state prod (gamma_i/pi)^{1/4} exp(-gamma_i x_i^2/2), grid-normalised."""
    xs, h = grid_axes(n, L)
    grids = np.meshgrid(*xs, indexing="ij")
    phi = np.ones(tuple(n))
    for g, gi in zip(grids, gamma):
        phi = phi * (gi / np.pi) ** 0.25 * np.exp(-0.5 * gi * g * g)
    return phi / np.sqrt(np.prod(h) * np.sum(phi * phi))


def energies(phi, V, varphi, beta, n, L, kernel):
    """E_kin, E_pot, E_int, E, mu and the virial residual I (Sec. 3.2)."""
    _, h = grid_axes(n, L)
    dv = np.prod(h)
    N = phi.size
    k2 = freq_squared(n, L)
    ph = np.fft.fftn(phi)
    Ekin = 0.5 * dv * np.sum(k2 * np.abs(ph) ** 2) / N
    dens = np.abs(phi) ** 2
    Epot = dv * np.sum(V * dens)
    Eint = 0.5 * beta * dv * np.sum(varphi * dens)
    E = Ekin + Epot + Eint
    mu = E + Eint
    if kernel == LAPLACE2D:
        virial = 2.0 * Ekin - 2.0 * Epot + beta / (4.0 * np.pi)
    else:
        virial = 2.0 * Ekin - 2.0 * Epot + Eint
    return dict(Ekin=Ekin, Epot=Epot, Eint=Eint, E=E, mu=mu, virial=virial)


def _cg(apply_A, b, x0, rtol, maxit):
    x = x0.copy()
    r = b - apply_A(x)
    p = r.copy()
    rr = np.sum(r * r)
    bn = np.sqrt(np.sum(b * b))
    for _ in range(maxit):
        if np.sqrt(rr) <= rtol * bn:
            break
        Ap = apply_A(p)
        alpha = rr / np.sum(p * Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = np.sum(r * r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def ground_state(n, L, kernel, beta, gamma, tau=1e-2, eps0=1e-10, max_iter=100000,
                 phi0=None, pot=None, cg_rtol=1e-14, cg_maxit=2000):
    """Backward-Euler normalized gradient flow; returns (phi, stats)."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in L)
    _, h = grid_axes(n, L)
    dv = np.prod(h)
    if pot is None:
        pot = DirectPotential(n, L, kernel)
    V = harmonic_trap(n, L, gamma)
    k2 = freq_squared(n, L)
    phi = ho_gaussian(n, L, gamma) if phi0 is None else np.array(phi0, dtype=np.float64)
    phi = phi / np.sqrt(dv * np.sum(phi * phi))
    res = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        varphi = pot(phi * phi)
        W = V + beta * varphi

        def apply_A(v):
            lap = np.real(np.fft.ifftn(0.5 * k2 * np.fft.fftn(v)))
            return v / tau + lap + W * v

        phi1 = _cg(apply_A, phi / tau, phi, cg_rtol, cg_maxit)
        phi_new = phi1 / np.sqrt(dv * np.sum(phi1 * phi1))
        res = np.max(np.abs(phi_new - phi)) / tau
        phi = phi_new
        if res <= eps0:
            break
    varphi = pot(phi * phi)
    st = energies(phi, V, varphi, beta, n, L, kernel)
    st.update(iters=it, residual=res, mass=dv * np.sum(phi * phi))
    return phi, st


def _strang(psi, dt, k2, V, beta, pot):
    kin = np.exp(-0.25j * dt * k2)
    psi = np.fft.ifftn(kin * np.fft.fftn(psi))
    varphi = pot(np.abs(psi) ** 2)
    psi = np.exp(-1j * (V + beta * varphi) * dt) * psi
    psi = np.fft.ifftn(kin * np.fft.fftn(psi))
    return psi


YOSHIDA_W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
YOSHIDA_W0 = -(2.0 ** (1.0 / 3.0)) / (2.0 - 2.0 ** (1.0 / 3.0))


def evolve(psi0, n, L, kernel, beta, gamma, dt, nsteps, order=2, V=None, pot=None, diag_every=0):
    """Time-splitting pseudospectral dynamics; returns (psi, diagnostics list of (mass, energy))."""
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in L)
    _, h = grid_axes(n, L)
    dv = np.prod(h)
    if pot is None:
        pot = DirectPotential(n, L, kernel)
    if V is None:
        V = harmonic_trap(n, L, gamma)
    k2 = freq_squared(n, L)
    psi = np.array(psi0, dtype=np.complex128).reshape(n)
    diags = []

    def diag(p):
        varphi = pot(np.abs(p) ** 2)
        st = energies(p, V, varphi, beta, n, L, kernel)
        return dv * np.sum(np.abs(p) ** 2), st["E"]

    if diag_every:
        diags.append(diag(psi))
    for s in range(1, nsteps + 1):
        if order == 2:
            psi = _strang(psi, dt, k2, V, beta, pot)
        elif order == 4:
            for w in (YOSHIDA_W1, YOSHIDA_W0, YOSHIDA_W1):
                psi = _strang(psi, w * dt, k2, V, beta, pot)
        else:
            raise ValueError("order must be 2 or 4")
        if diag_every and s % diag_every == 0:
            diags.append(diag(psi))
    return psi, diags
