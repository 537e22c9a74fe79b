"""The plain FFT passes of every line length the register-resident kernels take (64 to 512 points,
2D and 3D, with batches large enough that the short-column blocks fill the device), through the
time-splitting solver (libnlf.so, C-ABI) with beta = 0 and V = 0 (Sec. 4.1): each Strang step is
then the exact Fourier propagator exp(-i dt |mu|^2 / 2), which the oracle's split step applies with
numpy's FFT (`oracle.solvers.evolve`, potential switched off).

Bars: the relative max-norm error of 16 transforms (4 steps, two kinetic half steps each, a forward
and an inverse transform per half step) of length up to 2^9, about 16 x 9 rounding units: 1e-12 for
FP64 plans (u = 1.1e-16), 1e-5 for FP32 plans (u = 6e-8)."""
import numpy as np
import pytest

from oracle import solvers as so
from paper_1410_3584_amd import inputs
from gpu_util import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_3584_amd import nlf  # noqa: E402

BAR = {nlf.F64: 1e-12, nlf.F32: 1e-5}

# (grid, fields): rows and columns of 64 to 512 points; the batches put 256 or more column blocks
# on the device where a single field would not
CASES = [((64, 64), 1), ((128, 128), 32), ((256, 256), 8), ((512, 512), 4), ((64, 256), 1),
         ((64, 64, 64), 1), ((32, 64, 128), 1)]


@pytest.mark.parametrize("prec", [nlf.F64, nlf.F32])
@pytest.mark.parametrize("n,batch", CASES)
def test_free_evolution_is_the_fourier_propagator(n, batch, prec):
    print(f"[free evolution] n={n} batch={batch} prec={prec}", flush=True)
    L = tuple(8.0 for _ in n)
    kernel = nlf.COULOMB2D if len(n) == 2 else nlf.COULOMB3D
    gam = (1.0,) * len(n)
    dt, steps = 0.05, 4
    psi0 = [inputs.psi0_phase_modulated(n, L, seed=s) for s in range(batch)]
    plan = nlf.Plan(n, L, kernel, prec=prec, batch=batch)
    cdt = torch.complex128 if prec == nlf.F64 else torch.complex64
    psi = torch.tensor(np.stack(psi0), dtype=cdt, device="cuda")
    V = torch.zeros(int(np.prod(n)), dtype=torch.float64, device="cuda")
    plan.evolve(psi, 0.0, gam, dt, steps, V=V)
    got = psi.to(torch.complex128).cpu().numpy().reshape((batch,) + tuple(n))
    zero = np.zeros(tuple(n))
    for s in range(batch):
        want, _ = so.evolve(psi0[s], n, L, kernel, 0.0, gam, dt, steps, V=zero, pot=np.zeros_like)
        assert rel_err(got[s], want) <= BAR[prec], (s, rel_err(got[s], want))
