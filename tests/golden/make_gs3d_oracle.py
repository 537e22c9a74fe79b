"""Writes gs3d_oracle_h4.txt: the oracle's ground states of Table 'virial:3d:sps''s problem
(3D Coulomb kernel, V = (x^2 + y^2 + 4 z^2)/2, [-8,8]^3) for beta = -5 and 10 on a 64^3 grid
(h = 1/4), by the oracle's gradient flow (Sec. 3.1) with the oracle's split potential (Eq. '3.9'),
tau = 0.5, stopped at max|phi^{n+1} - phi^n| / tau <= 1e-10.  Calls only oracle/; takes about
ten minutes per beta on an 8-core host.

Usage (from the repository root): python tests/golden/make_gs3d_oracle.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import potential as op  # noqa: E402
from oracle import solvers as so  # noqa: E402
from oracle import split as sp  # noqa: E402

N, L, GAMMA, TAU, EPS0 = (64,) * 3, (8.0,) * 3, (1.0, 1.0, 2.0), 0.5, 1e-10
KEYS = ("E", "mu", "Ekin", "Epot", "Eint", "virial")


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gs3d_oracle_h4.txt")
    lines = ["# Oracle ground states of Table 'virial:3d:sps''s problem on 64^3 (h = 1/4) of [-8,8]^3,",
             "# V = (x^2+y^2+4z^2)/2, 3D Coulomb kernel by the oracle's split evaluation (Eq. '3.9'),",
             f"# gradient flow tau = {TAU}, stopped at residual <= {EPS0}; written by make_gs3d_oracle.py.",
             "# Columns: beta " + " ".join(KEYS) + " iters"]
    for beta in (-5.0, 10.0):
        t0 = time.time()
        _, st = so.ground_state(N, L, op.COULOMB3D, beta, GAMMA, tau=TAU, eps0=EPS0,
                                pot=lambda rho: sp.split_potential(rho, N, L))
        lines.append(f"{beta:g} " + " ".join(repr(float(st[k])) for k in KEYS) + f" {st['iters']}")
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
