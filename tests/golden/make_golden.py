"""Write the stored expected values under tests/golden/ using only the oracle.

    python tests/golden/make_golden.py

c2_j1j2_L18.json: the J1-J2 chain of the L=18 workload (J2=1, Delta=1,
W=2, seed 2): exact extremes (ARPACK), the target sigma_H at eps = 0.5, and
the 50 eigenvalues nearest it from the oracle's own FP64 POLFED solve
(oracle.lanczos.solve, pinned against dense diagonalisation at smaller L by
tests/test_oracle_pins.py), with the residual norms that certify them
(each eigenvalue lies within its residual of the spectrum of H).
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import chain, lanczos  # noqa: E402
from paper_2005_09534_amd import workloads  # noqa: E402


def c2():
    wl = workloads.c2()
    c = wl.chains[0]
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    E0, E1 = lanczos.extreme_eigenvalues(H)
    sigma = E0 + 0.5 * (E1 - E0)
    r = lanczos.solve(c.L, c.J1, c.J2, c.Delta, c.h, wl.nev, wl.block, sigma_H=sigma)
    return dict(workload=wl.name, L=c.L, J1=c.J1, J2=c.J2, Delta=c.Delta, h=list(c.h),
                E0=E0, E1=E1, sigma_H=sigma, nev=wl.nev, evals=list(map(float, r["E"])),
                resid=list(map(float, r["resid"])), K=int(r["K"]), m=int(r["m"]),
                source="oracle.lanczos.solve (FP64 POLFED, forward-recurrence filter)")


if __name__ == "__main__":
    out = os.path.join(HERE, "c2_j1j2_L18.json")
    data = c2()
    with open(out, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", out)
