"""Write the stored expected values under tests/golden/ using only the oracle.

    python tests/golden/make_golden.py c2            # the L=18 J1-J2 workload
    python tests/golden/make_golden.py c4 R [R ...]  # members R of the batch

Each file holds the definition-layer answer: the N_ev eigenvalues of H
nearest the target (main text, end of "POLFED algorithm"), taken from the
dense LAPACK eigenvalues of H in a window around the target
(``oracle.dense.nearest_dense_window``), together with the distance of the
first eigenvalue left out.  The window's half-width comes from the Gaussian
density of states so that it holds about three times N_ev eigenvalues.

As a cross-check the oracle's own FP64 POLFED solve (``oracle.lanczos.solve``)
is run on the same chain and must agree with the dense values to 1e-10 ||H||
before anything is written; its values and residual norms are stored beside
the definition layer (``evals_polfed``, ``resid_polfed``).

At L = 18 one dense reduction is 19 GB of memory and about 50 CPU-minutes on
8 cores.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import chain, chebyshev, dense, lanczos  # noqa: E402
from paper_2005_09534_amd import workloads  # noqa: E402


def _definition_layer(c, nev, sigma, E0, E1, H):
    """N_ev nearest eigenvalues of H by dense windowed eigh."""
    n = H.shape[0]
    Ebar = float(H.diagonal().sum()) / n
    G = chebyshev.dos_gamma(c.L, c.J1, c.J2, c.Delta, c.h)
    rho = n / (np.sqrt(2 * np.pi) * G) * np.exp(-0.5 * ((sigma - Ebar) / G) ** 2)
    hw = 1.5 * nev / rho          # expected count 2 hw rho = 3 nev
    while True:
        try:
            return dense.nearest_dense_window(H, sigma, nev, hw) + (hw,)
        except ValueError:
            hw *= 2.0


def record(name, c, nev, s):
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    E0, E1 = lanczos.extreme_eigenvalues(H)
    sigma = E0 + 0.5 * (E1 - E0)
    normH = max(abs(E0), abs(E1))
    t0 = time.time()
    evals, next_dist, count, hw = _definition_layer(c, nev, sigma, E0, E1, H)
    t_dense = time.time() - t0
    print(f"{name}: dense window (half-width {hw:.4g}, {count} eigenvalues) in {t_dense:.0f} s",
          flush=True)
    t0 = time.time()
    r = lanczos.solve(c.L, c.J1, c.J2, c.Delta, c.h, nev, s, sigma_H=sigma)
    t_polfed = time.time() - t0
    err = float(np.abs(np.asarray(r["E"]) - evals).max()) / normH
    print(f"{name}: oracle POLFED in {t_polfed:.0f} s, max |diff| / ||H|| = {err:.2e}", flush=True)
    if not err <= 1e-10:
        raise SystemExit(f"{name}: oracle POLFED disagrees with the dense definition ({err:.2e})")
    last = float(np.abs(evals - sigma).max())
    return dict(workload=name, L=c.L, J1=c.J1, J2=c.J2, Delta=c.Delta, W=c.W, seed=c.seed,
                h=list(map(float, c.h)), E0=E0, E1=E1, normH=normH, sigma_H=sigma, nev=nev,
                evals=list(map(float, evals)), last_dist=last, next_dist=next_dist,
                window_halfwidth=hw, window_count=count,
                source="oracle.dense.nearest_dense_window (dense LAPACK syevr, subset by value)",
                evals_polfed=list(map(float, r["E"])), resid_polfed=list(map(float, r["resid"])),
                polfed_block=s, polfed_K=int(r["K"]), polfed_m=int(r["m"]),
                polfed_vs_dense=err, t_dense_s=round(t_dense, 1), t_polfed_s=round(t_polfed, 1))


def c2():
    wl = workloads.c2()
    return "c2_j1j2_L18.json", record(wl.name, wl.chains[0], wl.nev, wl.block)


def c4_member(R):
    wl = workloads.c4()
    c = wl.chains[R]
    return f"c4_member{R}_L{c.L}.json", record(f"{wl.name}[{R}]", c, wl.nev, 4)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    jobs = [c2] if which == "c2" else [lambda R=int(a): c4_member(R) for a in sys.argv[2:]]
    for job in jobs:
        fname, data = job()
        out = os.path.join(HERE, fname)
        with open(out, "w") as f:
            json.dump(data, f, indent=1)
        print("wrote", out, flush=True)
