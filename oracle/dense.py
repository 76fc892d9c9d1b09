"""ORACLE (test infrastructure only) -- the definition of the answer.

The result of a POLFED solve is, by the paper's own statement (main text,
end of "POLFED algorithm"), the N_ev eigenpairs of H whose eigenvalues lie
nearest the target.  This module computes exactly that set by library
diagonalisation:

* ``nearest_dense``   : full dense eigendecomposition (numpy.linalg.eigh);
  the paper puts the dense limit at N ~ 5e4 (L = 18).
* ``nearest_shift_invert`` : ARPACK in shift-invert mode around the target
  (sparse LU); used where dense is too large (L = 18).  It is pinned against
  ``nearest_dense`` at L <= 14.

Ties in distance go to the lower eigenvalue; output is ascending.
"""

import numpy as np
import scipy.sparse.linalg as spla


def nearest_from_spectrum(w, sigma_H, nev):
    order = np.lexsort((w, np.abs(w - sigma_H)))[:nev]
    return np.sort(order)


def nearest_dense(H, sigma_H, nev, vectors=True):
    A = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    if vectors:
        w, V = np.linalg.eigh(A)
        idx = nearest_from_spectrum(w, sigma_H, nev)
        return w[idx], V[:, idx]
    w = np.linalg.eigvalsh(A)
    idx = nearest_from_spectrum(w, sigma_H, nev)
    return w[idx], None


def full_spectrum(H):
    A = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    return np.linalg.eigvalsh(A)


def nearest_shift_invert(H, sigma_H, nev, extra=10):
    """nev eigenvalues nearest sigma_H via ARPACK shift-invert (returns
    ascending eigenvalues and vectors).  Computes nev+extra and keeps the
    nearest nev, so a cluster cut by the boundary is resolved."""
    k = min(nev + extra, H.shape[0] - 2)
    w, V = spla.eigsh(H.tocsc(), k=k, sigma=sigma_H, which="LM", tol=1e-13)
    idx = nearest_from_spectrum(w, sigma_H, nev)
    return w[idx], V[:, idx]
