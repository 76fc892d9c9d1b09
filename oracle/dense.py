"""ORACLE (test infrastructure only) -- the definition of the answer.

The result of a POLFED solve is, by the paper's own statement (main text,
end of "POLFED algorithm"), the N_ev eigenpairs of H whose eigenvalues lie
nearest the target.  This module computes exactly that set by library
diagonalisation:

* ``nearest_dense``   : full dense eigendecomposition (numpy.linalg.eigh);
  the paper puts the dense limit at N ~ 5e4 (L = 18).
* ``nearest_shift_invert`` : ARPACK in shift-invert mode around the target
  (sparse LU).  It is pinned against ``nearest_dense`` at L <= 14.
* ``eigenvalues_in_window`` / ``nearest_dense_window`` : dense LAPACK
  eigenvalues (``scipy.linalg.eigh`` with ``subset_by_value``) of the
  eigenvalues in an interval around the target; this is still the full
  dense reduction of H, only the tridiagonal eigenvalues outside the window
  are not computed.  This is the practical definition at L = 18
  (N = 48,620: 19 GB of FP64 and about 50 CPU-minutes on 8 cores).  Both
  are pinned against the free-fermion spectrum of the XX chain at L = 12.

Ties in distance go to the lower eigenvalue; output is ascending.
"""

import numpy as np
import scipy.linalg
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


def eigenvalues_in_window(H, lo, hi):
    """All eigenvalues of the symmetric H in the half-open interval (lo, hi],
    ascending, by dense LAPACK (syevr on the densified matrix)."""
    A = H.toarray(order="F") if hasattr(H, "toarray") else np.asfortranarray(H, dtype=np.float64)
    w = scipy.linalg.eigh(A, eigvals_only=True, subset_by_value=(lo, hi), driver="evr",
                          overwrite_a=True, check_finite=False)
    return np.sort(w)


def nearest_dense_window(H, sigma_H, nev, halfwidth):
    """The nev eigenvalues nearest sigma_H (ties -> lower), ascending, from the
    dense eigenvalues in (sigma_H - halfwidth, sigma_H + halfwidth].  Also
    returns the distance of the first eigenvalue left out, so a caller can
    check the answer is separated from the rest.  Raises if the window holds
    no more than nev eigenvalues (it must hold the first one left out too)."""
    w = eigenvalues_in_window(H, sigma_H - halfwidth, sigma_H + halfwidth)
    if len(w) <= nev:
        raise ValueError(f"window of half-width {halfwidth} holds {len(w)} <= {nev} eigenvalues")
    order = np.lexsort((w, np.abs(w - sigma_H)))
    keep = np.sort(w[order[:nev]])
    next_dist = float(np.abs(w[order[nev]] - sigma_H))
    return keep, next_dist, len(w)
