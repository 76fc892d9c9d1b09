"""ORACLE (test infrastructure only) -- observables of the eigenpairs.

Main text, "Entanglement entropy and level statistics":

* the entanglement entropy of an eigenstate for the bipartition of the ring
  into the sites [x, x + L/2) and [x + L/2, x + L) (sites mod L) is
  S_E = -sum_i alpha_i^2 log(alpha_i^2) over its Schmidt coefficients
  alpha_i, averaged over the position x of the cut;
* the scaled entropy s_E = S_E / S_RMT(L), with the value of a chaotic chain
  in the zero-magnetisation sector S_RMT(L) = (L/2) ln 2 + (1/2 + ln(1/2))/2
  - 1/2;
* the gap ratio r_i = min(g_i, g_{i+1}) / max(g_i, g_{i+1}), g_i = E_{i+1} -
  E_i, averaged over the eigenvalues of those eigenstates.

Here a cut x is a bit offset: the first subsystem holds bits x .. x+L/2-1
(mod L) of the basis integer, i.e. sites x+1 .. x+L/2.  Cuts x and x + L/2
give the same bipartition, so the average runs over x = 0 .. L/2 - 1.

The Schmidt coefficients are the singular values of the coefficient matrix
psi[a][b] (a, b: the L/2-bit patterns of the two halves), taken here by
numpy.linalg.svd of the full 2^(L/2) x 2^(L/2) matrix.

Parity pins (tests/test_oracle_pins.py): zero for basis states, k ln 2 for k
singlets across the cut, SVD against the eigenvalues of the reduced density
matrix, a random state of the sector against S_RMT, and the Poisson and GOE
values of the gap ratio.
"""

import numpy as np

from . import chain


def cut_matrix(v, L, x, basis_states=None):
    """psi[a][b] of the vector v (length C(L, L/2), basis order) for the cut
    at bit x: a = bits x .. x+L/2-1, b = the other L/2 bits in ring order."""
    h = L // 2
    b = chain.basis(L) if basis_states is None else basis_states
    s = b.astype(np.int64)
    full = (1 << L) - 1
    t = ((s >> x) | (s << (L - x))) & full if x else s
    a_idx = t & ((1 << h) - 1)
    b_idx = t >> h
    psi = np.zeros((1 << h, 1 << (L - h)))
    psi[a_idx, b_idx] = np.asarray(v, dtype=np.float64)
    return psi


def entropy_from_schmidt(sv):
    """-sum p log p over p = sv^2 > 0."""
    p = np.asarray(sv, dtype=np.float64) ** 2
    p = p[p > 0.0]
    return float(-np.sum(p * np.log(p)))


def entanglement_entropy(v, L, x, basis_states=None):
    """S_E of v for the cut at bit x (natural logarithm)."""
    sv = np.linalg.svd(cut_matrix(v, L, x, basis_states), compute_uv=False)
    return entropy_from_schmidt(sv)


def entanglement_entropy_cut_average(v, L, basis_states=None):
    """S_E averaged over the L/2 distinct cut positions."""
    b = chain.basis(L) if basis_states is None else basis_states
    return float(np.mean([entanglement_entropy(v, L, x, b) for x in range(L // 2)]))


def s_rmt(L):
    """S_RMT(L) = (L/2) ln 2 + (1/2 + ln(1/2))/2 - 1/2."""
    return (L / 2) * np.log(2.0) + (0.5 + np.log(0.5)) / 2.0 - 0.5


def gap_ratios(E):
    """r_i = min(g_i, g_{i+1}) / max(g_i, g_{i+1}) of the sorted levels."""
    E = np.sort(np.asarray(E, dtype=np.float64))
    g = np.diff(E)
    lo = np.minimum(g[:-1], g[1:])
    hi = np.maximum(g[:-1], g[1:])
    return lo / hi


def mean_gap_ratio(E):
    return float(np.mean(gap_ratios(E)))
