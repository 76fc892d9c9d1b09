"""ORACLE (test infrastructure only) -- the spin chain of eq. (XXZ).

H = sum_{l=1,2} sum_{i=1..L} J_l (S^x_i S^x_{i+l} + S^y_i S^y_{i+l}
                                  + Delta S^z_i S^z_{i+l}) + sum_i h_i S^z_i

with periodic boundary conditions (paper, "Benchmark models").  The matrix is
taken in the S^z eigenbasis restricted to the zero-magnetisation sector, of
size C(L, L/2) (same paragraph).

Conventions (the paper fixes none; these are the readings used throughout):
* a basis state is an L-bit integer, bit i <-> site i+1, bit set <-> S^z=+1/2;
* basis order is ascending integer order;
* the bond sum is taken literally over i = 1..L with sites mod L, so for very
  small L a pair that appears twice is counted twice;
* the flip-flop part J(S^xS^x + S^yS^y) = (J/2)(S^+S^- + S^-S^+) gives the
  off-diagonal value +J/2 between states that differ by swapping an
  antiparallel pair (Supplement "Technical details": off-diagonals all equal
  to 1/2 at J=1), with no sign gauge.

Parity pins: basis and rank by brute force; CSR against a Kronecker-product
construction in the full 2^L space; trace closed form; free fermions.
"""

from math import comb

import numpy as np
import scipy.sparse as sp


def sector_dim(L):
    """C(L, L/2): size of the Sz=0 sector ("Benchmark models")."""
    return comb(L, L // 2)


def basis(L):
    """All L-bit integers with L/2 set bits, ascending, as uint32 (or uint64
    for L > 31).  Brute-force scan of 0 .. 2^L - 1."""
    dt = np.uint32 if L <= 31 else np.uint64
    x = np.arange(1 << L, dtype=dt)
    return x[np.bitwise_count(x) == L // 2]


def rank(states, basis_states):
    """Row index of each state in the ascending basis; -1 if absent."""
    states = np.asarray(states, dtype=basis_states.dtype)
    r = np.searchsorted(basis_states, states)
    r = np.minimum(r, len(basis_states) - 1)
    ok = basis_states[r] == states
    return np.where(ok, r, -1).astype(np.int64)


def _bonds(L):
    """(l, i, j) for every term of the literal double sum: l in {1,2},
    i = 0..L-1 (site i+1), j = (i+l) mod L."""
    return [(l, i, (i + l) % L) for l in (1, 2) for i in range(L)]


def diagonal(L, J1, J2, Delta, h, basis_states=None):
    """Diagonal of H in the Sz=0 basis, FP64:
    sum_l sum_i J_l Delta S^z_i S^z_{i+l} + sum_i h_i S^z_i."""
    b = basis(L) if basis_states is None else basis_states
    b = b.astype(np.int64)
    J = {1: J1, 2: J2}
    sz = [((b >> i) & 1).astype(np.float64) - 0.5 for i in range(L)]
    d = np.zeros(len(b))
    for l, i, j in _bonds(L):
        if J[l] != 0.0:
            d += J[l] * Delta * sz[i] * sz[j]
    for i in range(L):
        d += h[i] * sz[i]
    return d


def hamiltonian_csr(L, J1, J2, Delta, h):
    """H as a scipy CSR matrix (FP64), built by the literal sum of eq. (XXZ).
    Duplicate (row, col) entries are summed."""
    b = basis(L)
    bi = b.astype(np.int64)
    n = len(b)
    J = {1: J1, 2: J2}
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [diagonal(L, J1, J2, Delta, h, b)]
    for l, i, j in _bonds(L):
        if J[l] == 0.0:
            continue
        anti = ((bi >> i) & 1) != ((bi >> j) & 1)
        src = np.nonzero(anti)[0]
        flipped = bi[src] ^ ((1 << i) | (1 << j))
        dst = rank(flipped, b)
        assert (dst >= 0).all()
        # H[dst, src] = J_l / 2 : <s'| (J/2)(S+S- + S-S+) |s>
        rows.append(dst)
        cols.append(src)
        vals.append(np.full(len(src), 0.5 * J[l]))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    H.sum_duplicates()
    return H


def hamiltonian_row(L, J1, J2, Delta, h, s):
    """Row of H for one basis state s, by the literal sum of eq. (XXZ):
    returns {state': value} (the diagonal under s itself).  For sampled
    checks at sizes where the full CSR is too large."""
    s = int(s)
    J = {1: J1, 2: J2}
    out = {}
    d = 0.0
    for l, i, j in _bonds(L):
        if J[l] == 0.0:
            continue
        si, sj = (s >> i) & 1, (s >> j) & 1
        d += J[l] * Delta * (si - 0.5) * (sj - 0.5)
        if si != sj:
            t = s ^ ((1 << i) | (1 << j))
            out[t] = out.get(t, 0.0) + 0.5 * J[l]
    for i in range(L):
        d += h[i] * (((s >> i) & 1) - 0.5)
    out[s] = out.get(s, 0.0) + d
    return out
