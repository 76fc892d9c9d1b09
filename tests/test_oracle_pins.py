"""Pins of the CPU oracle against things other than itself.

Each test names what it pins.  Nothing here needs a GPU.
"""

import itertools
from math import comb, pi, sqrt

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize
import scipy.sparse as sps

from oracle import chain, chebyshev, dense, lanczos
from paper_2005_09534_amd import workloads


# ---------------------------------------------------------------------------
# basis and rank: brute force, combinatorics
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("L", [2, 4, 6, 8, 10, 12, 14, 16])
def test_basis_matches_combinations(L):
    """Sz=0 basis = all L/2-subsets of the L sites, as ascending integers."""
    b = chain.basis(L)
    ref = sorted(sum(1 << i for i in c) for c in itertools.combinations(range(L), L // 2))
    assert len(b) == comb(L, L // 2) == chain.sector_dim(L)
    assert b.tolist() == ref
    assert b[0] == (1 << (L // 2)) - 1
    assert b[-1] == ((1 << (L // 2)) - 1) << (L // 2)


@pytest.mark.parametrize("L", [4, 10, 16, 20])
def test_rank_is_colex_combinadic(L):
    """rank(s) = sum_t C(p_t, t) over set bits p_1 < p_2 < ... (t from 1):
    the colexicographic rank, which is the ascending-integer order."""
    b = chain.basis(L)
    rng = np.random.default_rng(L)
    pick = rng.choice(len(b), size=min(len(b), 500), replace=False)
    r = chain.rank(b[pick], b)
    for row, st in zip(pick, b[pick]):
        bits = [i for i in range(L) if (int(st) >> i) & 1]
        assert sum(comb(p, t + 1) for t, p in enumerate(bits)) == row
    assert (r == pick).all()
    # states outside the sector are reported absent
    bad = np.array([0, (1 << L) - 1, 1], dtype=b.dtype)
    assert (chain.rank(bad, b) == -1).all()


# ---------------------------------------------------------------------------
# H: Kronecker-product construction in the full 2^L space
# ---------------------------------------------------------------------------

def _kron_site(op, i, L):
    """Operator op on the site carried by bit i of the basis integer."""
    return sps.kron(sps.kron(sps.identity(1 << (L - 1 - i)), sps.csr_matrix(op)),
                    sps.identity(1 << i)).tocsr()


def _full_H(L, J1, J2, Delta, h):
    # single-site basis ordered (bit 0 = down, bit 1 = up)
    sx = 0.5 * np.array([[0, 1], [1, 0]], dtype=complex)
    sy = 0.5 * np.array([[0, -1j], [1j, 0]], dtype=complex)
    sz = 0.5 * np.array([[-1, 0], [0, 1]], dtype=complex)
    n = 1 << L
    H = sps.csr_matrix((n, n), dtype=complex)
    S = {a: [_kron_site(op, i, L) for i in range(L)] for a, op in (("x", sx), ("y", sy), ("z", sz))}
    for l, J in ((1, J1), (2, J2)):
        for i in range(L):
            j = (i + l) % L
            H = H + J * (S["x"][i] @ S["x"][j] + S["y"][i] @ S["y"][j] + Delta * S["z"][i] @ S["z"][j])
    for i in range(L):
        H = H + h[i] * S["z"][i]
    Sz = sum(S["z"])
    comm = abs(H @ Sz - Sz @ H).max()
    H = H.toarray()
    assert np.abs(H.imag).max() < 1e-15
    return H.real, comm


@pytest.mark.parametrize("L,J2", [(4, 0.0), (6, 0.0), (6, 1.0), (8, 0.7), (10, 1.0)])
def test_csr_matches_kronecker(L, J2):
    """Sz=0 block of the full-space H equals the oracle's CSR; Sz is
    conserved; H is exactly symmetric."""
    rng = np.random.default_rng(100 + L)
    Delta = float(rng.uniform(0.2, 1.5))
    h = rng.uniform(-3, 3, L)
    Hf, comm = _full_H(L, 1.0, J2, Delta, h)
    assert comm < 1e-13
    b = chain.basis(L).astype(np.int64)
    Hs = chain.hamiltonian_csr(L, 1.0, J2, Delta, h)
    assert np.abs(Hs.toarray() - Hf[np.ix_(b, b)]).max() < 1e-13
    assert (Hs != Hs.T).nnz == 0


@pytest.mark.parametrize("L,J2,Delta,expect", [(8, 0.0, 0.7, -14.0), (8, 1.0, 0.7, -28.0),
                                               (10, 1.0, 0.7, -98.0), (12, 0.0, 1.0, None),
                                               (14, 1.0, 0.55, None)])
def test_trace_closed_form(L, J2, Delta, expect):
    """Tr H = -N (J1+J2) Delta L / (4(L-1)): in Sz=0 every pair of distinct
    sites has <Sz_i Sz_j> = -1/(4(L-1)), and sum_r Sz_i = 0, so h drops out."""
    h = np.random.default_rng(L).uniform(-5, 5, L)
    N = comb(L, L // 2)
    tr = float(chain.diagonal(L, 1.0, J2, Delta, h).sum())
    closed = -N * (1.0 + J2) * Delta * L / (4.0 * (L - 1))
    assert abs(tr - closed) < 1e-9 * max(1.0, abs(closed))
    if expect is not None:
        assert abs(closed - expect) < 1e-12


def _free_fermion_spectrum(L, J1=1.0):
    """XX chain (Delta = 0, J2 = 0, h = 0) in the Sz=0 sector by
    Jordan-Wigner: L/2 fermions, single-particle energies J1 cos k with
    k = 2 pi (n + phi)/L, phi = 0 if L/2 is odd (periodic), 1/2 if L/2 is
    even (antiperiodic, the boundary bond picks up (-1)^(N_f - 1))."""
    Nf = L // 2
    phi = 0.0 if Nf % 2 == 1 else 0.5
    eps = J1 * np.cos(2 * pi * (np.arange(L) + phi) / L)
    return np.sort([eps[list(c)].sum() for c in itertools.combinations(range(L), Nf)])


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12])
def test_xx_chain_free_fermions(L):
    H = chain.hamiltonian_csr(L, 1.0, 0.0, 0.0, np.zeros(L))
    w = dense.full_spectrum(H)
    ff = _free_fermion_spectrum(L)
    assert np.abs(w - ff).max() < 1e-12
    if L == 4:
        assert np.allclose(w, [-sqrt(2), 0, 0, 0, 0, sqrt(2)], atol=1e-14)


def test_diagonal_special_case():
    """J1 = J2 = 0: H is diagonal with E_r = sum_i h_i (n_i - 1/2)."""
    L = 10
    h = np.random.default_rng(5).uniform(-2, 2, L)
    b = chain.basis(L).astype(np.int64)
    E = np.array([sum(h[i] * (((s >> i) & 1) - 0.5) for i in range(L)) for s in b])
    H = chain.hamiltonian_csr(L, 0.0, 0.0, 1.0, h)
    assert H.nnz == len(b)
    assert np.abs(H.diagonal() - E).max() < 1e-13


# ---------------------------------------------------------------------------
# the filter: Dirichlet-kernel closed form, eigenvector action
# ---------------------------------------------------------------------------

def _dirichlet(u, K):
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    small = np.abs(np.sin(u / 2)) < 1e-12
    out[small] = 2 * K + 1
    out[~small] = np.sin((K + 0.5) * u[~small]) / np.sin(u[~small] / 2)
    return out


def _P_closed(x, sigma, K):
    """P_K(cos th) = [D_K(th - a) + D_K(th + a)] / [D_K(0) + D_K(2a)],
    sigma = cos a, D_K(u) = sin((K+1/2)u)/sin(u/2): since
    1 + 2 sum_{n<=K} cos(n a) cos(n th) = (D_K(th-a) + D_K(th+a))/2."""
    a = np.arccos(sigma)
    th = np.arccos(np.asarray(x, dtype=np.float64))
    return (_dirichlet(th - a, K) + _dirichlet(th + a, K)) / (_dirichlet(np.array([0.0]), K) + _dirichlet(np.array([2 * a]), K))


@pytest.mark.parametrize("K", [1, 2, 22, 23, 200])
@pytest.mark.parametrize("sigma", [0.0, 0.3, -0.71])
def test_filter_closed_form(K, sigma):
    x = np.linspace(-0.999, 0.999, 301)
    assert np.abs(chebyshev.P_of_x(x, sigma, K) - _P_closed(x, sigma, K)).max() < 1e-12
    assert abs(chebyshev.P_of_x([sigma], sigma, K)[0] - 1.0) < 1e-13


@pytest.mark.parametrize("K", [21, 22, 200, 201])
def test_norm_D_at_centre(K):
    """At sigma = 0: D = K + 1 for even K, K for odd K."""
    assert abs(chebyshev.norm_D(0.0, K) - (K + 1 if K % 2 == 0 else K)) < 1e-9


def test_side_lobes_below_p():
    """The threshold p = 0.17 sits above every side lobe of P (largest
    positive lobe ~0.128 at large K); side lobes dip to about -0.217."""
    K = 400
    x = np.cos(np.linspace(0, pi, 200001))
    P = _P_closed(x, 0.0, K)
    main = np.abs(np.arccos(x) - pi / 2) < 2 * pi / (2 * K + 1)
    assert P[~main].max() < 0.17
    assert 0.12 < P[~main].max() < 0.135
    assert -0.225 < P.min() < -0.21


@pytest.mark.parametrize("K,sigma", [(0, 0.0), (1, 0.2), (7, 0.0), (60, 0.35), (151, -0.1)])
def test_filter_acts_on_eigenvectors(K, sigma):
    """P(H~) v = P(lambda~) v for every eigenvector v of H; pins the forward
    recurrence (incl. the rescale) against the scalar closed form."""
    L = 8
    h = np.random.default_rng(3).uniform(-2, 2, L)
    H = chain.hamiltonian_csr(L, 1.0, 0.5, 0.8, h)
    w, V = np.linalg.eigh(H.toarray())
    E0, E1 = lanczos.widened_bounds(w[0], w[-1], 1e-3)
    a, b = chebyshev.rescale_coeffs(E0, E1)
    Y = chebyshev.filter_block(H, V, E0, E1, sigma, K)
    Pw = _P_closed(a * w + b, sigma, K) if K > 0 else np.ones_like(w)
    assert np.abs(Y - V * Pw).max() < 1e-12


# ---------------------------------------------------------------------------
# density of states and the order rule
# ---------------------------------------------------------------------------

def test_gamma_is_infinite_temperature_width():
    """Gamma^2 = Tr(H^2)/2^L - (Tr H/2^L)^2 exactly in the full space for
    L >= 5 (all bonds distinct): each bond adds J^2 (2 + Delta^2)/16, each
    field h_i^2/4.  And at J1 = 1 with sum h^2 = L W^2/3 it equals the
    paper's Gamma = sqrt(L[(1+J2^2)/8 + Delta^2 (1+J2^2)/16 + W^2/12])."""
    L, J2, Delta = 8, 0.6, 0.8
    h = np.random.default_rng(9).uniform(-3, 3, L)
    Hf, _ = _full_H(L, 1.0, J2, Delta, h)
    n = Hf.shape[0]
    var = np.trace(Hf @ Hf) / n - (np.trace(Hf) / n) ** 2
    assert abs(chebyshev.dos_gamma(L, 1.0, J2, Delta, h) ** 2 - var) < 1e-12
    W = 2.5
    hW = np.full(L, W / sqrt(3.0))
    paper = sqrt(L * ((1 + J2 ** 2) / 8 + Delta ** 2 * (1 + J2 ** 2) / 16 + W ** 2 / 12))
    assert abs(chebyshev.dos_gamma(L, 1.0, J2, Delta, hW) - paper) < 1e-12


def test_n_states_between_is_integral_of_rho():
    N, Ebar, G, E0, E1 = 12870, -0.3, 3.1, -14.0, 13.0
    x_lo, x_hi = -0.05, 0.08
    num, _ = scipy.integrate.quad(lambda x: chebyshev.rho_tilde(x, N, Ebar, G, E0, E1), x_lo, x_hi,
                                  epsabs=1e-12, epsrel=1e-12)
    Elo = 0.5 * (x_lo * (E1 - E0) + E1 + E0)
    Ehi = 0.5 * (x_hi * (E1 - E0) + E1 + E0)
    assert abs(chebyshev.n_states_between(N, Ebar, G, Elo, Ehi) - num) < 1e-8 * num
    # total mass: all N states
    assert abs(chebyshev.n_states_between(N, Ebar, G, -1e3, 1e3) - N) < 1e-6


@pytest.mark.parametrize("K,sigma", [(50, 0.0), (333, 0.25), (2000, -0.4)])
def test_lobe_edges_hit_p(K, sigma):
    lo, hi = chebyshev.lobe_edges(sigma, K, 0.17)
    assert lo < sigma < hi
    assert abs(_P_closed([lo], sigma, K)[0] - 0.17) < 1e-9
    assert abs(_P_closed([hi], sigma, K)[0] - 0.17) < 1e-9
    # half-width against the asymptotic u*/(K+1/2) sin(alpha), sin(u*)/u* = 0.17
    ustar = scipy.optimize.brentq(lambda u: np.sin(u) / u - 0.17, 2.0, 3.0)
    assert abs(ustar - 2.6704) < 1e-3
    approx = ustar / (K + 0.5) * sqrt(1 - sigma ** 2)
    assert abs(0.5 * (hi - lo) - approx) < 0.02 * approx


def test_choose_K_asymptotics_and_scaling():
    """K ~ 2 u* rho~(sigma) sqrt(1-sigma^2) / N_ev - 1/2 at large K, and
    N_ev -> a N_ev gives K -> K/a (Supplement, "Benchmark")."""
    N, Ebar, G, E0, E1 = 705432, -2.6, 7.5, -29.0, 27.0
    sigma = 0.0
    rho = chebyshev.rho_tilde(sigma, N, Ebar, G, E0, E1)
    ustar = 2.67040
    for nev in (100, 400):
        K = chebyshev.choose_K(nev, sigma, 0.17, N, Ebar, G, E0, E1)
        approx = 2 * ustar * rho / nev - 0.5
        assert abs(K - approx) < 0.01 * approx
        f = lambda k: chebyshev.n_P(k, sigma, 0.17, N, Ebar, G, E0, E1)
        assert f(K) >= nev > f(K + 1)
    K1 = chebyshev.choose_K(100, sigma, 0.17, N, Ebar, G, E0, E1)
    K2 = chebyshev.choose_K(200, sigma, 0.17, N, Ebar, G, E0, E1)
    assert abs(K2 / K1 - 0.5) < 0.01


# ---------------------------------------------------------------------------
# the solve: dense diagonalisation, invariants, special cases
# ---------------------------------------------------------------------------

def _dense_check(L, J1, J2, Delta, h, nev, s, K=None, seed=0):
    res = lanczos.solve(L, J1, J2, Delta, h, nev, s, K=K, rng_seed=seed)
    H = chain.hamiltonian_csr(L, J1, J2, Delta, h)
    Ed, Vd = dense.nearest_dense(H, res["sigma_H"], nev)
    normH = max(abs(res["E0"]), abs(res["E1"]))
    return res, H, Ed, Vd, normH


def test_solve_c1_vs_dense():
    """The C1 workload (L=12 XXZ, W=3, N_ev=20, s=4, K=200): eigenvalues
    equal the 20 nearest the middle of the spectrum (main text claim)."""
    wl = workloads.c1()
    c = wl.chains[0]
    res, H, Ed, Vd, normH = _dense_check(c.L, c.J1, c.J2, c.Delta, c.h, wl.nev, wl.block, K=wl.K)
    assert res["nconv"] >= wl.nev
    assert np.abs(res["E"] - Ed).max() <= 1e-10 * normH
    assert res["resid"].max() <= 1e-8 * normH
    # eigenvectors: |<u, v>| = 1 up to the Davis-Kahan bound
    ov = np.abs(np.sum(res["V"] * Vd, axis=0))
    w = dense.full_spectrum(H)
    gaps = np.array([np.min(np.abs(np.delete(w, np.argmin(np.abs(w - e))) - e)) for e in Ed])
    assert (1 - ov <= (res["resid"] / gaps) ** 2 + 1e-10).all()


@pytest.mark.parametrize("L,J2,Delta,W,nev,s", [(10, 0.0, 1.0, 2.0, 10, 2), (12, 1.0, 0.55, 4.0, 16, 4),
                                                 (12, 0.0, 1.0, 1.0, 12, 1), (10, 1.0, 1.0, 6.0, 8, 8)])
def test_solve_auto_K_vs_dense(L, J2, Delta, W, nev, s):
    h = workloads.fields(L, W, 40 + L)
    res, H, Ed, Vd, normH = _dense_check(L, 1.0, J2, Delta, h, nev, s)
    assert np.abs(res["E"] - Ed).max() <= 1e-10 * normH
    assert res["resid"].max() <= 1e-8 * normH


def test_solve_widens_a_window_the_dos_made_too_narrow():
    """A short, strongly disordered chain (L = 14, W = 5, a realisation of the
    512-member batch) whose Gaussian-DOS order leaves only 18 eigenvalues
    with P >= p for N_ev = 20: the solve repeats with the window sized for
    twice as many eigenvalues and then returns exactly the 20 eigenvalues
    nearest the target; a chain whose window is wide enough keeps it."""
    c = workloads.chain(14, 5.0, 1207)
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    w = dense.full_spectrum(H)
    normH = max(abs(w[0]), abs(w[-1]))
    # the window of the first attempt, counted on the exact spectrum
    E0w, E1w = lanczos.widened_bounds(w[0], w[-1], 1e-3)
    a, b = chebyshev.rescale_coeffs(E0w, E1w)
    sig_t = a * (w[0] + 0.5 * (w[-1] - w[0])) + b
    K1 = chebyshev.choose_K(lanczos.window_count(20), sig_t, 0.17, H.shape[0],
                            float(H.diagonal().sum()) / H.shape[0],
                            chebyshev.dos_gamma(c.L, c.J1, c.J2, c.Delta, c.h), E0w, E1w)
    assert int((chebyshev.P_of_x(a * w + b, sig_t, K1) >= 0.17).sum()) < 20
    res = lanczos.solve(c.L, c.J1, c.J2, c.Delta, c.h, 20, 8)
    assert res["window_factor"] == 3.0 and res["K"] < K1
    Ed = w[dense.nearest_from_spectrum(w, res["sigma_H"], 20)]
    assert np.abs(res["E"] - Ed).max() <= 1e-10 * normH
    assert res["resid"].max() <= 1e-8 * normH
    ok = workloads.chain(14, 2.0, 1003)
    assert lanczos.solve(ok.L, ok.J1, ok.J2, ok.Delta, ok.h, 20, 8)["window_factor"] == 1.5


def test_lanczos_invariants():
    """Q^T Q = I, T symmetric, theta <= 1, converged theta = P(lambda~)."""
    L, nev, s = 12, 12, 4
    h = workloads.fields(L, 3.0, 11)
    res = lanczos.solve(L, 1.0, 0.0, 1.0, h, nev, s)
    Q, T = res["Qm"], res["T"]
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 1e-13
    assert np.abs(T - T.T).max() == 0.0
    assert res["theta"].max() <= 1.0 + 1e-12
    H = chain.hamiltonian_csr(L, 1.0, 0.0, 1.0, h)
    a, b = chebyshev.rescale_coeffs(res["E0w"], res["E1w"])
    th = _P_closed(a * res["E"] + b, res["sigma_t"], res["K"])
    top = np.sort(res["theta"])[::-1][:nev]
    assert np.abs(np.sort(th)[::-1] - top).max() < 1e-8


def test_solve_diagonal_case_is_a_sort():
    """J1 = J2 = 0: the answer is the N_ev basis states with E nearest the
    target, and the eigenvectors are unit vectors."""
    L, nev = 10, 8
    h = workloads.fields(L, 2.0, 77)
    b = chain.basis(L).astype(np.int64)
    E = np.array([sum(h[i] * (((st >> i) & 1) - 0.5) for i in range(L)) for st in b])
    sigma = 0.5 * (E.min() + E.max())
    res = lanczos.solve(L, 0.0, 0.0, 1.0, h, nev, 2, sigma_H=sigma)
    idx = np.lexsort((E, np.abs(E - sigma)))[:nev]
    assert np.abs(np.sort(E[idx]) - res["E"]).max() < 1e-10
    V = np.abs(res["V"])
    assert np.abs(V.max(axis=0) - 1.0).max() < 1e-8


def test_convergence_within_paper_cap_s1():
    """s = 1 with the paper's own rule (window of N_ev, 2.8 N_ev cap):
    converges with m < 2.8 N_ev (Supplement, "Convergence of POLFED")."""
    L, nev = 12, 20
    h = workloads.fields(L, 3.0, 7)
    res = lanczos.solve(L, 1.0, 0.0, 1.0, h, nev, 1, nev_window=nev, max_cols=int(2.8 * nev))
    assert res["nconv"] >= nev
    assert res["m"] < 2.8 * nev


def test_shift_invert_matches_dense():
    L = 12
    h = workloads.fields(L, 2.0, 3)
    H = chain.hamiltonian_csr(L, 1.0, 1.0, 1.0, h)
    w = dense.full_spectrum(H)
    sig = 0.5 * (w[0] + w[-1])
    a, _ = dense.nearest_dense(H, sig, 30, vectors=False)
    b, V = dense.nearest_shift_invert(H, sig, 30)
    assert np.abs(a - b).max() < 1e-10
    assert np.abs(H @ V - V * b).max() < 1e-9


def test_window_eigenvalues_against_free_fermions():
    """eigenvalues_in_window and nearest_dense_window (the definition at the
    sizes where only a window of the dense spectrum is taken) on the L = 12
    XX chain, whose whole spectrum is the free-fermion sums: the window holds
    exactly the sums in (lo, hi], and the nearest set, its size and the gap to
    the first value left out follow from a plain sort of those sums."""
    L = 12
    H = chain.hamiltonian_csr(L, 1.0, 0.0, 0.0, np.zeros(L))
    ff = _free_fermion_spectrum(L)
    # centres between levels (and one on a degenerate level, where ties go
    # to the lower value and every copy of it is kept or dropped together)
    for sig, hw, nev in [(0.37, 0.9, 25), (-1.21, 0.6, 7), (0.0, 0.5, 40)]:
        lo, hi = sig - hw, sig + hw
        want = ff[(ff > lo + 1e-9) & (ff <= hi - 1e-9)]
        got = dense.eigenvalues_in_window(H, lo, hi)
        assert len(got) == len(want) and np.abs(got - want).max() < 1e-12
        keep, nd, cnt = dense.nearest_dense_window(H, sig, nev, hw)
        assert cnt == len(want)
        d = sorted(want, key=lambda e: (abs(e - sig), e))
        assert np.abs(keep - np.sort(d[:nev])).max() < 1e-12
        assert abs(nd - abs(d[nev] - sig)) < 1e-12
    with pytest.raises(ValueError):
        dense.nearest_dense_window(H, 0.37, 10, 0.01)


def test_seed_and_block_invariance():
    L, nev = 12, 10
    h = workloads.fields(L, 2.5, 21)
    r1 = lanczos.solve(L, 1.0, 0.0, 1.0, h, nev, 2, rng_seed=1)
    r2 = lanczos.solve(L, 1.0, 0.0, 1.0, h, nev, 4, rng_seed=2)
    assert np.abs(r1["E"] - r2["E"]).max() < 1e-10 * max(abs(r1["E0"]), abs(r1["E1"]))


def test_hamiltonian_row_matches_csr():
    """The per-row form used for sampled checks at large L equals the CSR."""
    L = 10
    h = np.random.default_rng(2).uniform(-1, 1, L)
    H = chain.hamiltonian_csr(L, 1.0, 0.6, 0.9, h).tocsr()
    b = chain.basis(L)
    for r in (0, 7, 100, len(b) - 1):
        row = chain.hamiltonian_row(L, 1.0, 0.6, 0.9, h, b[r])
        dense_row = np.zeros(len(b))
        for st, v in row.items():
            dense_row[chain.rank([st], b)[0]] += v
        assert np.abs(dense_row - H.getrow(r).toarray().ravel()).max() < 1e-14


def test_capped_window_definition_and_law():
    """oracle.chebyshev.capped_window: the order fits the cap and one window
    fewer does not (its definition, checked with choose_K), and the window
    follows the paper's K ~ 1/N_win law (Supplement, "Benchmark": N_ev ->
    a N_ev gives K -> K/a) to within 15%."""
    L = 14
    c = workloads.chain(L, 2.0, 5)
    N = comb(L, L // 2)
    E0w, E1w = -0.9 * L, 0.85 * L
    Ebar = -(c.J1 + c.J2) * c.Delta * L / (4.0 * (L - 1))
    G = chebyshev.dos_gamma(L, c.J1, c.J2, c.Delta, c.h)
    nwin = 20
    K0 = chebyshev.choose_K(nwin, 0.0, 0.17, N, Ebar, G, E0w, E1w)
    for alpha in (2.0, 3.0):
        cap = int(K0 / alpha)
        w, K = chebyshev.capped_window(nwin, 0.0, 0.17, N, Ebar, G, E0w, E1w, cap)
        assert K <= cap < chebyshev.choose_K(w - 1, 0.0, 0.17, N, Ebar, G, E0w, E1w)
        assert abs(w / (alpha * nwin) - 1.0) < 0.15, (alpha, w)
    # a cap above the order leaves the window alone
    assert chebyshev.capped_window(nwin, 0.0, 0.17, N, Ebar, G, E0w, E1w, K0) == (nwin, K0)


def test_sign_normalise_conventions():
    """oracle.lanczos.sign_normalise: the entry of largest magnitude becomes
    positive, and among entries of equal magnitude the lowest index decides
    (the output convention of the eigenvectors).  Expected values written
    out by hand."""
    V = np.array([[0.5, -0.6, 0.3, 0.0],
                  [-0.8, 0.6, -0.3, -0.0],
                  [0.1, 0.2, 0.3, 0.0]])
    out = lanczos.sign_normalise(V)
    expect = np.array([[-0.5, 0.6, 0.3, 0.0],
                       [0.8, -0.6, -0.3, 0.0],
                       [-0.1, -0.2, 0.3, 0.0]])
    assert np.array_equal(out, expect)
    # a tie where the lowest index is the negative one flips the column
    W = np.array([[-0.7], [0.7], [0.1]])
    assert np.array_equal(lanczos.sign_normalise(W), np.array([[0.7], [-0.7], [-0.1]]))


def test_extreme_eigenvalues_sparse_branch_vs_dense():
    """oracle.lanczos.extreme_eigenvalues takes the ARPACK branch above 2000
    rows (L = 14: 3,432); both extremes equal the dense eigvalsh ones to
    1e-12 of ||H||."""
    c = workloads.chain(14, 3.0, 77, J2=0.4, Delta=0.8)
    H = chain.hamiltonian_csr(14, c.J1, c.J2, c.Delta, c.h)
    assert H.shape[0] > 2000
    lo, hi = lanczos.extreme_eigenvalues(H)
    w = np.linalg.eigvalsh(H.toarray())
    normH = max(abs(w[0]), abs(w[-1]))
    assert abs(lo - w[0]) <= 1e-12 * normH and abs(hi - w[-1]) <= 1e-12 * normH


# ---------------------------------------------------------------------------
# observables: entanglement entropy and gap ratio (main text, "Entanglement
# entropy and level statistics")
# ---------------------------------------------------------------------------

from oracle import observables  # noqa: E402


def test_entropy_of_basis_states_is_zero():
    L = 10
    b = chain.basis(L)
    for r in (0, 17, len(b) - 1):
        v = np.zeros(len(b))
        v[r] = 1.0
        for x in range(L // 2):
            assert observables.entanglement_entropy(v, L, x, b) == 0.0


def test_entropy_of_singlets_across_the_cut():
    """L = 8, a singlet on each of the bit pairs (0,1), (2,3), (4,5), (6,7):
    the cut at bit x splits 0 (x even) or 2 (x odd) singlets, so S_E = 0 or
    2 ln 2, and the cut average is ln 2 (closed form)."""
    L = 8
    b = chain.basis(L)
    v = np.zeros(len(b))
    for pattern in itertools.product((0, 1), repeat=4):   # which site of each pair is up
        s, sign = 0, 1.0
        for k, up_second in enumerate(pattern):
            s |= 1 << (2 * k + up_second)
            sign *= -1.0 if up_second else 1.0
        v[chain.rank([s], b)[0]] = sign / 4.0
    assert abs(np.linalg.norm(v) - 1.0) < 1e-15
    for x in range(L // 2):
        expect = 0.0 if x % 2 == 0 else 2.0 * np.log(2.0)
        assert abs(observables.entanglement_entropy(v, L, x, b) - expect) < 1e-13
    assert abs(observables.entanglement_entropy_cut_average(v, L, b) - np.log(2.0)) < 1e-13


def test_entropy_svd_equals_reduced_density_matrix():
    """Schmidt coefficients by SVD against the eigenvalues of the reduced
    density matrix rho_A = psi psi^T (two library routes)."""
    L = 10
    b = chain.basis(L)
    v = np.random.default_rng(3).standard_normal(len(b))
    v /= np.linalg.norm(v)
    for x in range(L // 2):
        psi = observables.cut_matrix(v, L, x, b)
        lam = np.linalg.eigvalsh(psi @ psi.T)
        lam = lam[lam > 1e-300]
        assert abs(observables.entanglement_entropy(v, L, x, b) + np.sum(lam * np.log(lam))) < 1e-12


def test_random_state_entropy_near_s_rmt():
    """A random state of the zero-magnetisation sector has the entropy of a
    chaotic chain: within 0.01 of S_RMT(14) = 7 ln 2 + (1/2 + ln 1/2)/2 -
    1/2 (dropping either correction term would miss by 0.1 or 0.5)."""
    L = 14
    b = chain.basis(L)
    v = np.random.default_rng(14).standard_normal(len(b))
    v /= np.linalg.norm(v)
    s = observables.entanglement_entropy_cut_average(v, L, b)
    assert abs(s - observables.s_rmt(L)) < 0.01
    assert abs(observables.s_rmt(14) - (7 * np.log(2) + (0.5 + np.log(0.5)) / 2 - 0.5)) < 1e-15


def test_gap_ratio_poisson_and_goe():
    """Mean gap ratio of uncorrelated levels: 2 ln 2 - 1 = 0.3863; of a GOE
    matrix (middle of its spectrum): 0.5307 (Atas et al., PRL 110, 084101
    (2013)).  Sampling errors here are about 0.001 and 0.006."""
    rng = np.random.default_rng(5)
    E = np.cumsum(rng.exponential(size=100000))
    assert abs(observables.mean_gap_ratio(E) - (2 * np.log(2) - 1)) < 0.01
    A = rng.standard_normal((3000, 3000))
    w = np.linalg.eigvalsh((A + A.T) / 2)
    assert abs(observables.mean_gap_ratio(w[750:2250]) - 0.5307) < 0.02
    r = observables.gap_ratios([0.0, 1.0, 3.0, 3.5])
    assert np.allclose(r, [0.5, 0.25])


# ---------------------------------------------------------------------------
# kernel polynomial density of states: trace identity, Jackson's kernel,
# closed-form measures, brute-force order rule
# ---------------------------------------------------------------------------

from oracle import kpm  # noqa: E402


def _chain_spectrum(L, W, seed, J2=0.0, Delta=1.0):
    c = workloads.chain(L, W, seed, J2=J2, Delta=Delta)
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    w = dense.full_spectrum(H)
    E0w, E1w = lanczos.widened_bounds(w[0], w[-1], 1e-3)
    a, b = chebyshev.rescale_coeffs(E0w, E1w)
    return H, w, a, b


@pytest.mark.parametrize("L,J2", [(8, 0.0), (10, 1.0)])
def test_kpm_stochastic_moments_over_a_basis_are_the_trace(L, J2):
    """Summed over the columns of any orthonormal basis (the unit vectors, or
    a random orthogonal matrix), sum_r <r|T_n(H~)|r> = Tr T_n(H~) = sum_i
    T_n(x_i) over the eigenvalues: the recurrence route against dense
    diagonalisation."""
    H, w, a, b = _chain_spectrum(L, 3.0, 5, J2=J2)
    N = H.shape[0]
    M = 41
    ref = kpm.moments_exact(w, a, b, M)
    assert ref[0] == 1.0
    assert np.abs(kpm.moments_stochastic(H, a, b, np.eye(N), M) - ref).max() < 1e-12
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((N, N)))
    assert np.abs(kpm.moments_stochastic(H.toarray(), a, b, Q, M) - ref).max() < 1e-12
    # a single eigenvector gives the moments of one level: T_n(x_i)
    ev = np.linalg.eigh(H.toarray())[1][:, 7]
    x7 = a * w[7] + b
    mu1 = kpm.moments_stochastic(H, a, b, 3.0 * ev, M)
    assert np.abs(mu1 - np.cos(np.arange(M) * np.arccos(x7))).max() < 1e-12


@pytest.mark.parametrize("M", [1, 2, 5, 16, 101, 256])
def test_jackson_kernel_closed_values_and_autocorrelation(M):
    """g_0 = 1, g_1 = cos(pi/(M+1)) (so a single level at x_0 keeps its mean
    at g_1 x_0), and g_n equals the normalised autocorrelation
    sum_v a_v a_{v+n} / sum_v a_v^2 of a_v = sin(pi (v+1)/(M+1)) -- the form
    that makes the damped density non-negative."""
    g = kpm.jackson(M)
    assert abs(g[0] - 1.0) < 1e-14
    if M > 1:
        assert abs(g[1] - np.cos(pi / (M + 1))) < 1e-14
    av = np.sin(pi * (np.arange(M) + 1) / (M + 1))
    auto = np.array([np.dot(av[:M - n], av[n:]) for n in range(M)]) / np.dot(av, av)
    assert np.abs(g - auto).max() < 1e-13


@pytest.mark.parametrize("M", [1, 8, 64])
def test_kpm_count_of_the_chebyshev_measure(M):
    """mu = (1, 0, 0, ...) is the measure 1/(pi sqrt(1 - x^2)): the count in
    [x_lo, x_hi] is N (arccos x_lo - arccos x_hi)/pi for any M."""
    mu = np.zeros(M)
    mu[0] = 1.0
    for x_lo, x_hi in [(-1.0, 1.0), (-0.3, 0.2), (0.9, 0.95), (-1.0, -0.99)]:
        ref = 1000 * (np.arccos(x_lo) - np.arccos(x_hi)) / pi
        assert abs(kpm.count(mu, 1000, x_lo, x_hi) - ref) < 1e-9


@pytest.mark.parametrize("x0", [0.0, 0.37, -0.8])
def test_kpm_single_level_weight_and_mean(x0):
    """A single level at x_0 (mu_n = T_n(x_0)): total weight 1 (count N over
    [-1, 1]) and mean position g_1 x_0, by quadrature of the density."""
    M = 64
    mu = np.cos(np.arange(M) * np.arccos(x0))
    assert abs(kpm.count(mu, 50, -1.0, 1.0) - 50.0) < 1e-9
    f = lambda t: float(kpm.density(mu, np.cos(t))[0] * np.cos(t) * np.sin(t))
    mean, _ = scipy.integrate.quad(f, 1e-9, pi - 1e-9, limit=500)
    assert abs(mean - np.cos(pi / (M + 1)) * x0) < 1e-6


def test_kpm_density_of_a_spectrum_nonnegative_and_counts():
    """Exact moments of an L = 12 spectrum: the Jackson-damped density is
    non-negative, integrates to N, and counts the eigenvalues of an interval
    to within the kernel's resolution (pi/M) at the interval's ends."""
    H, w, a, b = _chain_spectrum(12, 2.0, 9)
    N = H.shape[0]
    x = a * w + b
    for M in (64, 512):
        mu = kpm.moments_exact(w, a, b, M)
        grid = np.linspace(-0.999, 0.999, 2001)
        assert kpm.density(mu, grid).min() > -1e-10
        assert abs(kpm.count(mu, N, -1.0, 1.0) - N) < 1e-7
        for lo, hi in [(-0.2, 0.1), (0.3, 0.5)]:
            res = 3.0 * pi / M  # a few kernel widths
            inner = int(((x > lo + res) & (x < hi - res)).sum())
            outer = int(((x > lo - res) & (x < hi + res)).sum())
            cnt = kpm.count(mu, N, lo, hi)
            assert inner - 1 <= cnt <= outer + 1, (M, lo, hi, inner, cnt, outer)


def test_kpm_choose_K_against_a_scan():
    """The KPM order rule is max{K : n_P(K) >= nwin}: against a linear scan
    of n_P over K (Chebyshev measure, N = 2000, sigma~ = 0.3), and on a real
    spectrum's moments the lobe of the chosen K holds about nwin of its
    eigenvalues."""
    mu = np.zeros(16)
    mu[0] = 1.0
    K = kpm.choose_K(20, 0.3, 0.17, mu, 2000)
    f = [kpm.n_P(k, 0.3, 0.17, mu, 2000) for k in range(1, 200)]
    assert K == max(k for k, v in zip(range(1, 200), f) if v >= 20)
    H, w, a, b = _chain_spectrum(14, 1.0, 11)
    sig_t = a * (w[0] + 0.2 * (w[-1] - w[0])) + b
    mu = kpm.moments_exact(w, a, b, 256)
    K = kpm.choose_K(30, sig_t, 0.17, mu, H.shape[0])
    inside = int((chebyshev.P_of_x(a * w + b, sig_t, K) >= 0.17).sum())
    assert 27 <= inside <= 33


# ---------------------------------------------------------------------------
# optional Jackson-damped filter
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K,sigma", [(7, 0.0), (40, 0.3), (201, -0.77), (500, 0.9)])
def test_damped_filter_positive_and_a_single_level_density(K, sigma):
    """The Jackson-damped filter is non-negative on [-1, 1], is 1 at sigma,
    and is the KPM density of one level at sigma (moments T_n(sigma),
    K + 1 of them) times pi sqrt(1 - x^2), up to its normalisation D."""
    x = np.linspace(-0.9999, 0.9999, 3001)
    P = chebyshev.P_of_x(x, sigma, K, damping=1)
    assert P.min() > -1e-13
    assert abs(chebyshev.P_of_x(sigma, sigma, K, damping=1)[0] - 1.0) < 1e-12
    mu = np.cos(np.arange(K + 1) * np.arccos(sigma))
    rho = kpm.density(mu, x)
    D = chebyshev.norm_D(sigma, K, damping=1)
    assert np.abs(P * D - pi * np.sqrt(1.0 - x * x) * rho).max() < 1e-10 * D


@pytest.mark.parametrize("K", [400, 4000])
def test_damped_lobe_edges_hit_p_and_width(K):
    """The damped lobe edges sit at P = p, and their half-width in theta
    tends to 1.8265 pi/(K+2) (the closed form of the damped kernel,
    (E(u+b) + E(u-b))^2 with E(u) = sin(M u/2)/sin(u/2), b = pi/(M+1),
    M = K+1, against the definition sum used for the edges)."""
    for sigma in (0.0, 0.5):
        x_lo, x_hi = chebyshev.lobe_edges(sigma, K, 0.17, damping=1)
        for xe in (x_lo, x_hi):
            assert abs(chebyshev.P_of_x(xe, sigma, K, damping=1)[0] - 0.17) < 1e-9
        a = np.arccos(sigma)
        M, b = K + 1, pi / (K + 2)

        def E(u):
            return np.sin(M * u / 2) / np.sin(u / 2)

        def F(u):
            return (E(u + b) + E(u - b)) ** 2
        t = np.arccos(x_lo) - a
        closed = (F(t) + F(2 * a + t)) / (F(1e-9) + F(2 * a + 1e-9))
        assert abs(closed - 0.17) < 1e-6
        assert abs(t * (K + 2) / pi - 1.8265) < 0.01


def test_damped_choose_K_against_a_scan():
    """With damping the order rule is still max{K : n_P(K) >= nwin}: against
    a linear scan (Gaussian DOS, N = 200, sigma~ = 0.1)."""
    args = (0.1, 0.17, 200, 0.0, 2.0, -8.0, 8.0)
    K = chebyshev.choose_K(20, *args, damping=1)
    assert 20 < K < 400
    f = [chebyshev.n_P(k, *args, damping=1) for k in range(1, 500)]
    assert K == max(k for k, v in zip(range(1, 500), f) if v >= 20)
    # the damped lobe is wider, so the same window takes a higher order
    assert K > chebyshev.choose_K(20, *args)
