"""ORACLE (test infrastructure only) -- the polynomial spectral transformation.

eq. (polyTransf):  P^K_sigma(x) = (1/D) sum_{n=0}^{K} c_n T_n(x),
    c_n = sqrt(4 - 3 delta_{n0}) cos(n arccos sigma),   D such that P(sigma)=1.

The filter is applied here by the *forward* three-term recurrence
T_{n+1} = 2 x T_n - T_{n-1} (Supplement "Technical details"), accumulating
c_n T_n(H~) X -- deliberately not the Clenshaw form the GPU path uses, so the
two are algorithmically independent.

Order selection (main text "POLFED algorithm"; Supplement "Convergence"):
K is chosen so that the number n_P of eigenvalues of P(H~) with
theta >= p = 0.17 equals the number of requested eigenvalues.  n_P is the
integral of the density of states of H~ over the main lobe {x : P_K(x) >= p}.
The density of states is the Gaussian of the Supplement ("Convergence" eq. for
Gamma).  Readings (the paper is terse here):
* rho~ carries the Gaussian normalisation 1/(sqrt(2 pi) Gamma) and its centre
  is the mean energy Tr H / N; the paper's rho~(0) = (E1-E0) N / Gamma drops
  the constant;
* Gamma^2 = L (J1^2 + J2^2)(2 + Delta^2)/16 + sum_i h_i^2 / 4, the variance of
  H for this realisation; at J1 = 1 its disorder average is the paper's
  L[(1+J2^2)/8 + Delta^2 (1+J2^2)/16 + W^2/12];
* K = max{K : n_P(K) >= N_ev}; found by doubling then bisection on K; lobe
  edges by bisection in theta (x = cos theta).

Optional damped variant (not in the paper, whose expansion is undamped):
c_n times the Jackson factors g_n of the K+1 coefficients (``kpm.jackson``),
D again sum_n c_n T_n(sigma); the lobe edges and the order rule are those of
the damped P, evaluated here by its definition sum.

Parity pins: the Dirichlet-kernel closed form of P, D at sigma = 0,
P(H~)v = P(lambda~)v on eigenvectors, the asymptotic K formula; for the
damped P: non-negative everywhere, equal to pi sqrt(1 - x^2) times the
KPM density of a single level at sigma (up to D), and its lobe half-width
tending to 1.8265 pi/(K+2).
"""

from math import erf, sqrt, pi

import numpy as np


def cheb_coeffs(sigma, K):
    """c_0..c_K of eq. (polyTransf) for target sigma in H~ units."""
    n = np.arange(K + 1, dtype=np.float64)
    c = 2.0 * np.cos(n * np.arccos(sigma))
    c[0] = 1.0  # sqrt(4 - 3) cos(0)
    return c


def filter_coeffs(sigma, K, damping=0):
    """c_n of eq. (polyTransf), times the Jackson factors g_n of the K+1
    coefficients when damping = 1 (the optional damped variant; the paper's
    filter is undamped)."""
    c = cheb_coeffs(sigma, K)
    if damping:
        from . import kpm
        c = c * kpm.jackson(K + 1)
    return c


def norm_D(sigma, K, damping=0):
    """D = sum_n c_n T_n(sigma), so that P(sigma) = 1."""
    c = filter_coeffs(sigma, K, damping)
    n = np.arange(K + 1, dtype=np.float64)
    return float(np.sum(c * np.cos(n * np.arccos(sigma))))


def P_of_x(x, sigma, K, damping=0):
    """P^K_sigma(x) by its definition: (1/D) sum c_n cos(n arccos x)."""
    c = filter_coeffs(sigma, K, damping)
    D = norm_D(sigma, K, damping)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = np.arange(K + 1, dtype=np.float64)
    th = np.arccos(np.clip(x, -1.0, 1.0))
    return (np.cos(np.outer(th, n)) @ c) / D


def rescale_coeffs(E0, E1):
    """H~ = [2H - (E0 + E1)] / (E1 - E0) = a H + b  (main text)."""
    a = 2.0 / (E1 - E0)
    b = -(E0 + E1) / (E1 - E0)
    return a, b


def filter_block(H, X, E0, E1, sigma, K, damping=0):
    """Y = P^K_sigma(H~) X by the forward recurrence, FP64.
    H: scipy sparse (n x n) FP64; X: (n x s)."""
    a, b = rescale_coeffs(E0, E1)
    c = filter_coeffs(sigma, K, damping)
    D = norm_D(sigma, K, damping)

    def Ht(V):
        return a * (H @ V) + b * V

    X = np.asarray(X, dtype=np.float64)
    t_prev = X
    Y = c[0] * t_prev
    if K >= 1:
        t_cur = Ht(X)
        Y = Y + c[1] * t_cur
        for n in range(2, K + 1):
            t_next = 2.0 * Ht(t_cur) - t_prev
            Y = Y + c[n] * t_next
            t_prev, t_cur = t_cur, t_next
    return Y / D


# ---------------------------------------------------------------------------
# density of states and the order rule
# ---------------------------------------------------------------------------

def dos_gamma(L, J1, J2, Delta, h):
    """Width Gamma of the Gaussian density of states of H (realisation form)."""
    h = np.asarray(h, dtype=np.float64)
    g2 = L * (J1 * J1 + J2 * J2) * (2.0 + Delta * Delta) / 16.0 + float(np.sum(h * h)) / 4.0
    return sqrt(g2)


def n_states_between(N, Ebar, Gamma, Elo, Ehi):
    """Number of states of the Gaussian DOS (N states, centre Ebar, width
    Gamma) with energy in [Elo, Ehi]."""
    s = sqrt(2.0) * Gamma
    return 0.5 * N * (erf((Ehi - Ebar) / s) - erf((Elo - Ebar) / s))


def rho_tilde(x, N, Ebar, Gamma, E0, E1):
    """Density of states of H~ at x (states per unit of x)."""
    E = 0.5 * (x * (E1 - E0) + (E1 + E0))
    return N * (E1 - E0) / (2.0 * sqrt(2.0 * pi) * Gamma) * np.exp(-(E - Ebar) ** 2 / (2 * Gamma ** 2))


def _P_theta(theta, sigma, K, c, D):
    n = np.arange(K + 1, dtype=np.float64)
    return float(np.dot(np.cos(n * theta), c) / D)


def lobe_edges(sigma, K, p, iters=200, damping=0):
    """Edges (x_lo, x_hi) of the main lobe {P_K >= p} around sigma, by
    bisection in theta on [alpha, alpha + w] (right) and [alpha - w, alpha]
    (left), clipped to [0, pi]; w = 2 pi/(2K+1), the first zero of the
    undamped kernel, or 6 pi/(K+2) for the damped filter (its kernel's first
    zero is near 3 pi/(K+2) and its side lobes are far below p)."""
    c = filter_coeffs(sigma, K, damping)
    D = norm_D(sigma, K, damping)
    alpha = float(np.arccos(sigma))
    w = 6.0 * pi / (K + 2) if damping else 2.0 * pi / (2 * K + 1)

    def edge(t_in, t_out):
        # P(t_in) >= p; find crossing towards t_out
        if _P_theta(t_out, sigma, K, c, D) >= p:
            return t_out
        for _ in range(iters):
            mid = 0.5 * (t_in + t_out)
            if mid == t_in or mid == t_out:
                break
            if _P_theta(mid, sigma, K, c, D) >= p:
                t_in = mid
            else:
                t_out = mid
        return t_in

    th_r = edge(alpha, min(alpha + w, pi))   # larger theta -> smaller x
    th_l = edge(alpha, max(alpha - w, 0.0))
    return float(np.cos(th_r)), float(np.cos(th_l))


def n_P(K, sigma, p, N, Ebar, Gamma, E0, E1, damping=0):
    """Estimated number of eigenvalues of P^K(H~) that are >= p."""
    x_lo, x_hi = lobe_edges(sigma, K, p, damping=damping)
    Elo = 0.5 * (x_lo * (E1 - E0) + (E1 + E0))
    Ehi = 0.5 * (x_hi * (E1 - E0) + (E1 + E0))
    return n_states_between(N, Ebar, Gamma, Elo, Ehi)


def choose_K(nev, sigma, p, N, Ebar, Gamma, E0, E1, K_max=1 << 26, damping=0):
    """K = max{K >= 1 : n_P(K) >= nev}.  Doubling from K=1, then bisection."""
    f = lambda K: n_P(K, sigma, p, N, Ebar, Gamma, E0, E1, damping)
    if f(1) < nev:
        return 1
    lo = 1
    hi = 2
    while hi <= K_max and f(hi) >= nev:
        lo = hi
        hi *= 2
    if hi > K_max:
        return K_max
    # invariant: f(lo) >= nev, f(hi) < nev
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if f(mid) >= nev:
            lo = mid
        else:
            hi = mid
    return lo


def capped_window(nwin, sigma, p, N, Ebar, Gamma, E0, E1, K_cap, damping=0):
    """Window count under a cap on the order (the FP32 filter's rounding
    error grows like sqrt(K)): the smallest N_win >= nwin whose order
    choose_K(N_win) is at most K_cap, found by scanning upward.  A wider
    window takes a shorter filter at about the same total work (Supplement,
    "Benchmark for disorder spin chains": N_ev -> a N_ev gives K -> K/a).
    Returns (N_win, K).  Parity: pinned by its definition (the order fits,
    one fewer does not) and by the paper's K ~ 1/N_win law."""
    w = int(nwin)
    while True:
        K = choose_K(w, sigma, p, N, Ebar, Gamma, E0, E1, damping=damping)
        if K <= K_cap or w >= N:
            return w, K
        w += 1
