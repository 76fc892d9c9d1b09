"""ORACLE (test infrastructure only) -- density of states by the kernel
polynomial method.

The order K of the filter comes from the density of states of H~ at the
target (main text, "POLFED algorithm"); for a matrix whose density has no
closed form the paper points to the iterative estimators of Silver et al.,
which take Chebyshev moments of H~ from random vectors:

    mu_n = Tr T_n(H~) / N            (definition, from the eigenvalues)
    mu_n ~ sum_r <r|T_n(H~)|r> / sum_r <r|r>   (stochastic estimate)

and rebuild the density with Jackson damping (Weisse et al., Rev. Mod.
Phys. 78, 275 (2006), eqs. for the Jackson kernel):

    rho(x) = [g_0 mu_0 + 2 sum_{n=1}^{M-1} g_n mu_n T_n(x)] / (pi sqrt(1 - x^2)),
    g_n = [(M - n + 1) cos(pi n / (M + 1)) + sin(pi n / (M + 1)) cot(pi / (M + 1))] / (M + 1).

The number of states in [x_lo, x_hi] is N times the integral of rho; here it
is taken by adaptive quadrature in theta (x = cos theta, which removes the
end-point singularity), not by the closed form of the library.  The
stochastic moments are taken by applying the plain three-term recurrence n
times to each vector and projecting on it, not by the product identities the
library uses.

Readings: the estimate is normalised by sum <r|r> (so mu_0 = 1 exactly for
any vectors); the order rule is the one of ``chebyshev.choose_K`` with this
count in place of the Gaussian one.

Parity pins (tests/test_oracle_pins.py): stochastic moments over all basis
vectors equal the eigenvalue definition (the trace); g_0 = 1 and g_1 =
cos(pi/(M+1)); the Chebyshev measure (mu = delta_n0) counts N (t_lo - t_hi)/pi
states; a single level keeps unit weight with its mean at g_1 x_0; the
density of a real spectrum is non-negative and integrates to N; the order
rule on the Chebyshev measure against a brute-force scan over K.
"""

from math import pi

import numpy as np
from scipy import integrate

from . import chebyshev


def moments_exact(evals, a, b, M):
    """mu_n = (1/N) sum_i T_n(a E_i + b), n < M, from the eigenvalues E_i of H."""
    x = a * np.asarray(evals, dtype=np.float64) + b
    th = np.arccos(np.clip(x, -1.0, 1.0))
    n = np.arange(M, dtype=np.float64)
    return np.cos(np.outer(n, th)).mean(axis=1)


def moments_stochastic(H, a, b, R, M):
    """mu_n = sum_r <r|T_n(H~)|r> / sum_r <r|r>, n < M, over the columns r of
    R (n x nvec), with T_n(H~) r from the three-term recurrence.  H: scipy
    sparse or dense (N x N) FP64."""
    R = np.asarray(R, dtype=np.float64)
    if R.ndim == 1:
        R = R[:, None]

    def Ht(V):
        return a * (H @ V) + b * V

    norm = float(np.sum(R * R))
    mu = np.zeros(M)
    t_prev = R
    mu[0] = float(np.sum(R * t_prev)) / norm
    if M > 1:
        t_cur = Ht(R)
        mu[1] = float(np.sum(R * t_cur)) / norm
        for n in range(2, M):
            t_next = 2.0 * Ht(t_cur) - t_prev
            mu[n] = float(np.sum(R * t_next)) / norm
            t_prev, t_cur = t_cur, t_next
    return mu


def jackson(M):
    """Jackson damping factors g_0 .. g_{M-1}."""
    n = np.arange(M, dtype=np.float64)
    q = pi / (M + 1)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (M + 1)


def density(mu, x):
    """rho(x), states per unit of x per state (integrates to mu_0)."""
    mu = np.asarray(mu, dtype=np.float64)
    M = len(mu)
    g = jackson(M)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    th = np.arccos(np.clip(x, -1.0, 1.0))
    n = np.arange(M, dtype=np.float64)
    w = g * mu
    w[1:] *= 2.0
    return (np.cos(np.outer(th, n)) @ w) / (pi * np.sqrt(1.0 - x * x))


def count(mu, N, x_lo, x_hi):
    """N * integral of rho over [x_lo, x_hi]: with x = cos theta,
    (N/pi) * integral_{t_hi}^{t_lo} [g_0 mu_0 + 2 sum g_n mu_n cos(n t)] dt,
    by adaptive quadrature."""
    mu = np.asarray(mu, dtype=np.float64)
    M = len(mu)
    g = jackson(M)
    w = g * mu
    w[1:] *= 2.0
    n = np.arange(M, dtype=np.float64)
    t_lo = float(np.arccos(np.clip(x_lo, -1.0, 1.0)))
    t_hi = float(np.arccos(np.clip(x_hi, -1.0, 1.0)))
    f = lambda t: float(np.dot(w, np.cos(n * t)))
    # the integrand oscillates up to frequency M - 1: split into pieces of
    # at most a tenth of its period
    pieces = max(1, int(np.ceil((t_lo - t_hi) * M * 10.0 / (2.0 * pi))))
    edges = np.linspace(t_hi, t_lo, pieces + 1)
    total = 0.0
    for u, v in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(f, u, v, epsabs=1e-14, epsrel=1e-13, limit=200)
        total += val
    return N * total / pi


def n_P(K, sigma, p, mu, N, damping=0):
    """States of the KPM density inside the main lobe {P_K >= p}."""
    x_lo, x_hi = chebyshev.lobe_edges(sigma, K, p, damping=damping)
    return count(mu, N, x_lo, x_hi)


def choose_K(nev, sigma, p, mu, N, K_max=1 << 26, damping=0):
    """K = max{K >= 1 : n_P(K) >= nev} with the KPM count.  Doubling from
    K = 1, then bisection (n_P falls with K)."""
    f = lambda K: n_P(K, sigma, p, mu, N, damping)
    if f(1) < nev:
        return 1
    lo, hi = 1, 2
    while hi <= K_max and f(hi) >= nev:
        lo, hi = hi, hi * 2
    if hi > K_max:
        return K_max
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if f(mid) >= nev:
            lo = mid
        else:
            hi = mid
    return lo
