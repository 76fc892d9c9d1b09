"""The C-ABI library: loads, exports every declared entry point, and its host
math (no device work) agrees with the oracle.  No GPU needed."""

import ctypes
from math import comb

import numpy as np
import pytest

from oracle import chebyshev
from paper_2005_09534_amd import polfed as pf
from paper_2005_09534_amd import workloads


def test_library_exports_every_declared_symbol():
    names = pf.header_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(pf.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("L", [2, 4, 12, 18, 22, 26, 30])
def test_dim(L):
    assert pf.dim(L) == comb(L, L // 2)


@pytest.mark.parametrize("L", [1, 3, 0, 32, -2])
def test_dim_invalid(L):
    assert pf.dim(L) == -1


def test_default_opts():
    o = pf.default_opts()
    assert o.target == 0.5 and o.p == 0.17 and o.window_factor == 1.5 and o.tol == 1e-10
    assert o.dos == 0 and o.dos_moments == 256 and o.dos_vectors == 4


@pytest.mark.parametrize("sigma", [0.0, 0.37, -0.8])
@pytest.mark.parametrize("K", [0, 1, 7, 200, 5001])
def test_cheb_coeffs_match_oracle(sigma, K):
    c, D = pf.cheb_coeffs(sigma, K)
    # cos(n arccos sigma): a rounding of arccos is amplified n times in the
    # phase (argument n arccos(sigma) carries ~n eps absolute error), so
    # coefficients agree to ~2 n eps (the library evaluates sigma = 0
    # exactly)
    n = np.arange(K + 1)
    assert (np.abs(c - chebyshev.cheb_coeffs(sigma, K)) <= 2e-15 * (n + 4)).all()
    assert abs(D - chebyshev.norm_D(sigma, K)) < 1e-10 * max(1.0, D)


def test_cheb_coeffs_invalid():
    c = np.empty(3)
    d = ctypes.c_double()
    assert pf.LIB.polfed_cheb_coeffs(1.0, 2, c.ctypes.data_as(pf.P_double), ctypes.byref(d)) == pf.EINVAL
    assert pf.LIB.polfed_cheb_coeffs(0.0, -1, c.ctypes.data_as(pf.P_double), ctypes.byref(d)) == pf.EINVAL


@pytest.mark.parametrize("L,W,J2,nwin,sigma", [(12, 3.0, 0.0, 30, 0.0), (16, 1.0, 0.0, 75, 0.1),
                                                 (18, 2.0, 1.0, 75, 0.0), (22, 5.0, 0.0, 150, -0.05),
                                                 (26, 4.0, 0.0, 150, 0.0)])
def test_filter_order_matches_oracle(L, W, J2, nwin, sigma):
    """K from the density of states: integer-exact against the oracle's rule
    (same FP64 decisions, independent evaluation of P: closed form vs sum)."""
    c = workloads.chain(L, W, 7, J2=J2)
    m = pf.make_model(L, c.J1, c.J2, c.Delta, c.h)
    E0w, E1w = -0.9 * L, 0.85 * L
    K, rho = pf.filter_order(m, E0w, E1w, sigma, nwin)
    N = comb(L, L // 2)
    Ebar = -(c.J1 + c.J2) * c.Delta * L / (4.0 * (L - 1))
    G = chebyshev.dos_gamma(L, c.J1, c.J2, c.Delta, c.h)
    if K <= 3000:
        Ko = chebyshev.choose_K(nwin, sigma, 0.17, N, Ebar, G, E0w, E1w)
        assert K == Ko
    # the rule's defining inequalities, evaluated by the oracle
    f = lambda k: chebyshev.n_P(k, sigma, 0.17, N, Ebar, G, E0w, E1w)
    if K <= 20000:
        assert f(K) >= nwin > f(K + 1)
    assert abs(rho - chebyshev.rho_tilde(sigma, N, Ebar, G, E0w, E1w)) < 1e-9 * rho


@pytest.mark.parametrize("L,W,nwin,cap", [(12, 3.0, 20, 120), (12, 1.0, 10, 60), (14, 2.0, 30, 400)])
def test_fp32_order_cap_matches_oracle(L, W, nwin, cap):
    """The FP32 order cap: the library's window (doubling and bisection) is
    the oracle's (upward scan), window and order integer-exact; the order
    fits, one window fewer does not."""
    c = workloads.chain(L, W, 11)
    m = pf.make_model(L, c.J1, c.J2, c.Delta, c.h)
    E0w, E1w = -0.9 * L, 0.85 * L
    K0, _ = pf.filter_order(m, E0w, E1w, 0.0, nwin)
    assert K0 > cap  # the cases exercise the cap
    nw, K = pf.window_order(m, E0w, E1w, 0.0, nwin, cap)
    N = comb(L, L // 2)
    Ebar = -(c.J1 + c.J2) * c.Delta * L / (4.0 * (L - 1))
    G = chebyshev.dos_gamma(L, c.J1, c.J2, c.Delta, c.h)
    assert (nw, K) == chebyshev.capped_window(nwin, 0.0, 0.17, N, Ebar, G, E0w, E1w, cap)
    assert K <= cap < pf.filter_order(m, E0w, E1w, 0.0, nw - 1)[0]
    # no cap, or a cap above the order: the window stays
    assert pf.window_order(m, E0w, E1w, 0.0, nwin, 0) == (nwin, K0)
    assert pf.window_order(m, E0w, E1w, 0.0, nwin, K0) == (nwin, K0)


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    rc = pf.LIB.polfed_create(0, ctypes.byref(h))
    assert rc < 0 and not h.value
    assert pf.LIB.polfed_last_error(None)  # the reason is reported without a context


def test_one_hip_runtime_in_process():
    """The binding loads the library after torch, so the process maps a single
    HIP runtime (torch's); a second copy loaded first can fail to see the
    device."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    assert len(paths) == 1, paths


def test_gap_ratio_and_s_rmt_match_oracle():
    from oracle import observables
    E = np.random.default_rng(4).standard_normal(200)
    assert abs(pf.gap_ratio(E) - observables.mean_gap_ratio(E)) <= 1e-14
    for L in (8, 14, 26):
        assert abs(pf.s_rmt(L) - observables.s_rmt(L)) <= 1e-14
    with pytest.raises(pf.PolfedError):
        pf.gap_ratio([0.0, 1.0])


def _exact_moments(L, W, seed, M, J2=0.0, Delta=1.0):
    from oracle import chain, dense, kpm, lanczos
    c = workloads.chain(L, W, seed, J2=J2, Delta=Delta)
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    w = dense.full_spectrum(H)
    E0w, E1w = lanczos.widened_bounds(w[0], w[-1], 1e-3)
    a, b = chebyshev.rescale_coeffs(E0w, E1w)
    return kpm.moments_exact(w, a, b, M), w, a, b


@pytest.mark.parametrize("M", [1, 16, 256])
def test_kpm_count_matches_oracle(M):
    """The library's closed-form KPM count against the oracle's quadrature
    of the Jackson-damped density, on an L = 12 spectrum's moments."""
    from oracle import kpm
    mu, w, a, b = _exact_moments(12, 3.0, 21, M)
    N = len(w)
    for lo, hi in [(-1.0, 1.0), (-0.31, 0.07), (0.5, 0.5005), (-2.0, -0.9)]:
        got = pf.kpm_count(mu, N, lo, hi)
        ref = kpm.count(mu, N, lo, hi)
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref)), (lo, hi, got, ref)
    with pytest.raises(pf.PolfedError):
        pf.kpm_count(mu, N, 0.2, 0.1)


@pytest.mark.parametrize("L,W,J2,Delta,eps", [(12, 8.0, 0.0, 1.0, 0.3), (14, 0.5, 1.0, 0.55, 0.85),
                                             (14, 5.0, 0.0, 1.0, 0.5)])
def test_kpm_order_matches_oracle(L, W, J2, Delta, eps):
    """polfed_kpm_order (doubling and bisection with the closed-form count)
    is the oracle's KPM order rule, integer-exact; under a cap the window is
    the smallest whose order fits."""
    from oracle import kpm
    mu, w, a, b = _exact_moments(L, W, 11 if J2 == 0.0 else 12, 256, J2=J2, Delta=Delta)
    N = len(w)
    sig_t = a * (w[0] + eps * (w[-1] - w[0])) + b
    nw, K = pf.kpm_order(mu, N, sig_t, 30)
    assert nw == 30 and K == kpm.choose_K(30, sig_t, 0.17, mu, N)
    cap = max(2, K // 3)
    nw2, K2 = pf.kpm_order(mu, N, sig_t, 30, max_order=cap)
    assert nw2 > 30 and K2 <= cap
    assert K2 == kpm.choose_K(nw2, sig_t, 0.17, mu, N)
    assert kpm.choose_K(nw2 - 1, sig_t, 0.17, mu, N) > cap


@pytest.mark.parametrize("sigma,K", [(0.0, 0), (0.0, 31), (0.37, 200), (-0.8, 5001)])
def test_filter_coeffs_damped_match_oracle(sigma, K):
    """polfed_filter_coeffs with and without Jackson damping against the
    oracle's coefficients and normalisation."""
    for damping in (0, 1):
        c, D = pf.filter_coeffs(sigma, K, damping)
        ref = chebyshev.filter_coeffs(sigma, K, damping)
        assert np.abs(c - ref).max() <= 2e-15 * (K + 4)
        Dref = chebyshev.norm_D(sigma, K, damping)
        assert abs(D - Dref) <= 1e-12 * abs(Dref)
    with pytest.raises(pf.PolfedError):
        pf.filter_coeffs(0.1, 10, 2)


@pytest.mark.parametrize("L,W,nwin,sigma", [(12, 3.0, 20, 0.0), (14, 1.0, 30, 0.3),
                                            (16, 5.0, 10, -0.6)])
def test_damped_order_matches_oracle(L, W, nwin, sigma):
    """The order rule for the Jackson-damped filter (the library's closed
    form of the damped lobe) against the oracle's (its definition sum),
    integer-exact; and under a cap, the smallest window whose order fits."""
    c = workloads.chain(L, W, 11)
    m = pf.make_model(L, c.J1, c.J2, c.Delta, c.h)
    E0w, E1w = -0.9 * L, 0.85 * L
    N = comb(L, L // 2)
    Ebar = -(c.J1 + c.J2) * c.Delta * L / (4.0 * (L - 1))
    G = chebyshev.dos_gamma(L, c.J1, c.J2, c.Delta, c.h)
    nw, K = pf.filter_order_damped(m, E0w, E1w, sigma, nwin, 1)
    assert nw == nwin
    assert K == chebyshev.choose_K(nwin, sigma, 0.17, N, Ebar, G, E0w, E1w, damping=1)
    # undamped through the same call equals polfed_filter_order
    assert pf.filter_order_damped(m, E0w, E1w, sigma, nwin, 0)[1] == \
        pf.filter_order(m, E0w, E1w, sigma, nwin)[0]
    cap = max(2, K // 3)
    nw2, K2 = pf.filter_order_damped(m, E0w, E1w, sigma, nwin, 1, max_order=cap)
    assert (nw2, K2) == chebyshev.capped_window(nwin, sigma, 0.17, N, Ebar, G, E0w, E1w, cap,
                                                damping=1)
