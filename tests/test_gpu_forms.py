"""The forward three-term form of the filter and the incremental neighbour
ranks, on the GPU through the C ABI.

The forward form (t_{k+1} = 2 H~ t_k - t_{k-1}, c_k T_k(H~) X added term by
term) is checked against the oracle's filter, which uses the same recurrence
in plain FP64 on a CSR H, and against the library's Clenshaw form; the
incremental ranks (a binomial step from the row's own rank for bonds that do
not wrap) must give bit for bit what the rank tables give."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chain, chebyshev, dense, lanczos  # noqa: E402
from paper_2005_09534_amd import workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    from paper_2005_09534_amd import polfed
    return polfed


@pytest.fixture(scope="module")
def ctx(pf):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pf.Context(0)
    yield c
    c.close()


@pytest.fixture
def forward(ctx, pf):
    ctx.set_filter_form(pf.FORM_FORWARD)
    yield
    ctx.set_filter_form(pf.FORM_CLENSHAW)


def _model(pf, c):
    return pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h)


def _bounds(H):
    E0, E1 = lanczos.extreme_eigenvalues(H)
    return lanczos.widened_bounds(E0, E1, 1e-3)


# ------------------------------------------------------- forward filter --

@pytest.mark.parametrize("K", [0, 1, 2, 3, 7, 200, 201])
@pytest.mark.parametrize("sigma", [0.0, 0.31])
def test_forward_filter_fp64_vs_oracle(ctx, pf, forward, K, sigma):
    c = workloads.chain(12, 3.0, 1)
    H = chain.hamiltonian_csr(12, c.J1, c.J2, c.Delta, c.h)
    E0, E1 = _bounds(H)
    X = workloads.random_block(H.shape[0], 4, 2)
    Y = ctx.apply_filter(_model(pf, c), E0, E1, sigma, K, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = chebyshev.filter_block(H, X, E0, E1, sigma, K)
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_forward_filter_vs_oracle_L16_J2(ctx, pf, forward):
    c = workloads.chain(16, 2.0, 4, J2=1.0)
    H = chain.hamiltonian_csr(16, c.J1, c.J2, c.Delta, c.h)
    E0, E1 = _bounds(H)
    X = workloads.random_block(H.shape[0], 8, 3)
    Y = ctx.apply_filter(_model(pf, c), E0, E1, 0.0, 1500, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = chebyshev.filter_block(H, X, E0, E1, 0.0, 1500)
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_forward_and_clenshaw_agree(ctx, pf):
    """Two algorithms for one polynomial: FP64 results agree to rounding, and
    the FP32 forward filter matches the FP64 one to 1e-4 relative."""
    c = workloads.chain(14, 2.0, 6, J2=0.4)
    m = _model(pf, c)
    E0, E1, r0, r1 = ctx.bounds(m, 200)
    w = E1 - E0
    E0, E1 = E0 - r0 - 1e-3 * w, E1 + r1 + 1e-3 * w
    X = torch.from_numpy(workloads.random_block(pf.dim(14), 16, 4)).cuda()
    try:
        ctx.set_filter_form(pf.FORM_CLENSHAW)
        Yc = ctx.apply_filter(m, E0, E1, 0.12, 1200, X).cpu().numpy()
        ctx.set_filter_form(pf.FORM_FORWARD)
        Yf = ctx.apply_filter(m, E0, E1, 0.12, 1200, X).cpu().numpy()
        Yf32 = ctx.apply_filter(m, E0, E1, 0.12, 1200, X.float()).cpu().numpy()
    finally:
        ctx.set_filter_form(pf.FORM_CLENSHAW)
    scale = np.abs(Yc).max()
    assert np.abs(Yf - Yc).max() <= 1e-11 * scale
    assert np.abs(Yf32 - Yf).max() <= 1e-4 * scale


def test_forward_launches_and_bytes(ctx, pf, forward):
    """At sigma~ = 0 the odd coefficients vanish, so the forward form stops at
    the last even order; its byte count follows the stream model (five
    blocks per step where c_k != 0, three where it is 0, plus state word and
    diagonal)."""
    c = workloads.chain(10, 1.0, 3)
    m = _model(pf, c)
    n = pf.dim(10)
    X = torch.from_numpy(workloads.random_block(n, 4, 1)).cuda()
    ctx.filter_stats(reset=True)
    ctx.apply_filter(m, -25.0, 25.0, 0.0, 9, X)
    st = ctx.filter_stats(reset=True)
    assert st["launches"] == 8
    b, s = 8, 4
    per_row = (4 + b) * 8  # every step applies H~
    # step 1: out + V(=X) + src(X) + acc(Y) = 4 blocks; steps 2..7: out, V, W and
    # acc in/out when k is even (k = 2, 4, 6 -> 5 blocks; k = 3, 5, 7 -> 3); step 8
    # (last, even): no out, V, W, acc in/out = 4 blocks
    blocks = 4 + 3 * 5 + 3 * 3 + 4
    assert st["bytes"] == pytest.approx(n * (s * b * blocks + per_row))


@pytest.mark.parametrize("prec", [np.float64, np.float32])
def test_forward_graph_replays_match_direct(ctx, pf, forward, prec):
    c = workloads.chain(14, 2.0, 12)
    m = _model(pf, c)
    X = torch.from_numpy(workloads.random_block(pf.dim(14), 8, 1).astype(prec)).cuda()
    E0, E1, r0, r1 = ctx.bounds(m, 200)
    E0, E1 = E0 - r0 - 0.01 * (E1 - E0), E1 + r1 + 0.01 * (E1 - E0)
    ctx.set_graphs(False)
    try:
        ref = ctx.apply_filter(m, E0, E1, 0.1, 300, X).cpu()
        assert torch.isfinite(ref).all()
        ctx.set_graphs(True)
        Y = torch.empty_like(X)
        for rep in range(3):
            ctx.apply_filter(m, E0, E1, 0.1, 300, X, out=Y)
            _ = (X * 2).sum().item()  # eager work and a sync between replays
            assert torch.equal(Y.cpu(), ref), rep
    finally:
        ctx.set_graphs(True)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_with_forward_form(ctx, pf, forward, precision):
    """A whole solve (Lanczos blocks and, in FP32 mode, the FP64 refinement)
    with the forward form returns the dense answer."""
    wl = workloads.c1()
    c = wl.chains[0]
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    w = dense.full_spectrum(H)
    normH = max(abs(w[0]), abs(w[-1]))
    r = ctx.solve(_model(pf, c), wl.nev, block_size=wl.block, K=wl.K, precision=precision,
                  vectors=True)
    assert r["status"] == pf.OK
    Ed = w[dense.nearest_from_spectrum(w, r["info"]["sigma_energy"], wl.nev)]
    assert np.abs(r["E"] - Ed).max() <= 1e-10 * normH
    res = np.linalg.norm(H @ r["V"] - r["V"] * r["E"], axis=0)
    assert res.max() <= 1e-8 * normH


def test_batch_ignores_forward_setting(ctx, pf):
    """The batched solve filters with Clenshaw whatever the context's form,
    and leaves the setting as it found it."""
    cs = [workloads.chain(10, 2.0, 70 + i) for i in range(2)]
    ms = [_model(pf, c) for c in cs]
    ref = ctx.solve_batch(ms, 6, block_size=2, precision=0)
    ctx.set_filter_form(pf.FORM_FORWARD)
    try:
        got = ctx.solve_batch(ms, 6, block_size=2, precision=0)
        X = torch.from_numpy(workloads.random_block(pf.dim(10), 2, 1)).cuda()
        ctx.filter_stats(reset=True)
        ctx.apply_filter(ms[0], -25.0, 25.0, 0.0, 9, X)
        assert ctx.filter_stats(reset=True)["launches"] == 8  # still forward
    finally:
        ctx.set_filter_form(pf.FORM_CLENSHAW)
    np.testing.assert_array_equal(got["E"], ref["E"])


def test_filter_form_rejects_unknown(ctx, pf):
    with pytest.raises(pf.PolfedError):
        ctx.set_filter_form(2)


# ---------------------------------------------------- incremental ranks --

@pytest.mark.parametrize("L,J2,nvec,dtype", [(14, 0.7, 8, torch.float64), (18, 1.0, 16, torch.float64),
                                             (22, 0.5, 32, torch.float32),
                                             (26, 0.0, 1, torch.float64)])
def test_incremental_ranks_bitwise(ctx, pf, L, J2, nvec, dtype):
    """H X with neighbour ranks from binomial steps, and with neighbours read
    from the stored pattern, equals H X with the rank tables bit for bit, up
    to the full L = 26 chain (10,400,600 rows)."""
    c = workloads.chain(L, 3.0, 40 + L, J2=J2)
    m = _model(pf, c)
    n = pf.dim(L)
    g = torch.Generator(device="cuda").manual_seed(L)
    X = torch.randn((n, nvec), generator=g, device="cuda", dtype=torch.float64).to(dtype)
    prec = 1 if dtype == torch.float32 else 0
    saved = ctx.get_step_shape(L, nvec, prec)
    try:
        ctx.set_step_shape(L, nvec, prec, *saved[:5], 0)
        Yt = ctx.apply_h(m, X)
        ctx.set_step_shape(L, nvec, prec, *saved[:5], 1)
        Yi = ctx.apply_h(m, X)
        ctx.set_step_shape(L, nvec, prec, *saved[:5], 2)
        Yp = ctx.apply_h(m, X)
        torch.cuda.synchronize()
        assert torch.equal(Yt, Yi)
        assert torch.equal(Yt, Yp)
    finally:
        ctx.set_step_shape(L, nvec, prec, *saved)
    del X, Yt, Yi, Yp
    torch.cuda.empty_cache()


def test_incremental_ranks_vs_oracle(ctx, pf):
    """With incremental ranks, H X matches the oracle's CSR H (J2 != 0)."""
    c = workloads.chain(16, 2.5, 9, J2=0.8, Delta=0.7)
    H = chain.hamiltonian_csr(16, c.J1, c.J2, c.Delta, c.h)
    X = workloads.random_block(H.shape[0], 4, 8)
    saved = ctx.get_step_shape(16, 4, 0)
    try:
        ctx.set_step_shape(16, 4, 0, *saved[:5], 1)
        Y = ctx.apply_h(_model(pf, c), torch.from_numpy(X).cuda()).cpu().numpy()
    finally:
        ctx.set_step_shape(16, 4, 0, *saved)
    ref = H @ X
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
