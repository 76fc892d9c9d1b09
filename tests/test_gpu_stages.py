"""GPU parity of the stage calls of libpolfed against the CPU oracle.

Every call goes through the C ABI (paper_2005_09534_amd.polfed -> libpolfed.so).
Tolerances:
* basis, ranks: bit-exact (integer work);
* H.V in FP64: <= 1e-13 relative to max |HX| (a row sums <= 2L+1 terms);
* H.V in FP32 vs the FP64 result: <= 2e-6 relative (a few eps32);
* filter in FP64 vs the oracle's forward recurrence (same E0, E1, sigma,
  K): <= 1e-10 relative; FP32 filter vs FP64: <= 1e-4 relative per column;
* MFMA Gram / update vs numpy: <= 1e-13 relative to the operand scale.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chain, chebyshev, dense, lanczos  # noqa: E402
from paper_2005_09534_amd import workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09534_amd import polfed as pf
    c = pf.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def pf():
    from paper_2005_09534_amd import polfed
    return polfed


def _model(pf, c):
    return pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h)


# ------------------------------------------------------------ basis/rank --

@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 14, 16, 18, 20, 22, 26])
def test_basis_bit_exact(ctx, L):
    b = ctx.basis(L).cpu().numpy().view(np.uint32)
    ref = chain.basis(L)
    assert b.shape == ref.shape
    assert (b == ref).all()


@pytest.mark.parametrize("L", [4, 12, 20, 26])
def test_rank_bit_exact(ctx, L):
    ref = chain.basis(L)
    st = torch.from_numpy(ref.view(np.int32)).cuda()
    r = ctx.rank(L, st).cpu().numpy()
    assert (r == np.arange(len(ref))).all()
    # invalid states: wrong popcount, bits above L
    bad = np.array([0, 1, (1 << L) - 1, int(ref[0]) | (1 << L) if L < 31 else 0], dtype=np.uint32)
    rb = ctx.rank(L, torch.from_numpy(bad.view(np.int32)).cuda()).cpu().numpy()
    assert (rb == -1).all()


def test_rank_empty(ctx):
    out = ctx.rank(12, torch.empty(0, dtype=torch.int32, device="cuda"))
    assert out.numel() == 0


@pytest.mark.parametrize("L,J2,Delta", [(8, 0.0, 1.0), (12, 1.0, 0.55), (18, 1.0, 1.0)])
def test_diag(ctx, pf, L, J2, Delta):
    c = workloads.chain(L, 3.0, 11, J2=J2, Delta=Delta)
    d = ctx.diag(_model(pf, c)).cpu().numpy()
    ref = chain.diagonal(L, c.J1, c.J2, c.Delta, c.h)
    assert np.abs(d - ref).max() <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------------------------ H.V --

@pytest.mark.parametrize("L,J2", [(6, 0.0), (6, 1.0), (12, 0.0), (12, 1.0), (16, 0.7), (18, 1.0)])
@pytest.mark.parametrize("nvec", [1, 2, 4, 8, 16, 32, 64])
def test_apply_h_fp64(ctx, pf, L, J2, nvec):
    c = workloads.chain(L, 2.5, 20 + L, J2=J2, Delta=0.9)
    H = chain.hamiltonian_csr(L, c.J1, c.J2, c.Delta, c.h)
    X = workloads.random_block(H.shape[0], nvec, 5)
    Y = ctx.apply_h(_model(pf, c), torch.from_numpy(X).cuda()).cpu().numpy()
    ref = H @ X
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("L,nvec", [(12, 4), (16, 32), (18, 64), (18, 1)])
def test_apply_h_fp32(ctx, pf, L, nvec):
    c = workloads.chain(L, 5.0, 3)
    H = chain.hamiltonian_csr(L, c.J1, c.J2, c.Delta, c.h)
    X = workloads.random_block(H.shape[0], nvec, 6).astype(np.float32)
    Y = ctx.apply_h(_model(pf, c), torch.from_numpy(X).cuda()).cpu().numpy()
    ref = H @ X.astype(np.float64)
    assert np.abs(Y - ref).max() <= 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("L,nvec,dtype", [(26, 64, np.float32), (26, 16, np.float64),
                                          (22, 32, np.float32), (22, 32, np.float64)])
def test_apply_h_large_sampled_rows(ctx, pf, L, nvec, dtype):
    """Full-size chains (L=22: 705,432 rows; L=26: 10,400,600 rows; the
    widths of those workloads): 300 sampled rows against the oracle's
    per-row form."""
    wl = workloads.c5() if L == 26 else workloads.c3()
    c = wl.chains[0]
    m = _model(pf, c)
    n = pf.dim(L)
    g = torch.Generator(device="cuda").manual_seed(9)
    X = torch.randn((n, nvec), generator=g, device="cuda", dtype=torch.float64).to(
        torch.float32 if dtype == np.float32 else torch.float64)
    Y = ctx.apply_h(m, X)
    b = chain.basis(L)
    rows = np.unique(np.concatenate([[0, 1, n - 1], np.random.default_rng(1).integers(0, n, 297)]))
    Xs = X.to(torch.float64)
    for r in rows:
        ent = chain.hamiltonian_row(L, c.J1, c.J2, c.Delta, c.h, b[r])
        cols = chain.rank(np.array(list(ent.keys()), dtype=np.uint32), b)
        vals = torch.tensor(list(ent.values()), dtype=torch.float64, device="cuda")
        ref = (vals[:, None] * Xs[torch.from_numpy(cols).cuda()]).sum(0)
        got = Y[r].to(torch.float64)
        tol = (2e-6 if dtype == np.float32 else 1e-13) * float(ref.abs().max()) + 1e-30
        assert float((got - ref).abs().max()) <= tol * 4, (r, float((got - ref).abs().max()))
    del X, Y
    torch.cuda.empty_cache()


def test_apply_h_rejects_bad_width(ctx, pf):
    c = workloads.chain(8, 1.0, 1)
    X = torch.zeros((pf.dim(8), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PolfedError):
        ctx.apply_h(_model(pf, c), X)


# --------------------------------------------------------------- filter --

def _bounds(H):
    E0, E1 = lanczos.extreme_eigenvalues(H)
    return lanczos.widened_bounds(E0, E1, 1e-3)


@pytest.mark.parametrize("K", [0, 1, 2, 3, 7, 200])
@pytest.mark.parametrize("sigma", [0.0, 0.31])
def test_filter_fp64_vs_oracle(ctx, pf, K, sigma):
    c = workloads.chain(12, 3.0, 1)
    H = chain.hamiltonian_csr(12, c.J1, c.J2, c.Delta, c.h)
    E0, E1 = _bounds(H)
    X = workloads.random_block(H.shape[0], 4, 2)
    Y = ctx.apply_filter(_model(pf, c), E0, E1, sigma, K, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = chebyshev.filter_block(H, X, E0, E1, sigma, K)
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_filter_fp64_vs_oracle_L16_J2(ctx, pf):
    c = workloads.chain(16, 2.0, 4, J2=1.0)
    H = chain.hamiltonian_csr(16, c.J1, c.J2, c.Delta, c.h)
    E0, E1 = _bounds(H)
    X = workloads.random_block(H.shape[0], 8, 3)
    Y = ctx.apply_filter(_model(pf, c), E0, E1, 0.0, 1500, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = chebyshev.filter_block(H, X, E0, E1, 0.0, 1500)
    assert np.abs(Y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_filter_on_eigenvectors(ctx, pf):
    """P(H~) v = P(lambda~) v on exact eigenvectors (closed form of P)."""
    c = workloads.chain(10, 2.0, 8, J2=0.5)
    H = chain.hamiltonian_csr(10, c.J1, c.J2, c.Delta, c.h)
    w, V = np.linalg.eigh(H.toarray())
    E0, E1 = lanczos.widened_bounds(w[0], w[-1], 1e-3)
    a, b = chebyshev.rescale_coeffs(E0, E1)
    K = 60
    Vs = np.ascontiguousarray(V[:, :64])
    Y = ctx.apply_filter(_model(pf, c), E0, E1, 0.2, K, torch.from_numpy(Vs).cuda()).cpu().numpy()
    Pw = chebyshev.P_of_x(a * w[:64] + b, 0.2, K)
    assert np.abs(Y - Vs * Pw).max() < 1e-12


@pytest.mark.parametrize("prec", [np.float64, np.float32])
def test_filter_graph_replays_match_direct(ctx, pf, prec):
    """The captured graph of a filter application, replayed several times with
    eager work in between, gives bitwise the same result as direct launches."""
    c = workloads.chain(14, 2.0, 12)
    m = _model(pf, c)
    X = torch.from_numpy(workloads.random_block(pf.dim(14), 8, 1).astype(prec)).cuda()
    E0, E1, r0, r1 = ctx.bounds(m, 200)
    E0, E1 = E0 - r0 - 0.01 * (E1 - E0), E1 + r1 + 0.01 * (E1 - E0)
    ctx.set_graphs(False)
    ref = ctx.apply_filter(m, E0, E1, 0.1, 300, X).cpu()
    assert torch.isfinite(ref).all()
    ctx.set_graphs(True)
    Y = torch.empty_like(X)
    try:
        for rep in range(3):
            ctx.apply_filter(m, E0, E1, 0.1, 300, X, out=Y)
            _ = (X * 2).sum().item()  # eager work and a sync between replays
            assert torch.equal(Y.cpu(), ref), rep
    finally:
        ctx.set_graphs(True)


@pytest.mark.parametrize("L,K,nvec", [(16, 4000, 8), (18, 20000, 4)])
def test_filter_fp32_vs_fp64(ctx, pf, L, K, nvec):
    """FP32 filter vs FP64 filter on the same FP64 input rounded to FP32:
    max over columns of ||y32 - y64|| / ||y64|| <= 1e-4."""
    c = workloads.chain(L, 3.0, 30)
    m = _model(pf, c)
    E0, E1, r0, r1 = ctx.bounds(m, 200)
    w = E1 - E0
    E0w, E1w = E0 - r0 - 1e-3 * w, E1 + r1 + 1e-3 * w
    X = workloads.random_block(pf.dim(L), nvec, 4)
    X /= np.linalg.norm(X, axis=0)
    X32 = X.astype(np.float32)
    Y64 = ctx.apply_filter(m, E0w, E1w, 0.0, K, torch.from_numpy(X32.astype(np.float64)).cuda()).cpu().numpy()
    Y32 = ctx.apply_filter(m, E0w, E1w, 0.0, K, torch.from_numpy(X32).cuda()).cpu().numpy()
    rel = np.linalg.norm(Y32 - Y64, axis=0) / np.linalg.norm(Y64, axis=0)
    print(f"FP32 filter rel err L={L} K={K}: max {rel.max():.2e}")
    assert rel.max() <= 1e-4


# ---------------------------------------------------------- dense FP64 --

@pytest.mark.parametrize("n,p,q", [(1, 1, 1), (17, 5, 3), (1000, 16, 16), (100003, 64, 32),
                                   (50001, 100, 64), (20011, 320, 16), (333, 33, 47)])
def test_gram(ctx, n, p, q):
    rng = np.random.default_rng(n + p + q)
    X = rng.standard_normal((n, p))
    Y = rng.standard_normal((n, q))
    C = ctx.gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()).cpu().numpy()
    ref = X.T @ Y
    assert np.abs(C - ref).max() <= 1e-13 * max(1.0, np.sqrt(n)) * 10


def test_gram_strided(ctx):
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((5000, 96))
    U = rng.standard_normal((5000, 16))
    Qt = torch.from_numpy(Q).cuda()
    C = ctx.gram(Qt[:, :48], torch.from_numpy(U).cuda()).cpu().numpy()
    assert np.abs(C - Q[:, :48].T @ U).max() < 1e-11


def test_gram_deterministic(ctx):
    rng = np.random.default_rng(1)
    X = torch.from_numpy(rng.standard_normal((200003, 64))).cuda()
    a = ctx.gram(X, X).cpu().numpy()
    b = ctx.gram(X, X).cpu().numpy()
    assert (a == b).all()


@pytest.mark.parametrize("n,p,q,beta", [(1, 1, 1, 0.0), (1000, 16, 16, 1.0), (100003, 64, 32, -0.5),
                                        (3001, 320, 64, 1.0), (777, 7, 45, 0.0)])
def test_update(ctx, n, p, q, beta):
    rng = np.random.default_rng(n + p)
    X = rng.standard_normal((n, p))
    C = rng.standard_normal((p, q))
    Y0 = rng.standard_normal((n, q))
    Yt = torch.from_numpy(Y0.copy()).cuda()
    ctx.update(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(), Yt, alpha=-1.5, beta=beta)
    ref = -1.5 * X @ C + beta * Y0
    assert np.abs(Yt.cpu().numpy() - ref).max() <= 1e-13 * np.sqrt(p) * 10


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 65, 200])
def test_sym_eig(ctx, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V = ctx.sym_eig(torch.from_numpy(A).cuda())
    w, V = w.cpu().numpy(), V.cpu().numpy()
    wr = np.linalg.eigvalsh(A)
    scale = np.abs(wr).max()
    assert np.abs(w - wr).max() <= 1e-13 * scale * max(1, n / 10)
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-12
    assert np.abs(A @ V - V * w).max() <= 1e-12 * scale * max(1, n / 10)


def test_sym_eig_degenerate(ctx):
    """Repeated eigenvalues (the block structure of T_m can produce them)."""
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((40, 40)))
    d = np.repeat([1.0, -2.0, 0.5, 3.0], 10)
    A = (Q * d) @ Q.T
    A = 0.5 * (A + A.T)
    w, V = ctx.sym_eig(torch.from_numpy(A).cuda())
    assert np.abs(w.cpu().numpy() - np.sort(d)).max() < 1e-13
    V = V.cpu().numpy()
    assert np.abs(A @ V - V * w.cpu().numpy()).max() < 1e-12


# --------------------------------------------------------------- bounds --

@pytest.mark.parametrize("L,J2", [(12, 0.0), (14, 1.0), (18, 1.0)])
def test_bounds(ctx, pf, L, J2):
    c = workloads.chain(L, 2.0, 2, J2=J2)
    H = chain.hamiltonian_csr(L, c.J1, c.J2, c.Delta, c.h)
    E0x, E1x = lanczos.extreme_eigenvalues(H)
    E0, E1, r0, r1 = ctx.bounds(_model(pf, c), 200)
    # Lanczos Ritz values lie inside the spectrum; their residual bounds
    # cover the distance to the true extremes
    assert E0x - 1e-9 <= E0 <= E0x + r0 + 1e-9
    assert E1x - r1 - 1e-9 <= E1 <= E1x + 1e-9
    assert abs(E0 - E0x) < 1e-6 * abs(E0x) and abs(E1 - E1x) < 1e-6 * abs(E1x)


def test_filter_fp32_vs_fp64_at_the_l22_order(ctx, pf):
    """The L=22 workload's own filter (its chain, widened Lanczos bounds, the
    target at the middle of the spectrum, the order K the solve picks for
    N_win = 150, block width 32): the FP32 filter matches the FP64 one to
    1e-4 relative per column, and the FP64 filter is symmetric (X^T P X)."""
    wl = workloads.c3("fp32")
    c = wl.chains[0]
    m = _model(pf, c)
    n = pf.dim(c.L)
    E0, E1, r0, r1 = ctx.bounds(m, 200)
    w = E1 - E0
    E0w, E1w = E0 - r0 - 1e-3 * w, E1 + r1 + 1e-3 * w
    sig = (2.0 * (E0 + 0.5 * w) - (E0w + E1w)) / (E1w - E0w)
    K, _ = pf.filter_order(m, E0w, E1w, sig, 150)
    assert 20000 < K < 80000
    g = torch.Generator(device="cuda").manual_seed(3)
    X = torch.randn((n, 32), generator=g, device="cuda", dtype=torch.float64)
    X /= X.norm(dim=0)
    Y64 = ctx.apply_filter(m, E0w, E1w, sig, K, X)
    Y32 = ctx.apply_filter(m, E0w, E1w, sig, K, X.to(torch.float32)).to(torch.float64)
    rel = ((Y32 - Y64).norm(dim=0) / Y64.norm(dim=0)).max().item()
    print(f"L=22 K={K}: FP32 vs FP64 filter, max column relative difference {rel:.2e}")
    assert rel <= 1e-4
    G = (X.T @ Y64).cpu().numpy()
    assert np.abs(G - G.T).max() <= 1e-10 * np.abs(G).max()
    del X, Y64, Y32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,shape", [(0, (256, 2, 2, 1, 0, 0, 4)), (1, (512, 2, 2, 1, 0, 0, 2))])
def test_filter_l26_bench_shape_sampled_rows(ctx, pf, prec, shape):
    """The L = 26 chain (10,400,600 rows, 64 columns) through the filter in
    the launch configuration the benchmark times (XCD column slices: four of
    16 columns in FP64, two of 32 in FP32): Y = sum_k c_k T_k(H~) X / D at
    K = 2, i.e. (c_0 X + c_1 H~X + c_2 (2 H~^2 X - X)) / D, on 100 sampled
    rows against the oracle's per-row form of H (H~^2 X through the rows of
    each sampled row's neighbours), coefficients from the oracle."""
    c = workloads.c5().chains[0]
    m = _model(pf, c)
    L, n, s = 26, pf.dim(26), 64
    E0w, E1w = -0.9 * L - 0.5 * float(np.abs(c.h).sum()), 0.8 * L + 0.5 * float(np.abs(c.h).sum())
    a, b = chebyshev.rescale_coeffs(E0w, E1w)
    sig = 0.013
    K = 2
    cc = chebyshev.cheb_coeffs(sig, K)
    D = chebyshev.norm_D(sig, K)
    saved = ctx.get_step_shape(L, s, prec)
    g = torch.Generator(device="cuda").manual_seed(26)
    X = torch.randn((n, s), generator=g, device="cuda", dtype=torch.float64)
    if prec:
        X = X.float()
    try:
        ctx.set_step_shape(L, s, prec, *shape)
        Y = ctx.apply_filter(m, E0w, E1w, sig, K, X)
        torch.cuda.synchronize()
    finally:
        ctx.set_step_shape(L, s, prec, *saved)
    bas = chain.basis(L)
    Xs = X.to(torch.float64)

    def ht_row(state):  # {rank: H~ entry} of one row
        ent = chain.hamiltonian_row(L, c.J1, c.J2, c.Delta, c.h, state)
        cols = chain.rank(np.array(list(ent.keys()), dtype=np.uint32), bas)
        vals = a * np.array(list(ent.values()))
        r0 = int(chain.rank(np.array([state], dtype=np.uint32), bas)[0])
        vals[list(cols).index(r0)] += b
        return cols, vals

    def htx(cols, vals):
        return (torch.tensor(vals, device="cuda")[:, None] *
                Xs[torch.from_numpy(cols.astype(np.int64)).cuda()]).sum(0)

    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(3).integers(0, n, 98)]))
    worst = 0.0
    for r in rows:
        cols, vals = ht_row(bas[r])
        h1 = htx(cols, vals)
        h2 = torch.zeros(s, dtype=torch.float64, device="cuda")
        for cj, vj in zip(cols, vals):
            cj2, vj2 = ht_row(bas[cj])
            h2 += vj * htx(cj2, vj2)
        ref = (cc[0] * Xs[r] + cc[1] * h1 + cc[2] * (2.0 * h2 - Xs[r])) / D
        err = float((Y[r].to(torch.float64) - ref).abs().max() / ref.abs().max())
        worst = max(worst, err)
    print(f"L=26 filter K=2, shape {shape}: worst sampled-row error {worst:.2e}")
    assert worst <= (1e-5 if prec else 1e-12)
    del X, Y, Xs
    torch.cuda.empty_cache()
