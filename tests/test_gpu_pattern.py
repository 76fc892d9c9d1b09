"""The stored-pattern form of H~ V (the paper's own matrix form: column
indices only, the values J/2 implied) and the paper's J1-J2 benchmark
model (J2 = 1, Delta = 0.55) at the L = 20 size of its timing table."""

import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chain  # noqa: E402
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


@pytest.mark.parametrize("L,J2,Delta,nvec", [(12, 1.0, 0.55, 4), (16, 1.0, 0.55, 16), (16, 0.0, 1.0, 8)])
def test_stored_pattern_apply_h_vs_oracle(ctx, L, J2, Delta, nvec):
    """H X with neighbours from the stored pattern against the oracle's CSR
    H (FP64, 1e-13 of the largest entry)."""
    from paper_2005_09534_amd import polfed as pf
    c = workloads.chain(L, 3.0, 50 + L, J2=J2, Delta=Delta)
    m = pf.make_model(L, c.J1, c.J2, c.Delta, c.h)
    H = chain.hamiltonian_csr(L, c.J1, c.J2, c.Delta, c.h)
    X = workloads.random_block(H.shape[0], nvec, L)
    saved = ctx.get_step_shape(L, nvec, 0)
    try:
        ctx.set_step_shape(L, nvec, 0, *saved[:5], 2)
        Y = ctx.apply_h(m, torch.from_numpy(X).cuda()).cpu().numpy()
    finally:
        ctx.set_step_shape(L, nvec, 0, *saved)
    ref = H @ X
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_paper_j1j2_point_l20(ctx):
    """L = 20 J1-J2 (J2 = 1, Delta = 0.55), N_ev = 100 at the middle of the
    spectrum, FP64, s = 16: the solve with neighbours from the stored pattern
    returns bit for bit the solve with on-the-fly ranks (the same terms in
    the same order); status OK and every residual, recomputed here with the
    oracle's CSR H, within 1e-8 ||H||."""
    from paper_2005_09534_amd import polfed as pf
    wl = workloads.j1j2_paper(20, 100)
    c = wl.chains[0]
    m = pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h)
    out = {}
    saved = ctx.get_step_shape(20, wl.block, 0)
    try:
        for mode in (0, 2):
            ctx.set_step_shape(20, wl.block, 0, *saved[:5], mode)
            t0 = time.time()
            r = ctx.solve(m, wl.nev, block_size=wl.block, vectors=True)
            i = r["info"]
            print(f"rank mode {mode}: status {r['status']} in {time.time() - t0:.1f} s, K {i['K']}, "
                  f"m {i['m']}, filter {i['filter_gpu_s']:.1f} s", flush=True)
            assert r["status"] == pf.OK
            out[mode] = r
    finally:
        ctx.set_step_shape(20, wl.block, 0, *saved)
    assert np.array_equal(out[0]["E"], out[2]["E"])
    H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
    normH = out[0]["info"]["normH"]
    V = out[2]["V"]
    res = np.linalg.norm(H @ V - V * out[2]["E"], axis=0)
    assert res.max() <= 1e-8 * normH
