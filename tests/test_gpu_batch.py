"""Batched solves (many realisations, mixed L) through polfed_solve_batch.

Each member must equal the single solve of the same chain (same seed and
block size: eigenvalues within 1e-10 ||H||) and the dense definition; the
eigenvector layout is the concatenation of per-member column-major blocks.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import chain, dense, lanczos  # noqa: E402
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


def _members(R, Ls=(10, 12, 14)):
    out = []
    for r in range(R):
        L = Ls[r % len(Ls)]
        W = float(1 + (r // len(Ls)) % 5)
        out.append(workloads.chain(L, W, 2000 + r))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_single_and_dense(ctx, pf, precision):
    chains = _members(9)
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    nev, s = 10, 4
    res = ctx.solve_batch(models, nev, vectors=True, block_size=s, precision=precision)
    assert all(st == pf.OK for st in res["status"]), res["status"]
    for i, c in enumerate(chains):
        H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
        w = dense.full_spectrum(H)
        normH = max(abs(w[0]), abs(w[-1]))
        sig = res["info"][i]["sigma_energy"]
        Ed = w[dense.nearest_from_spectrum(w, sig, nev)]
        assert np.abs(res["E"][i] - Ed).max() <= 1e-10 * normH, i
        V = res["V"][i]
        r = np.linalg.norm(H @ V - V * res["E"][i], axis=0)
        assert r.max() <= 1e-8 * normH, (i, r.max())
        single = ctx.solve(models[i], nev, block_size=s, precision=precision)
        assert np.abs(single["E"] - res["E"][i]).max() <= 1e-10 * normH, i
        assert single["info"]["K"] == res["info"][i]["K"]


def test_batch_mixed_status_and_layout(ctx, pf):
    """One member of the batch cannot converge (tiny space); the others are
    unaffected, and statuses are reported per member."""
    good = workloads.chain(12, 2.0, 77)
    tiny = workloads.chain(8, 6.0, 106, J2=1.0)
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in (good, tiny, good)]
    res = ctx.solve_batch(models, 8, vectors=True, block_size=8)
    assert res["status"][0] == pf.OK and res["status"][2] == pf.OK
    assert res["status"][1] == pf.NOT_CONVERGED
    assert res["rc"] == pf.NOT_CONVERGED
    assert np.array_equal(res["E"][0], res["E"][2])
    assert res["V"][0].shape == (pf.dim(12), 8) and res["V"][1].shape == (pf.dim(8), 8)


def test_batched_workload_members_fp32(ctx, pf):
    """Members of the 512-realisation batch (its L = 14 ones, N_ev = 20, FP32
    filter, block size 8 as tuned) through polfed_solve_batch: every status
    OK, residuals under the FP32 bar, eigenvalues equal to dense ones."""
    wl = workloads.c4(24)
    chains = [c for c in wl.chains if c.L == 14][:5]
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    res = ctx.solve_batch(models, wl.nev, vectors=True, block_size=8, precision=1)
    assert all(st == pf.OK for st in res["status"]), res["status"]
    for i, c in enumerate(chains):
        H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
        w = dense.full_spectrum(H)
        normH = max(abs(w[0]), abs(w[-1]))
        Ed = w[dense.nearest_from_spectrum(w, res["info"][i]["sigma_energy"], wl.nev)]
        assert np.abs(res["E"][i] - Ed).max() <= 1e-10 * normH, i
        V = res["V"][i]
        r = np.linalg.norm(H @ V - V * res["E"][i], axis=0)
        assert r.max() <= 1e-8 * normH, (i, r.max())


def test_batched_workload_l14_sample_vs_dense(ctx, pf):
    """A wider sample of the 512-realisation batch: 24 of its L = 14 members
    (every fields strength W = 1..5), solved as one FP32 batch with the tuned
    block size, each against the dense spectrum: the 20 eigenvalues nearest
    the target, none skipped, residuals under the bar."""
    wl = workloads.c4()
    chains = [c for c in wl.chains if c.L == 14][::7][:24]
    assert sorted({c.W for c in chains}) == [1.0, 2.0, 3.0, 4.0, 5.0]
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    res = ctx.solve_batch(models, wl.nev, vectors=False, block_size=8, precision=1)
    assert all(st == pf.OK for st in res["status"]), res["status"]
    for i, c in enumerate(chains):
        H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
        w = dense.full_spectrum(H)
        normH = max(abs(w[0]), abs(w[-1]))
        Ed = w[dense.nearest_from_spectrum(w, res["info"][i]["sigma_energy"], wl.nev)]
        assert np.abs(res["E"][i] - Ed).max() <= 1e-10 * normH, (i, c.seed)
        assert res["resid"][i].max() <= 1e-8 * normH, (i, c.seed)


def test_batch_rejects_empty_and_oversized(ctx, pf):
    """An empty batch and an N_ev above a member's dimension are argument
    errors (nothing is computed)."""
    with pytest.raises(pf.PolfedError):
        ctx.solve_batch([], 4, block_size=4)
    small = workloads.chain(6, 1.0, 3)  # dim 20
    big = workloads.chain(10, 1.0, 4)
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in (big, small)]
    with pytest.raises(pf.PolfedError):
        ctx.solve_batch(models, 21, block_size=4)


@pytest.mark.parametrize("precision", [0, 1])
def test_narrow_window_is_widened(ctx, pf, precision):
    """A realisation of the 512-member batch (L = 14, W = 5) whose Gaussian-DOS
    window holds only 18 eigenvalues above p for N_ev = 20: both the batched
    and the single solve repeat it with the window sized for twice as many
    eigenvalues (info nev_window 60 instead of 30) and return the 20
    eigenvalues nearest the target, while the members around it keep their
    window."""
    narrow = workloads.chain(14, 5.0, 1207)
    others = [workloads.chain(14, 2.0, 1003), workloads.chain(14, 3.0, 1006)]
    chains = [others[0], narrow, others[1]]
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    nev = 20
    res = ctx.solve_batch(models, nev, vectors=True, block_size=8, precision=precision)
    assert all(st == pf.OK for st in res["status"]), res["status"]
    assert [i["nev_window"] for i in res["info"]] == [30, 60, 30]
    for i, c in enumerate(chains):
        H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
        w = dense.full_spectrum(H)
        normH = max(abs(w[0]), abs(w[-1]))
        Ed = w[dense.nearest_from_spectrum(w, res["info"][i]["sigma_energy"], nev)]
        assert np.abs(res["E"][i] - Ed).max() <= 1e-10 * normH, i
        V = res["V"][i]
        assert V.shape == (H.shape[0], nev)
        r = np.linalg.norm(H @ V - V * res["E"][i], axis=0)
        assert r.max() <= 1e-8 * normH, (i, r.max())
    single = ctx.solve(models[1], nev, block_size=8, precision=precision)
    assert single["status"] == pf.OK and single["info"]["nev_window"] == 60
    H = chain.hamiltonian_csr(narrow.L, narrow.J1, narrow.J2, narrow.Delta, narrow.h)
    w = dense.full_spectrum(H)
    normH = max(abs(w[0]), abs(w[-1]))
    assert np.abs(single["E"] - res["E"][1]).max() <= 1e-10 * normH


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_mixes_j2_at_one_length(ctx, pf, precision):
    """Two L = 12 members, one without and one with next-nearest couplings,
    in one batch: each must get its own bond set in the batched filter (the
    batch groups members by whether J2 is zero) and equal the dense answer."""
    chains = [workloads.chain(12, 2.0, 71), workloads.chain(12, 2.0, 72, J2=1.0, Delta=0.55)]
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    nev = 8
    res = ctx.solve_batch(models, nev, vectors=True, block_size=4, precision=precision)
    assert res["status"] == [pf.OK, pf.OK]
    for i, c in enumerate(chains):
        H = chain.hamiltonian_csr(c.L, c.J1, c.J2, c.Delta, c.h)
        w = dense.full_spectrum(H)
        normH = max(abs(w[0]), abs(w[-1]))
        Ed = w[dense.nearest_from_spectrum(w, res["info"][i]["sigma_energy"], nev)]
        assert np.abs(res["E"][i] - Ed).max() <= 1e-10 * normH, i
        V = res["V"][i]
        assert np.linalg.norm(H @ V - V * res["E"][i], axis=0).max() <= 1e-8 * normH, i


def test_batch_member_error_leaves_the_others(ctx, pf):
    """A member whose target lies outside its own spectrum fails alone: its
    status is POLFED_EINVAL and its outputs stay untouched, the others are
    solved, and the call returns POLFED_NOT_CONVERGED (a warning)."""
    good = workloads.chain(10, 2.0, 81)
    narrow = workloads.chain(10, 0.05, 82, J1=0.05)   # spectrum within about +-0.3
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in (good, narrow, good)]
    H = chain.hamiltonian_csr(good.L, good.J1, good.J2, good.Delta, good.h)
    w = dense.full_spectrum(H)
    normH = max(abs(w[0]), abs(w[-1]))
    sigma = w[0] + 0.3 * (w[-1] - w[0])       # inside the first spectrum only
    assert sigma < -1.0
    res = ctx.solve_batch(models, 6, vectors=False, block_size=2, target_kind=1, target=sigma)
    assert res["status"][1] == pf.EINVAL
    assert np.isnan(res["E"][1]).all() and np.isnan(res["resid"][1]).all()  # untouched
    assert res["status"][0] == pf.OK and res["status"][2] == pf.OK
    assert res["rc"] == pf.NOT_CONVERGED
    Ed = w[dense.nearest_from_spectrum(w, sigma, 6)]
    for i in (0, 2):
        assert np.abs(res["E"][i] - Ed).max() <= 1e-10 * normH


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_length_launch_equals_separate_batches(ctx, pf, precision):
    """Realisations of different L with one block size share every batched
    launch (each brings its own basis; tile ranges per realisation): the
    mixed batch returns what the per-L batches return (eigenvalues within
    1e-10 ||H||, same K), and FP32 members go through the batched FP64
    refinement in both."""
    chains = _members(12, Ls=(10, 12, 14, 16))
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    nev, s = 8, 4
    mixed = ctx.solve_batch(models, nev, vectors=False, block_size=s, precision=precision)
    assert all(st == pf.OK for st in mixed["status"]), mixed["status"]
    for L in (10, 12, 14, 16):
        idx = [i for i, c in enumerate(chains) if c.L == L]
        sep = ctx.solve_batch([models[i] for i in idx], nev, vectors=False, block_size=s,
                              precision=precision)
        for k, i in enumerate(idx):
            normH = mixed["info"][i]["normH"]
            assert np.abs(sep["E"][k] - mixed["E"][i]).max() <= 1e-10 * normH, (L, i)
            assert sep["info"][k]["K"] == mixed["info"][i]["K"]
    if precision == 1:
        assert max(i["refine_passes"] for i in mixed["info"]) >= 1


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_column_slices_bitwise(ctx, pf, precision):
    """The batched kernel with its block split into XCD column slices (the
    recurrence buffers slice-major) computes the same numbers as unsplit: a
    batch at s = 32 (FP64 filter), and the FP64 refinement filters of an
    FP32 batch (width 32 or 64), give identical eigenvalues with 1 and with
    4 slices."""
    chains = [workloads.chain(12, 2.0, 3100 + r) for r in range(3)]
    models = [pf.make_model(c.L, c.J1, c.J2, c.Delta, c.h) for c in chains]
    keys = [(12, 32, 0), (12, 64, 0)] if precision == 1 else [(12, 32, 0)]
    saved = {k: ctx.get_batch_shape(*k) for k in keys}
    out = {}
    try:
        for ns in (1, 4):
            for k in keys:
                sh = saved[k]
                ctx.set_batch_shape(*k, *sh[:5], ns)
            s = 8 if precision == 1 else 32
            r = ctx.solve_batch(models, 40, vectors=False, block_size=s, precision=precision)
            assert all(st == pf.OK for st in r["status"]), r["status"]
            out[ns] = r
    finally:
        for k in keys:
            ctx.set_batch_shape(*k, *saved[k])
    assert np.array_equal(out[1]["E"], out[4]["E"])
    if precision == 1:
        assert max(i["refine_passes"] for i in out[4]["info"]) >= 1
