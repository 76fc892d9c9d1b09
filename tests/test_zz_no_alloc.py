"""polfed_gram_static, the Gram product for callers that cannot allocate:
through the C ABI, against polfed_gram (the same product with the
context's workspace) and a NumPy product, on two calls in a row -- the
second one smaller, on the fixed device array the first one filled -- plus
the empty case and the size limit."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_09534_amd import polfed as pf
    c = pf.Context(0)
    yield c
    c.close()


def _case(ctx, n, p, q, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn((n, p), generator=g, device="cuda", dtype=torch.float64)
    Y = torch.randn((n, q), generator=g, device="cuda", dtype=torch.float64)
    ref = ctx.gram(X, Y)
    out = torch.full((p, q), float("nan"), dtype=torch.float64, device="cuda")
    got = ctx.gram_static(X, Y, out)
    torch.cuda.synchronize()
    exact = X.cpu().numpy().T @ Y.cpu().numpy()
    scale = np.abs(X.cpu().numpy()).T @ np.abs(Y.cpu().numpy())  # rounding scale per entry
    g_np, r_np = got.cpu().numpy(), ref.cpu().numpy()
    assert np.all(np.isfinite(g_np))
    assert np.abs(g_np - r_np).max() <= 1e-13 * scale.max()
    assert np.abs(g_np - exact).max() <= 1e-13 * scale.max()
    return g_np


def test_gram_static_two_calls_second_smaller(ctx):
    big = _case(ctx, 705432, 640, 64, 1)     # the chunk count limited by the array (51 of 102)
    small = _case(ctx, 48620, 24, 16, 2)     # the array still holds the first call's tiles
    assert big.shape == (640, 64) and small.shape == (24, 16)


def test_gram_static_empty_and_limit(ctx):
    from paper_2005_09534_amd import polfed as pf
    X = torch.zeros((0, 8), dtype=torch.float64, device="cuda")
    Y = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    out = torch.full((8, 4), 7.0, dtype=torch.float64, device="cuda")
    ctx.gram_static(X, Y, out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    # p * q beyond the fixed array (2^21 doubles): refused, output untouched
    Xb = torch.zeros((4, 4096), dtype=torch.float64, device="cuda")
    Yb = torch.zeros((4, 1024), dtype=torch.float64, device="cuda")
    ob = torch.full((4096, 1024), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PolfedError) as e:
        ctx.gram_static(Xb, Yb, ob)
    assert e.value.code == pf.EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((ob == 3.0).all())
