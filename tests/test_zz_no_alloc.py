"""The allocation-free FP32 forward pass of the learned-guess network (thc_mlp_forward_noalloc)
against the allocating one (thc_mlp_forward), through the C ABI: two calls in a row, the second
with fewer rows, each equal to the allocating pass; the row limit is refused on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def thc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc as mod
    mod.load()
    return mod


def test_forward_noalloc_matches_forward(thc):
    net = thc.MLP(n_in=10, width=256, n_out=2, seed=5)
    rng = np.random.default_rng(11)
    mu_in, sd_in = rng.standard_normal(10), 0.5 + rng.random(10)
    net.set_norm(mu_in, sd_in, [0.1, -0.2], [2.0, 0.5])
    for rows in (3000, 517):  # second call smaller: stale activations of the first stay in scratch
        _say("forward_noalloc rows", rows)
        X = torch.from_numpy(rng.standard_normal((rows, 10)).astype(np.float32)).cuda()
        want = net.forward(X)
        got = torch.full((rows, 2), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        net.forward_noalloc(X, got)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] >= free0  # no device memory taken by the call
        g, w = got.cpu().numpy(), want.cpu().numpy()
        err = np.abs(g - w).max() / np.abs(w).max()
        _say("  max rel diff", err)
        assert err <= 1e-6, err  # same kernels and order of operations: agreement to FP32 rounding
    net.close()


def test_forward_noalloc_refuses_rows_beyond_scratch(thc):
    net = thc.MLP(n_in=10, width=256, n_out=2, seed=5)
    X = torch.zeros((16009, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(thc.ThcError, match="scratch capacity of 16008 rows"):
        net.forward_noalloc(X)
    ok = net.forward_noalloc(X[:16008].contiguous())
    torch.cuda.synchronize()
    assert torch.isfinite(ok).all()
    net.close()
