"""The gradient entry point that allocates nothing (sim_mlp_grad_noalloc)
against the workspace one (sim_mlp_grad), through the C ABI: the same
kernels on the same rows must give the same gradient and loss bit for bit,
on two calls in a row (the second with fewer rows, so that partial sums
left in the static scratch by the first call must not leak into it), and a
batch beyond the static scratch is refused before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_net(torch, seed):
    from paper_2106_14405_amd import mlp as M
    rng = np.random.default_rng(seed)
    p = M.init_params(seed)
    for k in ("b1", "b2", "b3"):
        a, b, _ = M.SLICES[k]
        p[a:b] = (rng.normal(size=b - a) * 0.1).astype(np.float32)
    net = M.Net(device="cuda:0", params=p)
    net.mean.copy_(torch.as_tensor(rng.normal(size=16).astype(np.float32)))
    net.std.copy_(torch.as_tensor((0.2 + rng.random(16) * 3).astype(np.float32)))
    return net


def rows_and_targets(torch, seed, n):
    rng = np.random.default_rng(seed)
    x = torch.as_tensor((rng.normal(size=(n, 16)) * 2.0).astype(np.float32), device="cuda:0")
    t = torch.as_tensor(rng.normal(size=(n, 3)).astype(np.float32), device="cuda:0")
    return x, t


def test_noalloc_grad_equals_workspace_grad(torch_cuda):
    torch = torch_cuda
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    cap = int(lib.sim_mlp_grad_noalloc_max_rows())
    assert cap == 16384
    net = make_net(torch, 11)
    x, t = rows_and_targets(torch, 12, 40000)
    perm = np.random.default_rng(13).permutation(40000).astype(np.int32)
    # first call: the full static scratch, gathered rows; second: fewer rows, no gather
    for n, rows in ((cap, torch.as_tensor(perm[:cap], device="cuda:0")), (777, None)):
        print(f"noalloc gradient: n={n} rows={'gathered' if rows is not None else 'contiguous'}", flush=True)
        g_ref = net.compute_grad(x, t, rows, n=n).clone()
        l_ref = net.loss.clone()
        net.grad.fill_(float("nan"))
        net.loss.fill_(float("nan"))
        g_new = net.compute_grad_noalloc(x, t, rows, n=n).clone()
        l_new = net.loss.clone()
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all()
        assert torch.equal(g_new, g_ref), f"n={n}: gradients differ"
        assert torch.equal(l_new, l_ref), f"n={n}: losses differ"


def test_noalloc_grad_rejects_oversized_batch(torch_cuda):
    torch = torch_cuda
    from paper_2106_14405_amd import _lib as L
    net = make_net(torch, 21)
    cap = int(L.load().sim_mlp_grad_noalloc_max_rows())
    x, t = rows_and_targets(torch, 22, cap + 1)
    with pytest.raises(L.SimError, match="static scratch"):
        net.compute_grad_noalloc(x, t)
    with pytest.raises(L.SimError):
        net.compute_grad_noalloc(x, t, n=0)
