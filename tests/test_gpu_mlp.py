"""GPU parity of the learned warm start's network kernels against the oracle.

Forward: the matrix-core inference (the routine the step runs) against the
oracle's bf16-emulating forward, |dy| <= 4e-3 (|y| + 1).  Gradient: against
the oracle's FP64 backward on the same bf16-rounded forward, cosine >= 0.999
and relative L2 <= 1e-2 per tensor.  Adam: against the oracle's update.
Export: bit-exact bf16 rounding.  The learned step: one step of settled drop
scenes in LEARNED mode against the oracle's learned step.
"""
import numpy as np
import pytest

from gpu_util import compare, gpu_results, gpu_sim, oracle_warmup, snapshot32
from helpers import DT, S
from oracle import oracle as O

pytestmark = pytest.mark.gpu

NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def random_net(seed):
    """Flat float32 parameters with nonzero biases, and feature statistics."""
    from paper_2106_14405_amd import mlp as M
    rng = np.random.default_rng(seed)
    p = M.init_params(seed)
    for k in ("b1", "b2", "b3"):
        a, b, _ = M.SLICES[k]
        p[a:b] = (rng.normal(size=b - a) * 0.1).astype(np.float32)
    mean = rng.normal(size=16).astype(np.float32)
    std = (0.2 + rng.random(16) * 3).astype(np.float32)
    return p, mean, std


def make_net(torch, seed):
    from paper_2106_14405_amd import mlp as M
    p, mean, std = random_net(seed)
    net = M.Net(device="cuda:0", params=p)
    net.mean.copy_(torch.as_tensor(mean))
    net.std.copy_(torch.as_tensor(std))
    net.export()
    named = M.unflatten(p)
    named["mean"] = mean.astype(np.float64)
    named["std"] = std.astype(np.float64)
    return net, named


def features(seed, n, mean, std):
    rng = np.random.default_rng(seed)
    return (mean + std * rng.normal(size=(n, 16)) * 1.5).astype(np.float32)


@pytest.mark.parametrize("n", [1, 37, 64, 1000, 4113])
def test_forward_matches_bf16_oracle(torch_cuda, n):
    torch = torch_cuda
    net, named = make_net(torch, 11)
    x = features(n, n, named["mean"], named["std"])
    y = net.forward(torch.as_tensor(x, device="cuda:0")).cpu().numpy().astype(np.float64)
    ref = O.mlp_forward(named, x.astype(np.float64), bf16=True)
    err = np.abs(y - ref) / (np.abs(ref) + 1.0)
    assert err.max() <= 4e-3, (n, err.max())
    # far from the bar on average: disagreements are isolated bf16 rounding flips
    assert np.median(err) <= 1e-5


def test_forward_empty(torch_cuda):
    torch = torch_cuda
    net, _ = make_net(torch, 12)
    y = net.forward(torch.zeros((0, 16), dtype=torch.float32, device="cuda:0"))
    assert tuple(y.shape) == (0, 3)


def test_stats_match_numpy(torch_cuda):
    torch = torch_cuda
    from paper_2106_14405_amd import mlp as M
    rng = np.random.default_rng(13)
    x = (rng.normal(size=(30011, 16)) * np.linspace(0.01, 30, 16) + np.linspace(-5, 5, 16)).astype(np.float32)
    net = M.Net(device="cuda:0")
    net.fit_stats(torch.as_tensor(x, device="cuda:0"))
    xd = x.astype(np.float64)
    assert np.all(np.abs(net.mean.cpu().numpy() - xd.mean(0)) <= 1e-6 * (np.abs(xd.mean(0)) + xd.std(0)))
    np.testing.assert_allclose(net.std.cpu().numpy(), xd.std(0), rtol=1e-6)


def _grad_named(g):
    from paper_2106_14405_amd import mlp as M
    return M.unflatten(g)


@pytest.mark.parametrize("n,subset", [(1000, False), (70, False), (2000, True)])
def test_grad_matches_oracle(torch_cuda, n, subset):
    torch = torch_cuda
    net, named = make_net(torch, 14)
    rng = np.random.default_rng(15)
    x = features(16, n, named["mean"], named["std"])
    t = (rng.normal(size=(n, 3)) * 2.0).astype(np.float32)
    xd, td = torch.as_tensor(x, device="cuda:0"), torch.as_tensor(t, device="cuda:0")
    if subset:
        rows = rng.permutation(n)[:333].astype(np.int32)
        g = net.compute_grad(xd, td, torch.as_tensor(rows, device="cuda:0")).cpu().numpy()
        xs, ts = x[rows], t[rows]
    else:
        g = net.compute_grad(xd, td).cpu().numpy()
        xs, ts = x, t
    loss = float(net.loss.item())
    loss_o, g_o = O.mlp_loss_grad(named, xs.astype(np.float64), ts.astype(np.float64), bf16=True)
    assert abs(loss - loss_o) <= 1e-3 * abs(loss_o)
    gn = _grad_named(g)
    for k in NAMES:
        a, b = gn[k].reshape(-1), g_o[k].reshape(-1)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert cos >= 0.999 and rel <= 1e-2, (k, cos, rel)


def test_grad_bitwise_reproducible(torch_cuda):
    torch = torch_cuda
    net, named = make_net(torch, 17)
    x = torch.as_tensor(features(18, 3000, named["mean"], named["std"]), device="cuda:0")
    t = torch.randn((3000, 3), generator=torch.Generator(device="cuda:0").manual_seed(0), device="cuda:0")
    g1 = net.compute_grad(x, t).clone()
    l1 = net.loss.clone()
    g2 = net.compute_grad(x, t).clone()
    assert torch.equal(g1, g2) and torch.equal(l1, net.loss)


def test_adam_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_2106_14405_amd import mlp as M
    p0, _, _ = random_net(19)
    net = M.Net(device="cuda:0", params=p0)
    rng = np.random.default_rng(20)
    p, m, v = p0.astype(np.float64), np.zeros(M.NP), np.zeros(M.NP)
    for k, scale in enumerate([0.01, 3.0, 0.02, 0.5], 1):   # the second and fourth exceed the clip norm
        g = (rng.normal(size=M.NP) * scale / np.sqrt(M.NP) * 10).astype(np.float32)
        net.grad.copy_(torch.as_tensor(g))
        lr = 1e-3 * (1 - k / 10)
        net.adam(lr, clip=0.5)
        p, m, v, _, norm = O.adam_step(p, m, v, g.astype(np.float64), k, lr, clip=0.5)
        assert abs(float(net.gnorm.item()) - norm) <= 1e-5 * norm
        got = net.params.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, p, rtol=0, atol=2e-7)
        np.testing.assert_allclose(net.m.cpu().numpy(), m, rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(net.v.cpu().numpy(), v, rtol=1e-5, atol=1e-12)


def test_export_bitexact(torch_cuda):
    torch = torch_cuda
    from paper_2106_14405_amd import mlp as M
    p, _, _ = random_net(21)
    net = M.Net(device="cuda:0", params=p)
    torch.cuda.synchronize()
    wb = net.wbf.cpu().float().numpy().astype(np.float64)
    bs = net.bias.cpu().numpy()
    w = np.concatenate([p[0:1024], p[1088:5184], p[5248:5440]])
    ref = np.array([O.bf16(float(v)) for v in w])
    np.testing.assert_array_equal(wb, ref)
    np.testing.assert_array_equal(bs, np.concatenate([p[1024:1088], p[5184:5248], p[5440:5443]]))


def test_gather_rows_match_export(torch_cuda):
    """Logged rows are the new contacts' exported features and impulses in
    units of |g| dt / k_n, scenes in order, flagged scenes skipped."""
    torch = torch_cuda
    from paper_2106_14405_amd import mlp as M
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_drop(6, seed0=40)
    sim = Sim(b, warm=O.PREV, tol=1e-6, threads=64)
    sim.set_export(True)
    for _ in range(60):
        sim.step(None, DT, 300)
    x, t = M.gather(sim)
    torch.cuda.synchronize()
    c = {k: v.cpu().numpy() for k, v in sim.contacts().items() if v is not None}
    flags = sim.stats["flags"].cpu().numpy()
    xs, ts = [], []
    for s in range(b.n_scenes):
        if flags[s]:
            continue
        nc = int(c["count"][s])
        f = c["features"][:, s, :nc].T
        new = f[:, 15] > 0
        kn = f[:, 4] + f[:, 5] + f[:, 6] + f[:, 7]
        xs.append(f[new])
        ts.append((c["lam"][:, s, :nc].T * (kn / (9.81 * DT))[:, None])[new])
    xs, ts = np.concatenate(xs), np.concatenate(ts)
    assert x.shape[0] == xs.shape[0] > 0
    np.testing.assert_array_equal(x.cpu().numpy(), xs)
    np.testing.assert_allclose(t.cpu().numpy(), ts, rtol=2e-6, atol=1e-9)
    # capped gather keeps the first rows; saturated targets
    x2, t2 = M.gather(sim, cap=3)
    assert x2.shape[0] == 3
    np.testing.assert_array_equal(x2.cpu().numpy(), xs[:3])
    _, t3 = M.gather(sim, target_clip=0.5)
    np.testing.assert_allclose(t3.cpu().numpy(), np.clip(ts, -0.5, 0.5), rtol=2e-6, atol=1e-9)


@pytest.mark.parametrize("seed,garbage", [(0, False), (1, False), (2, True)])
def test_learned_step_parity(torch_cuda, seed, garbage):
    """One LEARNED step from oracle-settled drop states (early enough for new
    contacts), solved tight; a garbage network (outputs of order 1e3) must be
    rejected for the cold start on both sides."""
    torch = torch_cuda
    b = S.batch_drop(4, seed0=60 + 4 * seed)
    ora = oracle_warmup(b, 30)
    net, named = make_net(torch, 22 + seed)
    if garbage:
        from paper_2106_14405_amd import mlp as M
        a, e, _ = M.SLICES["b3"]
        net.params[a:e] = torch.tensor([800.0, -600.0, 700.0], device="cuda:0")
        net.export()
        named["b3"] = np.array([800.0, -600.0, 700.0])
    ora.set_mlp(named, bf16=True)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=O.LEARNED, tol=1e-6, threads=64)
    net.attach(sim)
    sim.step(None, DT, 500)
    r = ora.step(iters=500, tol=1e-6, warm=O.LEARNED, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    # tolerance 1e-6 m/s is the float32 residual's rounding floor: stop
    # decisions within a factor 2 of it are ties (as for the features below)
    rep = compare(b, g, r, ora, tol_band=1.0)
    assert rep["scenes"] - rep["flagged"] >= 2 and rep["contacts"] >= 50
    fell_g = g["stats"]["flags"] & O.F_FELLBACK
    fell_o = r["flags"] & O.F_FELLBACK
    assert np.array_equal(fell_g != 0, fell_o != 0)
    if garbage:
        new = [s for s in range(b.n_scenes) if (r["c_feat"][s, :r["n_contacts"][s], 15] > 0).any()]
        assert new and all(fell_o[s] for s in new)


@pytest.mark.parametrize("warm", [O.COLD, O.PREV])
def test_features_match_oracle(torch_cuda, warm):
    """The 16 exported warm-start features of every contact, in canonical
    order, against the oracle's (settled drop scenes, one step)."""
    torch = torch_cuda
    b = S.batch_drop(4, seed0=80)
    ora = oracle_warmup(b, 40)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=warm, tol=1e-6, threads=64)
    sim.step(None, DT, 300)
    r = ora.step(iters=300, tol=1e-6, warm=warm, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    # at 1e-6 m/s the float32 residual is within a decade of its rounding
    # floor (impulses near 1 N s, 6e-8 relative, effective inverse masses
    # near 10): stop decisions within a factor 2 of the tolerance are ties
    rep = compare(b, g, r, ora, tol_band=1.0)
    assert rep["contacts"] >= 50
    for s in range(b.n_scenes):
        if r["ambiguous"][s]:
            continue
        nc = int(r["n_contacts"][s])
        fg = g["features"][:, s, :nc].T.astype(np.float64)
        fo = r["c_feat"][s, :nc]
        # velocities and impulses agree to the step's rounding; geometry terms to 1e-4 relative
        scale = np.maximum(np.abs(fo), 1.0)
        err = np.abs(fg - fo) / scale
        assert err.max() <= 1e-3, (s, err.max(axis=0))
        np.testing.assert_array_equal(fg[:, 15] > 0, fo[:, 15] > 0)
