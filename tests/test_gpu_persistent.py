"""The persistent launch for batches of uneven scene sizes.

Scenes are routed to whole-workgroup teams (256 threads, all the LDS) or to
single-wave teams (a quarter of the LDS each), taken from two queues in
descending size by one persistent launch replayed from a HIP graph.  Its
results must equal the one-workgroup-per-scene launch bit for bit, step
after step (graph replays, both cache parities, resets), in every warm-start
mode; against the oracle it must meet the usual parity bar; the autotuner
must leave the state as it found it.
"""
import numpy as np
import pytest

from gpu_util import compare, gpu_results, gpu_sim, oracle_warmup, report, snapshot32
from helpers import DT, S
from oracle import oracle as O

pytestmark = pytest.mark.gpu

CAP = 2048  # batch-wide pair/contact capacity: 4 per body at 512 bodies (6 per body below 341)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make(batch, warm, persistent, wave_max=128, tol=1e-4):
    from paper_2106_14405_amd.sim import Sim
    sim = Sim(batch, max_pairs=CAP, max_contacts=CAP, warm=warm, tol=tol, threads=64)
    if persistent:
        sim.set_persistent(True, wave_max)
    return sim


def state(sim):
    import torch
    torch.cuda.synchronize()
    cnt, key, lam = sim.cache()
    return dict(pose=sim.pose.cpu().numpy().copy(), vel=sim.vel.cpu().numpy().copy(),
                count=cnt.cpu().numpy().copy(), key=key.cpu().numpy().copy(), lam=lam.cpu().numpy().copy(),
                **{k: v.cpu().numpy().copy() for k, v in sim.stats.items()})


def assert_same(a, b, where):
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{where}: {k} differs"


@pytest.mark.parametrize("warm", [O.COLD, O.PREV, O.LEARNED])
def test_persistent_equals_plain(torch_cuda, warm):
    torch = torch_cuda
    b = S.batch_uneven(40, seed0=20000, lo=16, hi=512)
    counts = b.counts()
    assert counts.max() > 256 and counts.min() < 48
    sims = [make(b, warm, False), make(b, warm, True)]
    if warm == O.LEARNED:
        from paper_2106_14405_amd import mlp as M
        net = M.Net(device="cuda:0", seed=3)
        net.std.fill_(2.0)
        for sm in sims:
            net.attach(sm)
    for t in range(70):
        for sm in sims:
            sm.step(None, DT, 30)
        if t % 10 == 9 or t == 69:
            assert_same(state(sims[0]), state(sims[1]), f"step {t}")
    st = state(sims[1])
    assert st["contacts"].sum() > 1000  # the late steps are contact-rich


def test_persistent_resets_and_replays(torch_cuda):
    """Graph replays over both cache parities with masked resets in between."""
    torch = torch_cuda
    b = S.batch_uneven(32, seed0=20100, lo=16, hi=512)
    sims = [make(b, O.PREV, False), make(b, O.PREV, True, wave_max=64)]
    pose0 = torch.tensor(b.pose.T.copy(), device="cuda:0").contiguous()
    vel0 = torch.tensor(b.vel.T.copy(), device="cuda:0").contiguous()
    rng = np.random.default_rng(5)
    for t in range(90):
        if t in (40, 65):
            mask = torch.tensor(rng.random(b.n_scenes) < 0.4, device="cuda:0")
            for sm in sims:
                sm.reset(mask, pose0, vel0)
        for sm in sims:
            sm.step(None, DT, 20)
    assert_same(state(sims[0]), state(sims[1]), "after resets")


def test_persistent_oracle_parity(torch_cuda):
    """One step of a settled uneven batch through the persistent launch
    against the oracle (keys bit-exact, values within 1e-4)."""
    b = S.batch_uneven(4, seed0=20200, lo=16, hi=128)
    ora = oracle_warmup(b, 60)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, max_contacts=CAP, max_pairs=CAP, warm=O.PREV, tol=1e-5, threads=64)
    sim.set_persistent(True, 48)
    sim.step(None, DT, 200)
    r = ora.step(iters=200, tol=1e-5, warm=O.PREV, max_pairs=CAP, max_contacts=CAP)
    rep = compare(b, gpu_results(sim), r, ora, contact_values=True, tol_band=0.02)
    report("persistent launch, tolerance 1e-5", rep)
    assert rep["contacts"] > 30


def test_autotune_keeps_state(torch_cuda):
    torch = torch_cuda
    b = S.batch_uneven(48, seed0=20300, lo=16, hi=512)
    sims = [make(b, O.PREV, False), make(b, O.PREV, True)]
    for t in range(50):
        for sm in sims:
            sm.step(None, DT, 20)
    before = state(sims[1])
    best = sims[1].autotune(steps=3, dt=DT, iters=20)
    # a routing table over the body-count buckets present (16 to 512 bodies: buckets 0..5)
    assert 0 <= best < (1 << 6)
    after = state(sims[1])
    for k in ("pose", "vel", "count", "key", "lam"):
        assert np.array_equal(before[k], after[k]), k
    for t in range(5):
        for sm in sims:
            sm.step(None, DT, 20)
    assert_same(state(sims[0]), state(sims[1]), "after autotune")
    # any stored table routes the same batch to the same bits
    for mask in (0, 0b000111, 0b111111):
        sims[1].set_persistent_table(mask)
        for t in range(3):
            for sm in sims:
                sm.step(None, DT, 20)
        assert_same(state(sims[0]), state(sims[1]), f"table {mask:06b}")
