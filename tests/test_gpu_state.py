"""Checkpoint and resume through the C ABI: a saved state restored into the
same handle (or a fresh one of the same batch layout) continues bit for bit
as the run it was saved from; a blob of another layout is refused.  The
colouring's starting colours (the previous step's colours, kept beside the
contact cache) are not part of the state and differ between these runs: the
results must not depend on them."""
import numpy as np
import pytest

from helpers import DT, S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def snap(sim):
    import torch
    torch.cuda.synchronize()
    cnt, key, lam = sim.cache()
    return [x.cpu().numpy().copy() for x in (sim.pose, sim.vel, sim.theta, cnt, key, lam)]


@pytest.mark.parametrize("persistent", [False, True])
def test_save_load_roundtrip(torch_cuda, persistent):
    torch = torch_cuda
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_clutter(12, seed0=10000)
    acts = torch.as_tensor(np.stack([S.arm_actions(3, 12, t) for t in range(60)]), device="cuda:0")
    sim = Sim(b, max_contacts=512, max_pairs=512, warm=L.PREV, tol=1e-4)
    if persistent:
        sim.set_persistent(True)
    for t in range(40):
        sim.step(acts[t], DT, 20)
    blob = sim.save_state()
    for t in range(40, 55):
        sim.step(acts[t], DT, 20)
    ref = snap(sim)
    sim.load_state(blob)
    for t in range(40, 55):
        sim.step(acts[t], DT, 20)
    got = snap(sim)
    for a, g in zip(ref, got):
        assert np.array_equal(a, g)
    # a fresh handle of the same layout resumes the same way
    sim2 = Sim(b, max_contacts=512, max_pairs=512, warm=L.PREV, tol=1e-4)
    sim2.load_state(blob)
    for t in range(40, 55):
        sim2.step(acts[t], DT, 20)
    for a, g in zip(ref, snap(sim2)):
        assert np.array_equal(a, g)
    # another layout is refused
    other = Sim(S.batch_clutter(4, seed0=10000), max_contacts=512, max_pairs=512)
    with pytest.raises(L.SimError):
        other.load_state(blob)
