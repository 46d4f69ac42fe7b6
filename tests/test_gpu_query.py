"""GPU parity of the batched arm collision queries (motion planning: every
configuration a sampling planner visits is checked against the scene)
against the oracle's brute force over every (link, obstacle) pair.

Bar: the collision flag bit-exact wherever the oracle's least separation is
outside the tie band of the clearance (1e-5 m); the least separation within
1e-5 m wherever both sides found a contact inside the clearance (float32
forward kinematics of a 1.2 m chain and float32 contact geometry against
float64: errors of a few 1e-7 m).  Configurations: even ones uniform in
[-pi, pi] per joint, odd ones leaning out over the floor and furniture, 96
per scene (one full block of 64 and a ragged tail of 32)."""
import numpy as np
import pytest

from gpu_util import gpu_sim, oracle_warmup, snapshot32
from helpers import S
from oracle import oracle as O

pytestmark = pytest.mark.gpu

BAND = 1e-5
PHI_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def compare(hit_g, phi_g, hit_o, phi_o, amb_o, clearance, label):
    hit_g = hit_g.astype(bool)
    hit_o = hit_o.astype(bool)
    decided = amb_o == 0
    bad = decided & (hit_g != hit_o)
    assert not bad.any(), f"{label}: {int(bad.sum())} flags differ, first at {np.argwhere(bad)[0]}"
    both = hit_g & hit_o & (phi_o <= clearance - BAND)
    err = np.abs(phi_g[both].astype(np.float64) - phi_o[both])
    assert err.size == 0 or err.max() <= PHI_TOL, f"{label}: separation error {err.max():.3g}"
    # where no contact is within the clearance the GPU reports +inf
    assert np.all(np.isinf(phi_g[~hit_g]))
    print(f"\n{label}: {hit_o.size} configurations, {hit_o.mean():.1%} colliding, "
          f"{int((~decided).sum())} in the tie band, max separation error "
          f"{(err.max() if err.size else 0.0):.2e} m over {err.size}")
    return hit_o.mean()


def run_both(torch, b, ora, M, clearances, seed=5, scenes=None, **kw):
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, **kw)
    before = sim.pose.clone()
    q = S.arm_configurations(seed, b.n_scenes, M)
    qt = torch.as_tensor(q, device=sim.device)
    out = []
    for c in clearances:
        h, p = sim.query_arm(qt, c)
        torch.cuda.synchronize()
        hit_o, phi_o, amb_o = ora.arm_query(q.astype(np.float64), c, scenes=scenes)
        hg, pg = h.cpu().numpy(), p.cpu().numpy()
        if scenes is not None:
            sl = slice(*scenes)
            hg, pg, hit_o, phi_o, amb_o = hg[sl], pg[sl], hit_o[sl], phi_o[sl], amb_o[sl]
        out.append((hg, pg, hit_o, phi_o, amb_o, c))
    # the queries read the state and do not change it
    assert torch.equal(sim.pose, before)
    return out


@pytest.mark.parametrize("clearance", [0.0, 0.05])
def test_query_clutter_parity(torch_cuda, clearance):
    b = S.batch_clutter(16, seed0=10000)
    ora = oracle_warmup(b, 150, iters=20)
    for hg, pg, ho, po, ao, c in run_both(torch_cuda, b, ora, 96, [clearance]):
        frac = compare(hg, pg, ho, po, ao, c, f"clutter 16 scenes, clearance {c}")
        assert 0.1 < frac < 0.9


def test_query_benchmark_size_sampled(torch_cuda):
    """All 1,024 clutter scenes x 64 configurations in one launch (the size
    the benchmark times); the oracle checks every 64th scene."""
    b = S.batch_clutter(1024, seed0=10000)
    ora = O.OracleSim(b)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, max_contacts=512, max_pairs=1024)
    torch = torch_cuda
    q = S.arm_configurations(9, 1024, 64)
    h, p = sim.query_arm(torch.as_tensor(q, device=sim.device), 0.02)
    hg, pg = h.cpu().numpy(), p.cpu().numpy()
    for s in range(0, 1024, 64):
        ho, po, ao = ora.arm_query(q.astype(np.float64), 0.02, scenes=(s, s + 1))
        compare(hg[s:s + 1], pg[s:s + 1], ho[s:s + 1], po[s:s + 1], ao[s:s + 1], 0.02, f"scene {s}")


def test_query_large_scenes(torch_cuda):
    """Scenes of 1,051 bodies (beyond a workgroup's LDS for the step): the
    query keeps only the obstacle boxes in LDS and runs at any size."""
    b = S.pack([S.clutter_scene(30001 + k, n_dynamic=1024) for k in range(2)])
    ora = oracle_warmup(b, 60, iters=10)
    for hg, pg, ho, po, ao, c in run_both(torch_cuda, b, ora, 70, [0.0], max_contacts=4096, max_pairs=6144):
        compare(hg, pg, ho, po, ao, c, "1,051-body scenes")


def test_query_edge_cases(torch_cuda):
    torch = torch_cuda
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_clutter(3, seed0=10000)
    sim = Sim(b)
    h, p = sim.query_arm(torch.zeros((3, 0, 7), dtype=torch.float32, device=sim.device))
    assert h.shape == (3, 0)
    with pytest.raises(L.SimError):
        sim.query_arm(torch.zeros((3, 4, 7), dtype=torch.float32, device=sim.device), -0.1)
    with pytest.raises(L.SimError):
        sim.query_arm(torch.zeros((3, 4, 7), dtype=torch.float32, device=sim.device), float("nan"))
    nb = S.batch_drop(2, seed0=0)
    with pytest.raises(L.SimError, match="no arm"):
        Sim(nb).query_arm(torch.zeros((2, 4, 7), dtype=torch.float32, device="cuda:0"))
    # a scene with nothing but the arm: only the ground can be hit
    only = S.pack([S.clutter_scene(10000, n_static=0, n_each=0)])
    ora = O.OracleSim(only)
    sim = Sim(only)
    q = S.arm_configurations(3, 1, 130)
    h, p = sim.query_arm(torch.as_tensor(q, device=sim.device), 0.0)
    ho, po, ao = ora.arm_query(q.astype(np.float64), 0.0)
    compare(h.cpu().numpy(), p.cpu().numpy(), ho, po, ao, 0.0, "arm only")
