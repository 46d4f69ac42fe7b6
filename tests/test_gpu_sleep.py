"""Sleeping islands on the GPU (localized physics): one step of clutter
scenes whose piles the oracle has settled with sleeping on, against the
oracle's step from the same float32 state and rest counters.  Pairs,
contact keys and geometry bit-exact outside the tied pairs; colours
(including -1 for the contacts of sleeping bodies), impulses, states and the
rest counters outside the tied islands; the persistent launch and the
global-memory working set give the same bits as the plain launch; the
learned warm start is refused together with sleeping."""
import numpy as np
import pytest

from gpu_util import compare, gpu_results, gpu_set_rest, gpu_sim, report, snapshot32
from helpers import DT, S
from oracle import oracle as O

pytestmark = pytest.mark.gpu

V_S, T_S = 0.02, 30


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def settled_sleeping(batch, steps, iters=20):
    ora = O.OracleSim(batch)
    ora.set_sleep(V_S, T_S)
    for t in range(steps):
        act = S.arm_actions(1, batch.n_scenes, t) if batch.arm else None
        ora.step(actions=act, iters=iters, warm=O.PREV, outputs=False)
    return ora


def step_both(torch, b, ora, warm, iters, tol=0.0, threads=64, step_index=0):
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=warm, tol=tol, threads=threads)
    sim.set_sleep(V_S, T_S)
    gpu_set_rest(sim, ora.rest)
    act = S.arm_actions(7, b.n_scenes, step_index) if b.arm else None
    sim.step(torch.as_tensor(act, device=sim.device) if act is not None else None, DT, iters)
    r = ora.step(actions=act, iters=iters, tol=tol, warm=warm, max_pairs=sim.max_pairs,
                 max_contacts=sim.max_contacts)
    return sim, gpu_results(sim), r


@pytest.mark.parametrize("warm,tol,iters", [(O.PREV, 0.0, 20), (O.COLD, 1e-4, 1000), (O.PREV, 1e-4, 1000)])
def test_sleeping_step_parity(torch_cuda, warm, tol, iters):
    b = S.batch_clutter(8, seed0=10000)
    ora = settled_sleeping(b, 300)
    asleep_before = int((ora.rest >= T_S).sum())
    sim, g, r = step_both(torch_cuda, b, ora, warm, iters, tol=tol, step_index=300)
    rep = compare(b, g, r, ora, contact_values=True, tol_band=0.02 if tol > 0 else None, check_rest=True)
    report(f"sleeping clutter warm={warm} tol={tol:g}", rep)
    n_sleep_o = sum(int((r["c_colour"][s, :int(r["n_contacts"][s])] == -1).sum()) for s in range(b.n_scenes))
    n_sleep_g = sum(int((g["colour"][s, :int(g["count"][s])] == -1).sum()) for s in range(b.n_scenes))
    print(f"bodies at rest for {T_S}+ steps: {asleep_before}; sleeping contacts oracle {n_sleep_o}, GPU {n_sleep_g}")
    assert n_sleep_o > 200 and n_sleep_g > 200
    assert rep["contacts_solved"] >= 500
    assert rep["excluded_frac"] <= 0.5


def state(sim):
    import torch
    torch.cuda.synchronize()
    cnt, key, lam = sim.cache()
    return dict(pose=sim.pose.cpu().numpy().copy(), vel=sim.vel.cpu().numpy().copy(),
                rest=sim.rest.cpu().numpy().copy(), count=cnt.cpu().numpy().copy(),
                key=key.cpu().numpy().copy(), lam=lam.cpu().numpy().copy(),
                **{k: v.cpu().numpy().copy() for k, v in sim.stats.items()})


@pytest.mark.parametrize("variant", ["persistent", "hbm"])
def test_sleeping_launches_bit_identical(torch_cuda, variant):
    """Uneven drop scenes stepped 240 steps with sleeping on: the persistent
    launch, and every scene's working set in global memory, give the same
    bits as one workgroup per scene in LDS (rest counters included), and
    bodies do fall asleep."""
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_uneven(24, seed0=20400, lo=16, hi=400)
    sims = []
    for alt in (False, True):
        kw = dict(max_pairs=2048, max_contacts=2048, warm=O.PREV, tol=1e-4, threads=64)
        if alt and variant == "hbm":
            kw["hbm_min_bodies"] = 1
        sm = Sim(b, **kw)
        if alt and variant == "persistent":
            sm.set_persistent(True, 64)
        sm.set_sleep(V_S, T_S)
        sims.append(sm)
    for t in range(240):
        for sm in sims:
            sm.step(None, DT, 200)
        if t % 60 == 59:
            a, c = state(sims[0]), state(sims[1])
            for k in a:
                assert np.array_equal(a[k], c[k]), f"step {t}: {k} differs"
    assert (state(sims[0])["rest"] >= T_S).sum() > 500


def test_learned_start_refused_with_sleeping(torch_cuda):
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_drop(2, seed0=3)
    sim = Sim(b, warm=O.PREV)
    sim.set_sleep(V_S, T_S)
    with pytest.raises(L.SimError, match="sleeping"):
        sim.set_solver(L.PGS, L.LEARNED, 1e-4)
    sim2 = Sim(b, warm=O.LEARNED)
    with pytest.raises(L.SimError, match="learned"):
        sim2.set_sleep(V_S, T_S)
    with pytest.raises(L.SimError):
        sim.set_sleep(-1.0, T_S)
    sim.set_sleep(0.0, 0)      # off again
