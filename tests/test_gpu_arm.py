"""The articulated arm on the GPU (arm 2: one articulated body in reduced
coordinates driven by PD joint motors, Sec. 1 and Sec. 5) against the
oracle: one step from the same float32 state, joint rates and motor state.

Pairs, contacts, colours, impulses and body states as in every parity test
(`compare`, the arm's links as one body for the tie islands); the arm's
joint angles, joint rates, motor targets and motor impulses besides.  The
persistent launch and the global-memory working set give the same bits as
one workgroup per scene; modes the arm does not support are refused."""
import numpy as np
import pytest

from gpu_util import arm_snapshot32, compare, gpu_results, gpu_sim, oracle_warmup, report, snapshot32
from helpers import DT, S, custom_batch
from oracle import oracle as O

pytestmark = pytest.mark.gpu

HORIZONTAL = np.array([0.0, np.pi / 2, 0.0, 0.0, 0.0, 0.0, 0.0])
TH_BAR = 1e-5       # rad: one step's angle change is dt * rate
QD_BAR = 1e-4       # rad/s, relative to the rate with a 1 rad/s floor (the state bar of the bodies)
LAM_M_BAR = 1e-3    # motor impulses, relative to the largest (N m s)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def sweep_actions(n, t):
    """Motor-target rates that swing the arm out and round through the
    clutter: shoulder and elbow pitch down for 110 steps while the base yaws
    at 0.8 to 1 rad/s (one rate per scene)."""
    a = np.zeros((n, 7))
    a[:, 0] = 0.8 * (1 + 0.25 * np.arange(n) / max(n - 1, 1))
    a[:, 1] = 1.0 if t < 110 else 0.0
    a[:, 3] = 0.4 if t < 110 else 0.0
    return a.astype(np.float32)


def sweep_warmup(b, steps):
    ora = O.OracleSim(b)
    for t in range(steps):
        ora.step(actions=sweep_actions(b.n_scenes, t), iters=20, warm=O.PREV, outputs=False)
    return ora


def step_both(torch, b, ora, warm, iters, tol=0.0, act_seed=7, step_index=0, threads=64, sweep=False, **kw):
    pose, vel, theta, cache = snapshot32(ora)
    ast = arm_snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=warm, tol=tol, threads=threads, **kw)
    sim.arm_state.copy_(torch.as_tensor(ast))
    act = sweep_actions(b.n_scenes, step_index) if sweep else S.arm_actions(act_seed, b.n_scenes, step_index)
    sim.step(torch.as_tensor(act, device=sim.device), DT, iters)
    r = ora.step(actions=act, iters=iters, tol=tol, warm=warm, max_pairs=sim.max_pairs,
                 max_contacts=sim.max_contacts)
    return sim, gpu_results(sim), r


def check_arm(b, g, r, ora, tol_mode=False):
    """Joint angles, rates, targets and motor impulses of every scene whose
    arm no tie touched and whose sweep counts agree."""
    ast_g = g["arm_state"]
    ast_o = ora.arm_state.reshape(-1, 3, 7)
    th_g, th_o = g["theta"], ora.theta.reshape(-1, 7)
    np.testing.assert_allclose(ast_g[:, 1], ast_o[:, 1], rtol=0, atol=1e-6)   # targets
    worst = dict(th=0.0, qd=0.0, lam=0.0)
    for s in range(b.n_scenes):
        b1 = int(b.body_offset[s + 1])
        if r["tied"][b1 - 7:b1].any() or int(g["stats"]["sweeps"][s]) != int(r["sweeps"][s]):
            continue
        eth = np.abs(th_g[s] - th_o[s]).max()
        eqd = (np.abs(ast_g[s, 0] - ast_o[s, 0]) / np.maximum(np.abs(ast_o[s, 0]), 1.0)).max()
        scale = max(np.abs(ast_o[s, 2]).max(), 1e-12)
        elam = np.abs(ast_g[s, 2] - ast_o[s, 2]).max() / scale
        worst["th"], worst["qd"], worst["lam"] = max(worst["th"], eth), max(worst["qd"], eqd), max(worst["lam"], elam)
        assert eth <= TH_BAR, f"scene {s}: joint angle error {eth:.3e}"
        assert eqd <= QD_BAR, f"scene {s}: joint rate error {eqd:.3e}"
        assert elam <= (3e-2 if tol_mode else LAM_M_BAR), f"scene {s}: motor impulse error {elam:.3e}"
    print(f"[arm] max err theta {worst['th']:.1e} rate {worst['qd']:.1e} motor impulse/scale {worst['lam']:.1e}",
          flush=True)


def test_arm_alone_parity(torch_cuda):
    """Arm-only scenes at four postures: no contact rows, the motors alone."""
    bodies = [[] for _ in range(4)]
    b = custom_batch(bodies, arm=2)
    b.arm_theta = np.random.default_rng(5).uniform(-0.8, 0.8, (4, 7)).astype(np.float32)
    ora = oracle_warmup(b, 30, iters=20, warm=O.PREV)
    sim, g, r = step_both(torch_cuda, b, ora, O.PREV, 20, step_index=30)
    rep = compare(b, g, r, ora, contact_values=True)
    report("arm alone", rep)
    check_arm(b, g, r, ora)


def test_balls_on_arm_parity(torch_cuda):
    """Two balls resting on the held, horizontal arm: contacts on the arm."""
    from test_oracle_arm_dynamic import chain
    o, a, c = chain(HORIZONTAL)
    balls = [dict(shape=S.SPHERE, param=[0.05, 0.0, 0.0], mass=0.5, mu=0.8,
                  pos=c[1] + np.array([d, 0.0, S.ARM_RADIUS + 0.05 - 0.001])) for d in (-0.08, 0.08)]
    b = custom_batch([balls, balls], arm=2, theta=HORIZONTAL)
    ora = oracle_warmup(b, 60, iters=40, warm=O.PREV)
    sim, g, r = step_both(torch_cuda, b, ora, O.PREV, 40, step_index=60)
    rep = compare(b, g, r, ora, contact_values=True)
    report("balls on the arm", rep)
    assert rep["contacts_solved"] >= 4
    check_arm(b, g, r, ora)
    np.testing.assert_allclose(g["stats"]["arm_force"], r["arm_force"], rtol=1e-3)


@pytest.mark.parametrize("warm,tol,iters", [(O.PREV, 0.0, 20), (O.COLD, 0.0, 20), (O.PREV, 1e-4, 1000)])
def test_clutter_arm_parity(torch_cuda, warm, tol, iters):
    """Clutter with the articulated arm swung through it (90 oracle steps of
    sweep_actions: the arm meets piles, shelves and static boxes, some
    motors at their bound), one step."""
    b = S.batch_clutter(8, seed0=10000, arm=2)
    ora = sweep_warmup(b, 90)
    sim, g, r = step_both(torch_cuda, b, ora, warm, iters, tol=tol, step_index=90, sweep=True)
    rep = compare(b, g, r, ora, contact_values=True, tol_band=0.02 if tol > 0 else None)
    report(f"clutter, articulated arm, warm={warm} tol={tol:g}", rep)
    n_arm = 0
    for s in range(b.n_scenes):
        n = int(r["n_contacts"][s])
        keys = r["c_key"][s, :n]
        nb = int(b.body_offset[s + 1] - b.body_offset[s])
        a, bb = keys >> 20, (keys >> 8) & 0xFFF
        n_arm += int(np.sum((a >= nb - 7) | ((bb >= nb - 7) & (bb != 0xFFF))))
    print(f"contacts on the arm: {n_arm}", flush=True)
    assert n_arm >= 4 and rep["contacts_solved"] >= 500
    check_arm(b, g, r, ora, tol_mode=tol > 0)
    np.testing.assert_allclose(g["stats"]["arm_force"], r["arm_force"], rtol=2e-2, atol=1e-3)


def state(sim):
    import torch
    torch.cuda.synchronize()
    cnt, key, lam = sim.cache()
    return dict(pose=sim.pose.cpu().numpy().copy(), vel=sim.vel.cpu().numpy().copy(),
                theta=sim.theta.cpu().numpy().copy(), arm=sim.arm_state.cpu().numpy().copy(),
                count=cnt.cpu().numpy().copy(), key=key.cpu().numpy().copy(), lam=lam.cpu().numpy().copy(),
                **{k: v.cpu().numpy().copy() for k, v in sim.stats.items()})


@pytest.mark.parametrize("variant", ["persistent", "hbm", "threads"])
def test_arm_launches_bit_identical(torch_cuda, variant):
    """60 steps of clutter with the articulated arm under actions: the
    persistent launch, every working set in global memory, or 256 threads a
    scene give the same bits as one 64-thread workgroup per scene in LDS."""
    torch = torch_cuda
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_clutter(12, seed0=10300, arm=2)
    sims = []
    for alt in (False, True):
        kw = dict(max_pairs=2048, max_contacts=2048, warm=O.PREV, tol=1e-4, threads=64)
        if alt and variant == "hbm":
            kw["hbm_min_bodies"] = 1
        if alt and variant == "threads":
            kw["threads"] = 256
        sm = Sim(b, **kw)
        if alt and variant == "persistent":
            sm.set_persistent(True, 64)
        sims.append(sm)
    for t in range(60):
        act = torch.as_tensor(sweep_actions(b.n_scenes, t + 40), device="cuda:0", dtype=torch.float32)
        for sm in sims:
            sm.step(act, DT, 200)
        if t % 20 == 19:
            x, y = state(sims[0]), state(sims[1])
            for k in x:
                assert np.array_equal(x[k], y[k]), f"step {t}: {k} differs"
    assert np.abs(state(sims[0])["arm"][:, 0]).max() > 0.05   # the arm did move


def test_arm_refusals(torch_cuda):
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    b = S.batch_clutter(2, seed0=10000, arm=2)
    with pytest.raises(L.SimError):
        Sim(b, solver=L.JACOBI)
    with pytest.raises(L.SimError):
        Sim(b, warm=O.LEARNED)
    sim = Sim(b, warm=O.PREV)
    with pytest.raises(L.SimError, match="articulated"):
        sim.set_solver(L.JACOBI, L.PREV, 0.0)
    with pytest.raises(L.SimError):
        sim.set_motors(1.5, 10.0)
    with pytest.raises(L.SimError):
        sim.set_motors(0.3, -1.0)
    sim.set_motors(0.3, 10.0)
    k = S.batch_clutter(2, seed0=10000, arm=True)
    sk = Sim(k, warm=O.PREV)
    with pytest.raises(L.SimError, match="articulated"):
        sk.set_motors(0.3, 10.0)
