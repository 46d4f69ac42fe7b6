"""Training and evaluation of the learned warm start.

Logging: plain runs with the classic warm start, solved tight (tolerance
1e-6 m/s, cap 1000 sweeps), export on; after every step the library gathers
each new contact's 16 features and the network's target, its converged
impulse in units of |g| dt / k_n (saturated at +-32).  Training: minibatch
Adam with global gradient-norm clipping and a linearly decaying learning
rate (the optimizer setup of the paper's monolithic policy, appendix B.2:
clip 0.5; the learning rate is raised from its 1e-4 to 1e-3, which fits
the small new-contact set in fewer epochs).  Evaluation: held-out scenes
stepped at a working tolerance in COLD, PREV and LEARNED modes, recording
sweeps, flags and residual per scene-step and wall time per step.

    python -m paper_2106_14405_amd.train --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import _lib as L
from . import scenes
from .mlp import NP, Net, gather, train
from .sim import Sim

DT = 1.0 / 120.0


def log_dataset(n_scenes: int = 512, seed0: int = 1000, steps: int = 120, tol: float = 1e-6, cap: int = 1000,
                device: str = "cuda:0", max_contacts: int = 512, target_clip: float = 32.0, warm: int = L.PREV,
                verbose: bool = False):
    """Features [n, 16] and targets [n, 3] of tight plain runs on drop scenes (classic warm start by default)."""
    b = scenes.batch_drop(n_scenes, seed0=seed0)
    sim = Sim(b, warm=warm, tol=tol, threads=64, max_contacts=max_contacts, max_pairs=max_contacts,
              device=device)
    sim.set_export(True)
    xs, ts = [], []
    for k in range(steps):
        sim.step(None, DT, cap)
        x, t = gather(sim, target_clip=target_clip)
        xs.append(x.clone())
        ts.append(t.clone())
        if verbose and (k + 1) % 20 == 0:
            print(f"  logged step {k + 1}/{steps}: {sum(int(a.shape[0]) for a in xs)} rows", flush=True)
    sim.close()
    return torch.cat(xs), torch.cat(ts)


def fit(x: torch.Tensor, t: torch.Tensor, epochs: int = 100, batch: int = 4096, lr: float = 1e-3,
        clip: float = 0.5, seed: int = 0, device: str = "cuda:0", log=None) -> Net:
    net = Net(device=device, seed=seed)
    net.fit_stats(x)
    return train(net, x, t, epochs=epochs, batch=batch, lr=lr, clip=clip, seed=seed, log=log)


def save(net: Net, path: str, meta: dict | None = None):
    np.savez(path, params=net.params.cpu().numpy(), mean=net.mean.cpu().numpy(), std=net.std.cpu().numpy(),
             meta=np.array(json.dumps(meta or {})))


def load(path: str, device: str = "cuda:0") -> Net:
    z = np.load(path, allow_pickle=False)
    p = z["params"].astype(np.float32)
    if p.shape != (NP,):
        raise ValueError(f"{path}: expected {NP} parameters")
    net = Net(device=device, params=p)
    net.mean.copy_(torch.as_tensor(z["mean"].astype(np.float32)))
    net.std.copy_(torch.as_tensor(z["std"].astype(np.float32)))
    net.export()
    return net


def evaluate(mode: int, net: Net | None = None, n_scenes: int = 100, seed0: int = 2000, steps: int = 120,
             tol: float = 1e-4, cap: int = 200, device: str = "cuda:0", max_contacts: int = 512):
    """Sweeps, flags, contacts and residuals [steps, S] and per-step wall milliseconds of one mode."""
    b = scenes.batch_drop(n_scenes, seed0=seed0)
    sim = Sim(b, warm=mode, tol=tol, threads=64, max_contacts=max_contacts, max_pairs=max_contacts,
              device=device)
    if mode == L.LEARNED:
        if net is None:
            raise ValueError("LEARNED mode needs a network")
        net.attach(sim)
    sweeps = torch.zeros((steps, n_scenes), dtype=torch.int32, device=sim.device)
    flags = torch.zeros((steps, n_scenes), dtype=torch.int32, device=sim.device)
    contacts = torch.zeros((steps, n_scenes), dtype=torch.int32, device=sim.device)
    resid = torch.zeros((steps, n_scenes), dtype=torch.float32, device=sim.device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    stream = sim.stream
    ev[0].record(stream)
    for k in range(steps):
        sim.step(None, DT, cap)
        ev[k + 1].record(stream)
        sweeps[k].copy_(sim.stats["sweeps"])
        flags[k].copy_(sim.stats["flags"])
        contacts[k].copy_(sim.stats["contacts"])
        resid[k].copy_(sim.stats["residual"])
    torch.cuda.synchronize()
    ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    sim.close()
    return dict(sweeps=sweeps.cpu().numpy(), flags=flags.cpu().numpy(), contacts=contacts.cpu().numpy(),
                residual=resid.cpu().numpy(), ms=ms)


def summary(r: dict, skip: int = 0) -> dict:
    """Mean / p50 / p95 sweeps over scene-steps with contacts, % capped, % fell back, ms per step."""
    sw, fl, nc = r["sweeps"][skip:], r["flags"][skip:], r["contacts"][skip:]
    m = nc > 0
    s = sw[m].astype(np.float64)
    return dict(mean=float(s.mean()) if s.size else 0.0, p50=float(np.percentile(s, 50)) if s.size else 0.0,
                p95=float(np.percentile(s, 95)) if s.size else 0.0,
                capped=float(np.mean(fl[m] & L.FLAG_NOT_CONVERGED > 0)) if s.size else 0.0,
                fellback=float(np.mean(fl[m] & L.FLAG_FELLBACK > 0)) if s.size else 0.0,
                ms=float(np.mean(r["ms"][skip:])), scene_steps=int(m.sum()))


def paired(ra: dict, rb: dict, skip: int = 0) -> dict:
    """Paired comparison of two modes run on the same scenes: per scene, the
    mean sweeps over the scene-steps with contacts in both runs, and per step
    the batch's wall milliseconds; mean difference (a - b) and its 95%
    interval (1.96 standard errors)."""
    sa, sb = ra["sweeps"][skip:].astype(np.float64), rb["sweeps"][skip:].astype(np.float64)
    m = (ra["contacts"][skip:] > 0) & (rb["contacts"][skip:] > 0)
    cnt = m.sum(axis=0)
    ok = cnt > 0
    d = ((sa * m).sum(axis=0)[ok] - (sb * m).sum(axis=0)[ok]) / cnt[ok]
    dm = np.asarray(ra["ms"][skip:], np.float64) - np.asarray(rb["ms"][skip:], np.float64)
    ci = lambda x: float(1.96 * x.std(ddof=1) / np.sqrt(x.size)) if x.size > 1 else float("nan")
    return dict(sweeps=float(d.mean()) if d.size else 0.0, sweeps_ci95=ci(d), ms=float(dm.mean()),
                ms_ci95=ci(dm), scenes=int(d.size), steps=int(dm.size))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--scenes", type=int, default=512)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=240)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--clip", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-scenes", type=int, default=4096)
    ap.add_argument("--eval-seed0", type=int, default=2000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    t0 = time.time()
    x, t = log_dataset(a.scenes, a.seed0, a.steps, verbose=True)
    print(f"dataset: {x.shape[0]} rows in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    net = fit(x, t, a.epochs, a.batch, a.lr, a.clip, a.seed,
              log=lambda ep, loss: print(f"  epoch {ep + 1}: batch loss {loss:.4f}", flush=True))
    torch.cuda.synchronize()
    print(f"trained in {time.time() - t0:.1f} s", flush=True)
    res = {}
    for name, mode in (("cold", L.COLD), ("prev", L.PREV), ("learned", L.LEARNED)):
        res[name] = summary(evaluate(mode, net if mode == L.LEARNED else None, a.eval_scenes, a.eval_seed0,
                                     a.steps))
        print(name, json.dumps(res[name]), flush=True)
    if a.out:
        save(net, a.out, dict(vars(a), rows=int(x.shape[0]), eval=res))


if __name__ == "__main__":
    main()
