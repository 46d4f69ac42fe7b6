"""Benchmark: env-steps/s of the batched rigid-body step on one MI355X.

One env-step = one scene advanced by one call of the step at dt = 1/120 s.
Workload (default): 1,024 clutter scenes x (20 static boxes + 108 dynamic
spheres/boxes/capsules + a kinematic 7-link capsule arm driven by seeded
joint velocities in [-1, 1] rad/s), plain projected Gauss-Seidel (no learned
warm start), residual tolerance 1e-4 m/s with a cap of 20 sweeps, float32.
Synthetic, seeded inputs stand in for the paper's rearrangement scenes.
--workload uneven: 4,096 drop scenes with 16-512 dynamic bodies
(log-uniform) through the persistent launch (autotuned queue split, HIP
graph replay), every scene reset to its initial state after an episode of
U[100, 300] steps.  --workload drop: 1,024 drop scenes of 64 bodies.

After the timed run (untimed), learned vs plain: the committed warm-start
network against plain PGS (cold start) and the classic warm start on
held-out drop scenes at residual 1e-4 with a cap of 200 sweeps.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload clutter|uneven|drop]

Prints one JSON line.  W untimed steps let the dropped objects land; the K
timed steps run back to back on the simulation's stream between HIP events.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/sec at contact residual 1e-4; PGS iterations, learned vs plain"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per unit of work (float32 structure of arrays):
B_DYN = 144.0      # per dynamic body per step: state read+write 104 B + constants 40 B
B_STATIC = 52.0    # per static or kinematic body per step: pose + shape + material
B_CONTACT = 40.0   # per contact per step: cache read 20 B + write 20 B
B_SWEEP = 240.0    # per contact per sweep if the solver state were streamed from memory


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=150)
    ap.add_argument("--workload", default="clutter", choices=["clutter", "drop", "uneven"])
    ap.add_argument("--scenes", type=int, default=None)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--warm", default="cold", choices=["cold", "prev"])
    ap.add_argument("--threads", type=int, default=64)
    ap.add_argument("--max-contacts", type=int, default=None)
    ap.add_argument("--max-pairs", type=int, default=None)
    ap.add_argument("--launch", default=None, choices=["plain", "persistent"],
                    help="uneven workload: persistent (default) or one workgroup per scene")
    ap.add_argument("--learned-eval", type=int, default=1)
    ap.add_argument("--learned-scenes", type=int, default=2048)
    ap.add_argument("--learned-steps", type=int, default=240)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-scenes", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="only run an elementwise copy of this many MiB (counter calibration)")
    return ap.parse_args()


def probe_copy(mib):
    """Elementwise copy b = a + 0 of `mib` MiB, 5 launches: reads and writes
    exactly mib MiB each; used to scale the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.add(a, 0.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"probe_copy_mib": mib, "launches": 5}))


def kernel_hash():
    h = hashlib.sha256()
    for f in ("step.hip", "geom.h", "sim_internal.h", "mlp_mfma.h", "mlp.hip"):
        p = os.path.join(ROOT, "paper_2106_14405_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"step_kernel_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(batch_fn, n_scenes, warm_steps, timed_steps, iters, tol, warm, arm):
    """The FP64 oracle, single thread, on a sample of the same workload."""
    from oracle import oracle as O
    from paper_2106_14405_amd import scenes as S
    b = batch_fn(n_scenes)
    o = O.OracleSim(b)
    w = O.PREV if warm == "prev" else O.COLD
    for t in range(warm_steps):
        o.step(actions=S.arm_actions(1, n_scenes, t) if arm else None, iters=iters, tol=tol, warm=w,
               outputs=False)
    acts = [S.arm_actions(1, n_scenes, warm_steps + t) if arm else None for t in range(timed_steps)]
    t0 = time.perf_counter()
    for t in range(timed_steps):
        o.step(actions=acts[t], iters=iters, tol=tol, warm=w, outputs=False)
    dt = time.perf_counter() - t0
    return dict(value=n_scenes * timed_steps / dt, unit="env-steps/s", cores=1, kind="oracle",
                sample=f"{n_scenes} scenes x {timed_steps} steps after {warm_steps} untimed steps, "
                       f"same workload, same sweep cap and tolerance, one host thread")


def reset_schedule(n_scenes, n_steps, seed=7):
    """[n_steps, S] uint8 masks: each scene restarts after U[100, 300] steps."""
    rng = np.random.default_rng(seed)
    m = np.zeros((n_steps, n_scenes), np.uint8)
    nxt = rng.integers(100, 301, size=n_scenes)
    for t in range(n_steps):
        hit = nxt == t
        m[t, hit] = 1
        nxt[hit] += rng.integers(100, 301, size=int(hit.sum()))
    return m


def workload_name(w, n_scenes, batch):
    if w == "clutter":
        return (f"clutter: {n_scenes} scenes x {batch.n_bodies // n_scenes} bodies (20 static boxes, "
                "108 dynamic spheres/boxes/capsules, 7-link kinematic arm)")
    if w == "uneven":
        c = batch.counts()
        return (f"uneven: {n_scenes} drop scenes, {int(c.min())}-{int(c.max())} dynamic spheres/boxes "
                f"(log-uniform), {batch.n_bodies} bodies")
    return f"drop: {n_scenes} scenes x 64 dynamic bodies (32 spheres + 32 boxes)"


def learned_vs_plain(n_scenes, steps):
    """Held-out drop scenes (seeds 2000+) at residual 1e-4, cap 200 sweeps:
    plain PGS (cold), classic warm start, the committed learned warm start."""
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd import train as T
    path = os.path.join(ROOT, "paper_2106_14405_amd", "weights", "warmstart_drop.npz")
    if not os.path.exists(path):
        return None
    net = T.load(path)
    res = {}
    for name, mode in (("cold", L.COLD), ("prev", L.PREV), ("learned", L.LEARNED)):
        r = T.evaluate(mode, net if mode == L.LEARNED else None, n_scenes=n_scenes, seed0=2000, steps=steps,
                       tol=1e-4, cap=200)
        res[name] = T.summary(r)
    res["workload"] = (f"{n_scenes} held-out drop scenes x {steps} steps, tolerance 1e-4 m/s, cap 200 sweeps; "
                       "mean/p50/p95 sweeps per scene-step with contacts, ms per step of the whole batch")
    return res


def main():
    a = parse()
    if a.probe_copy_mib:
        probe_copy(a.probe_copy_mib)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    from paper_2106_14405_amd import scenes as S
    if a.workload == "clutter":
        n_scenes = a.scenes or 1024
        batch_fn = lambda n: S.batch_clutter(n, seed0=10000)
        arm = True
        max_contacts = a.max_contacts or 512
        max_pairs = a.max_pairs or max_contacts
    elif a.workload == "uneven":
        n_scenes = a.scenes or 4096
        batch_fn = lambda n: S.batch_uneven(n, seed0=20000, lo=16, hi=512)
        arm = False
        max_contacts = a.max_contacts or 2048
        max_pairs = a.max_pairs or 2560   # 512-body piles reach 4.2 pairs per body
    else:
        n_scenes = a.scenes or 1024
        batch_fn = lambda n: S.batch_drop(n, seed0=0)
        arm = False
        max_contacts = a.max_contacts or 384
        max_pairs = a.max_pairs or max_contacts
    batch = batch_fn(n_scenes)              # generated before the GPU is touched
    K, W = a.steps, a.warmup
    acts_np = (np.stack([S.arm_actions(1, n_scenes, t) for t in range(W + K)]) if arm else None)

    import torch

    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    warm = L.PREV if a.warm == "prev" else L.COLD
    sim = Sim(batch, max_contacts=max_contacts, max_pairs=max_pairs, warm=warm, tol=a.tol,
              threads=a.threads, device=dev)
    acts = torch.as_tensor(acts_np, device=dev) if arm else None
    resets = None
    tuned = None
    persistent = a.workload == "uneven" and a.launch != "plain"
    if a.workload == "uneven":
        if persistent:
            sim.set_persistent(True)
            tuned = sim.autotune(steps=3, dt=1.0 / 120.0, iters=a.iters)
        resets = torch.as_tensor(reset_schedule(n_scenes, W + K), device=dev)
        pose0 = sim.pose.clone()
        vel0 = sim.vel.clone()

    def one(t):
        if resets is not None:
            sim.reset(resets[t], pose0, vel0)
        sim.step(acts[t] if arm else None, 1.0 / 120.0, a.iters)

    for t in range(W):
        one(t)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(sim.stream)
    for t in range(K):
        one(W + t)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / K
    value = n_scenes * K / (ms / 1e3)
    # statistics pass (untimed): the same trajectory continued for 10 steps
    st = dict(contacts=[], sweeps=[], conv=[], flags=[], pairs=[], colours=[], resid=[])
    for t in range(10):
        if resets is not None:
            sim.reset(torch.zeros_like(resets[0]), pose0, vel0)
        sim.step(acts[(W + K + t) % (W + K)] if arm else None, 1.0 / 120.0, a.iters)
        s = {k: v.cpu().numpy() for k, v in sim.stats.items()}
        st["contacts"].append(s["contacts"].mean())
        st["pairs"].append(s["pairs"].mean())
        st["colours"].append(s["colours"].mean())
        st["sweeps"].append(s["sweeps"].mean())
        st["conv"].append(np.mean(s["residual"] <= a.tol) if a.tol > 0 else float("nan"))
        st["flags"].append(np.mean((s["flags"] & (L.FLAG_NONFINITE | L.FLAG_CAPACITY)) != 0))
        st["resid"].append(np.median(s["residual"]))
    contacts = float(np.mean(st["contacts"]))
    motion = batch.motion
    n_dyn = int(np.sum(motion == S.DYNAMIC))
    n_other = int(batch.n_bodies - n_dyn)
    bytes_launch = B_DYN * n_dyn + B_STATIC * n_other + B_CONTACT * contacts * n_scenes
    achieved = bytes_launch / (ms_step / 1e3) / 1e9
    traffic = measured_traffic(a.workload)
    kname = "step_persistent" if persistent else "step_kernel"
    sweep_bytes = B_SWEEP * contacts * n_scenes * float(np.mean(st["sweeps"]))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload_name(a.workload, n_scenes, batch),
            "scenes": n_scenes, "bodies": int(batch.n_bodies), "dynamic_bodies": n_dyn,
            "dt": 1.0 / 120.0, "sweep_cap": a.iters, "tolerance_m_per_s": a.tol,
            "warm_start": a.warm, "solver": "pgs",
            "threads_per_scene": a.threads if not persistent else "autotuned: 64 (one wave) or 256",
            "max_contacts_per_scene": max_contacts, "max_pairs_per_scene": max_pairs,
            **({"launch": "persistent, HIP graph" if persistent else "one workgroup per scene",
                "wave_max_bodies": tuned, "resets": "each scene after U[100, 300] steps"}
               if a.workload == "uneven" else {}),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kname, "bytes_per_launch": bytes_launch,
            "sweep_equivalent_GBs": sweep_bytes / (ms_step / 1e3) / 1e9,
        },
        "solver_stats": {
            "contacts_per_scene": contacts, "pairs_per_scene": float(np.mean(st["pairs"])),
            "colours_per_scene": float(np.mean(st["colours"])), "sweeps_mean": float(np.mean(st["sweeps"])),
            "frac_scene_steps_at_tol": float(np.mean(st["conv"])), "median_residual": float(np.mean(st["resid"])),
            "frac_capacity_or_nonfinite": float(np.mean(st["flags"])),
            "sweeps_learned": None, "sweeps_plain": float(np.mean(st["sweeps"])),
        },
        "cpu_baseline": None,
    }
    sim.close()
    del sim
    torch.cuda.synchronize()
    if a.learned_eval:
        lv = learned_vs_plain(a.learned_scenes, a.learned_steps)
        if lv is not None:
            out["solver_stats"]["sweeps_learned"] = lv["learned"]["mean"]
            out["solver_stats"]["sweeps_plain"] = lv["cold"]["mean"]
            out["learned_vs_plain"] = lv
    if a.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(batch_fn, a.cpu_scenes, W, a.cpu_steps, a.iters, a.tol, a.warm, arm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
