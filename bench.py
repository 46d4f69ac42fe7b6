"""Benchmark: env-steps/s of the batched rigid-body step on one MI355X at
contact residual 1e-4, and PGS sweeps with the learned warm start against
plain PGS.

One env-step = one scene advanced by one call of the step at dt = 1/120 s.
Default workload (clutter): 1,024 scenes x (20 static boxes + 108 dynamic
spheres/boxes/capsules + a kinematic 7-link capsule arm driven by seeded
joint velocities in [-1, 1] rad/s), float32.  Synthetic, seeded inputs stand
in for the paper's rearrangement scenes (ReplicaCAD furniture, YCB objects,
the Fetch arm).

Protocol.  The dropped objects are first settled, untimed, for --settle
steps (the scenes start from a settled pile whatever --warmup says, as the
paper's clutter is settled offline before episodes start).  The settled
state is saved; then for each warm-start mode (cold: plain PGS from zero
impulses; prev: the classic warm start from the previous step's impulses;
learned: the committed network) the state is restored, W untimed and K
timed steps run at residual tolerance --tol (m/s) with a sweep cap --cap,
timed with HIP events on the simulation's stream.  The same W + K steps are
then replayed from the restored state (the step is deterministic, so the
replay reproduces the timed steps bit for bit) to collect per scene-step
sweeps, residuals and flags.  `value` is the headline mode's env-steps/s;
`frac_at_tol` says how many scene-steps reached the tolerance.

Also reported: the roofline of the step kernel (algorithmic HBM bytes per
launch over its measured duration, against the 8 TB/s peak; measured
traffic from committed rocprofv3 counters of the same window), learned vs
plain on held-out small drop scenes (64 bodies, seeds 2000+, tolerance 1e-4,
cap 200), and the FP64 oracle on the host cores as a CPU baseline.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload clutter|uneven|drop]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/sec at contact residual 1e-4; PGS iterations, learned vs plain"
HBM_PEAK_GBS = 8000.0
DT = 1.0 / 120.0
# algorithmic bytes per unit of work (float32 structure of arrays):
B_DYN = 144.0      # per dynamic body per step: state read+write 104 B + constants 40 B
B_STATIC = 52.0    # per static or kinematic body per step: pose + shape + material
B_CONTACT = 40.0   # per contact per step: cache read 20 B + write 20 B
B_SWEEP = 240.0    # per contact per sweep if the solver state were streamed from memory
MODES = ("cold", "prev", "learned", "prev_sleep")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle", type=int, default=300, help="untimed settling steps before any mode runs")
    ap.add_argument("--workload", default="clutter", choices=["clutter", "drop", "uneven", "scale"])
    ap.add_argument("--scenes", type=int, default=None)
    ap.add_argument("--tol", type=float, default=None, help="residual tolerance (m/s); 1e-4, scale 1e-5")
    ap.add_argument("--cap", type=int, default=None, help="sweep cap at the tolerance")
    ap.add_argument("--headline", default=None, help="prev; scale: learned")
    ap.add_argument("--modes", default=",".join(MODES),
                    help="warm starts to time; a _sleep suffix turns sleeping islands on for that mode")
    ap.add_argument("--sleep-speed", type=float, default=0.02, help="sleeping islands: at-rest speed (m/s)")
    ap.add_argument("--sleep-steps", type=int, default=30, help="sleeping islands: steps at rest before sleep")
    ap.add_argument("--no-replay", action="store_true", help="skip the statistics replay (profiling runs)")
    ap.add_argument("--threads", type=int, default=64)
    ap.add_argument("--max-contacts", type=int, default=None)
    ap.add_argument("--max-pairs", type=int, default=None)
    ap.add_argument("--launch", default=None, choices=["plain", "persistent"],
                    help="uneven workload: persistent (default) or one workgroup per scene")
    ap.add_argument("--pool", type=int, default=4, help="uneven workload: fresh states per scene in the reset pool")
    ap.add_argument("--arm-eval", type=int, default=1,
                    help="clutter: also time variants of the workload: the articulated arm (PD joint "
                         "motors), cabinets with doors and drawers, convex hulls")
    ap.add_argument("--learned-eval", type=int, default=1)
    ap.add_argument("--learned-scenes", type=int, default=2048)
    ap.add_argument("--learned-steps", type=int, default=240)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-scenes-per-thread", type=int, default=8)
    ap.add_argument("--cpu-steps", type=int, default=150)
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
    for f in ("step.hip", "arm.h", "geom.h", "hull.h", "sim_internal.h", "mlp_mfma.h", "mlp.hip"):
        p = os.path.join(ROOT, "paper_2106_14405_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def window_tag(workload, mode, settle, tol, cap, n_scenes):
    return f"{workload}{n_scenes}-settle{settle}-{mode}-tol{tol:g}-cap{cap}"


def measured_traffic(workload, tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and on the same window; else None."""
    p = os.path.join(ROOT, "profiles", f"step_kernel_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != kernel_hash() or d.get("window") != tag:
        return None
    return d.get("hbm_bytes_per_launch")


def progress(msg):
    """One line on stderr per finished phase."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    lim = os.environ.get("OMP_NUM_THREADS")
    if lim and lim.isdigit() and int(lim) > 0:
        n = min(n, int(lim))
    return max(1, n)


def cpu_baseline(batch, settle, timed_steps, cap, tol, warm, arm):
    """The FP64 oracle on the host cores: the same workload on a sample of
    scenes (one contiguous chunk per thread), settled in the oracle itself
    (untimed), then `timed_steps` steps at the same tolerance, cap and warm
    start, all threads timed together."""
    from oracle import oracle as O
    from paper_2106_14405_amd import scenes as S
    n = batch.n_scenes
    o = O.OracleSim(batch)
    nth = min(host_threads(), n)
    acts = [S.arm_actions(1, n, t) if arm else None for t in range(settle + timed_steps)]
    w = {"cold": O.COLD, "prev": O.PREV}.get(warm, O.PREV)
    bounds = [(k * n // nth, (k + 1) * n // nth) for k in range(nth)]

    def run(t0, t1, iters, tl, wm):
        errors = []

        def work(s0, s1):
            try:
                for t in range(t0, t1):
                    o.step(actions=acts[t], iters=iters, tol=tl, warm=wm, outputs=False, scenes=(s0, s1))
            except Exception as e:   # re-raised below: a failed chunk must not be timed as done
                errors.append(e)
        th = [threading.Thread(target=work, args=b) for b in bounds]
        start = time.perf_counter()
        for x in th:
            x.start()
        for x in th:
            x.join()
        if errors:
            raise RuntimeError(f"oracle baseline failed in {len(errors)} of {len(th)} threads") from errors[0]
        return time.perf_counter() - start

    run(0, settle, 20, 0.0, O.PREV)
    secs = run(settle, settle + timed_steps, cap, tol, w)
    return dict(value=n * timed_steps / secs, unit="env-steps/s", cores=nth, kind="oracle",
                sample=(f"{n} scenes x {timed_steps} steps of the same workload after {settle} untimed settling steps "
                        f"in the oracle; tolerance {tol:g} m/s, cap {cap}, {warm} start; {nth} host threads, "
                        f"one chunk of scenes each; {secs:.1f} s wall"))


def batch_in_chunks(fn, n, chunk=1024):
    """A batch generated in chunks of scenes (fn(first scene, count)), with a
    progress line per chunk; chunk k uses seeds shifted by its first scene."""
    from paper_2106_14405_amd import scenes as S
    parts = []
    for k in range(0, n, chunk):
        parts.append(fn(k, min(chunk, n - k)))
        progress(f"generated {min(k + chunk, n)} of {n} scenes")
    return concat_batches(parts) if len(parts) > 1 else parts[0]


def concat_batches(parts):
    from paper_2106_14405_amd import scenes as S
    off = [np.zeros(1, np.int32)]
    base = 0
    for b in parts:
        off.append(b.body_offset[1:] + base)
        base += b.n_bodies
    cat = lambda k: np.concatenate([getattr(b, k) for b in parts])
    return S.Batch(body_offset=np.concatenate(off).astype(np.int32), shape=cat("shape"), motion=cat("motion"),
                   param=cat("param"), mass=cat("mass"), friction=cat("friction"), restitution=cat("restitution"),
                   pose=cat("pose"), vel=cat("vel"), arm=parts[0].arm, arm_base=cat("arm_base"),
                   arm_theta=cat("arm_theta"))


def reset_schedule(n_scenes, n_steps, pool_size, seed=7):
    """[n_steps, S] uint8 masks (each scene restarts after U[100, 300] steps)
    and int32 pool entries (a scene's r-th reset takes entry r mod K)."""
    rng = np.random.default_rng(seed)
    m = np.zeros((n_steps, n_scenes), np.uint8)
    idx = np.zeros((n_steps, n_scenes), np.int32)
    done = np.zeros(n_scenes, np.int64)
    nxt = rng.integers(100, 301, size=n_scenes)
    for t in range(n_steps):
        hit = nxt == t
        m[t, hit] = 1
        idx[t] = done % pool_size
        done[hit] += 1
        nxt[hit] += rng.integers(100, 301, size=int(hit.sum()))
    return m, idx


def workload_name(w, n_scenes, batch):
    if w == "clutter":
        return (f"clutter: {n_scenes} scenes x {batch.n_bodies // n_scenes} bodies (20 static boxes, "
                "108 dynamic spheres/boxes/capsules, 7-link kinematic arm), settled")
    if w == "uneven":
        c = batch.counts()
        return (f"uneven: {n_scenes} drop scenes, {int(c.min())}-{int(c.max())} dynamic spheres/boxes "
                f"(log-uniform), {batch.n_bodies} bodies")
    if w == "scale":
        c = batch.counts() - 27
        return (f"scale: {n_scenes} clutter scenes, {int(c.min())}-{int(c.max())} dynamic spheres/boxes/capsules "
                f"(log-uniform, mean {c.mean():.0f}) + 20 static boxes + 7-link kinematic arm, {batch.n_bodies} "
                "bodies, settled")
    return f"drop: {n_scenes} scenes x 64 dynamic bodies (32 spheres + 32 boxes), settled"


def learned_vs_plain(n_scenes, steps):
    """Held-out small drop scenes (64 bodies, seeds 2000+) at residual 1e-4,
    cap 200 sweeps: plain PGS (cold), classic warm start, the committed
    learned warm start; paired per-scene differences with 95% intervals."""
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd import train as T
    path = os.path.join(ROOT, "paper_2106_14405_amd", "weights", "warmstart_drop.npz")
    if not os.path.exists(path):
        return None
    net = T.load(path)
    res, raw = {}, {}
    for name, mode in (("cold", L.COLD), ("prev", L.PREV), ("learned", L.LEARNED)):
        r = T.evaluate(mode, net if mode == L.LEARNED else None, n_scenes=n_scenes, seed0=2000, steps=steps,
                       tol=1e-4, cap=200)
        raw[name] = r
        res[name] = T.summary(r)
    res["learned_minus_prev"] = T.paired(raw["learned"], raw["prev"])
    res["learned_minus_cold"] = T.paired(raw["learned"], raw["cold"])
    res["workload"] = (f"{n_scenes} held-out drop scenes x {steps} steps, tolerance 1e-4 m/s, cap 200 sweeps; "
                       "mean/p50/p95 sweeps per scene-step with contacts, ms per step of the whole batch; "
                       "paired: per-scene mean sweeps and per-step ms, mean difference and 95% interval")
    return res


def extra_mode(batch, acts, a, max_contacts, max_pairs, cap, dev, workload):
    """A variant of the clutter workload (the articulated arm with the same
    per-step action rates as motor-target rates; cabinets with doors and
    drawers; convex hulls): settled like the headline, then the same window
    timed with the classic warm start at the same tolerance and cap."""
    import torch
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    sim = Sim(batch, max_contacts=max_contacts, max_pairs=max_pairs, warm=L.PREV, tol=0.0, threads=a.threads,
              device=dev)
    K, W, T0 = a.steps, a.warmup, a.settle
    act = (lambda t: acts[t]) if batch.arm else (lambda t: None)
    for t in range(T0):
        sim.step(act(t), DT, 20)
    sim.set_solver(L.PGS, L.PREV, a.tol)
    for t in range(W):
        sim.step(act(T0 + t), DT, cap)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(sim.stream)
    for t in range(K):
        sim.step(act(T0 + W + t), DT, cap)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # statistics of the last timed step (a replay of the window would double the run)
    r = dict(ms_per_step=ms / K, env_steps_per_s=batch.n_scenes * K / (ms / 1e3), workload=workload,
             bodies_per_scene=float(batch.n_bodies / batch.n_scenes),
             last_step_sweeps_mean=float(sim.stats["sweeps"].float().mean().item()),
             last_step_frac_at_tol=float((sim.stats["residual"] <= a.tol).float().mean().item()),
             last_step_contacts_mean=float(sim.stats["contacts"].float().mean().item()))
    if sim.arm_state is not None:
        r["last_step_arm_force_mean_N"] = float(sim.stats["arm_force"].mean().item())
        r["joint_rate_max"] = float(sim.arm_state[:, 0].abs().max().item())
    if sim.joint_state is not None:
        js = sim.joint_state.cpu().numpy()
        parts = batch.joint > 0
        r["parts_per_scene"] = float(parts.sum() / batch.n_scenes)
        r["parts_moved_frac"] = float(np.mean(np.abs(js[0, parts]) > 1e-3))
    sim.close()
    del sim
    torch.cuda.synchronize()
    return r


def _hull_scene(seed):
    from paper_2106_14405_amd import scenes as S
    return S.drop_scene(seed, n_spheres=27, n_boxes=27, n_capsules=27, n_hulls=27, size=(0.03, 0.3), edge=4.0)


def summarise(sweeps, resid, flags, contacts, tol):
    """Statistics over scene-steps [K, S] (scene-steps with contacts for sweeps)."""
    from paper_2106_14405_amd import _lib as L
    m = contacts > 0
    s = sweeps[m].astype(np.float64)
    pct = lambda q: float(np.percentile(s, q)) if s.size else 0.0
    return dict(sweeps_mean=float(s.mean()) if s.size else 0.0, sweeps_p50=pct(50), sweeps_p95=pct(95),
                sweeps_p99=pct(99), sweeps_max=int(s.max()) if s.size else 0,
                worst_scene_sweeps_mean=float(sweeps.max(axis=1).mean()),
                frac_at_tol=float(np.mean(resid <= tol)), median_residual=float(np.median(resid)),
                frac_fellback=float(np.mean((flags & L.FLAG_FELLBACK) != 0)),
                frac_capacity_or_nonfinite=float(np.mean((flags & (L.FLAG_NONFINITE | L.FLAG_CAPACITY)) != 0)),
                contacts_per_scene=float(contacts.mean()))


def main():
    a = parse()
    if a.probe_copy_mib:
        probe_copy(a.probe_copy_mib)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    from paper_2106_14405_amd import scenes as S
    if a.workload == "clutter":
        n_scenes = a.scenes or 1024
        batch_fn = lambda n: S.batch_clutter(n, seed0=10000)
        arm = True
        max_contacts = a.max_contacts or 512
        max_pairs = a.max_pairs or max_contacts
        cap = a.cap or 1000
    elif a.workload == "scale":
        n_scenes = a.scenes or 16384
        batch_fn = lambda n: batch_in_chunks(lambda k, m: S.batch_scale(m, seed0=30000 + k, lo=64, hi=1024), n)
        arm = True
        max_contacts = a.max_contacts or 4096
        max_pairs = a.max_pairs or 6144    # a settled 1,024-body pile reaches 3.9 pairs per body
        cap = a.cap or 500
    elif a.workload == "uneven":
        n_scenes = a.scenes or 4096
        batch_fn = lambda n: S.batch_uneven(n, seed0=20000, lo=16, hi=512)
        arm = False
        max_contacts = a.max_contacts or 2048
        max_pairs = a.max_pairs or 2560   # 512-body piles reach 4.2 pairs per body
        cap = a.cap or 1000
    else:
        n_scenes = a.scenes or 1024
        batch_fn = lambda n: S.batch_drop(n, seed0=0)
        arm = False
        max_contacts = a.max_contacts or 384
        max_pairs = a.max_pairs or max_contacts
        cap = a.cap or 1000
    if a.tol is None:
        a.tol = 1e-5 if a.workload == "scale" else 1e-4
    if a.headline is None:
        a.headline = "learned" if a.workload == "scale" else "prev"
    modes = [m for m in a.modes.split(",") if m]
    if a.headline not in modes:
        modes.append(a.headline)
    # every host-side input is generated before the GPU is touched
    batch = batch_fn(n_scenes)
    extra = []   # (name, batch, description): variants of the clutter workload
    if a.workload == "clutter" and a.arm_eval:
        extra.append(("prev_articulated_arm", S.batch_clutter(n_scenes, seed0=10000, arm=2),
                      "clutter scenes with the articulated arm (dynamic links of 2.0-0.5 kg, Kp 0.3, 10 N s)"))
        extra.append(("prev_cabinets", S.batch_clutter(n_scenes, seed0=10000, arm=2, cabinets=2),
                      "the articulated-arm clutter with 2 cabinets a scene (a hinged door and a drawer each)"))
        extra.append(("prev_hulls", S.pack(S._map(_hull_scene, [10000 + s for s in range(n_scenes)], None)),
                      "drop scenes of 27 spheres, 27 boxes, 27 capsules and 27 convex hulls (prisms, bipyramids, "
                      "chamfered boxes), sizes 0.03-0.3 m, dropped in a 4 m cube"))
    pool = S.reset_pool(batch, a.pool, seed=40000, kind="drop") if a.workload == "uneven" else None
    cpu_batch = None
    if a.cpu_baseline and a.workload != "uneven":
        cpu_batch = batch_fn(a.cpu_scenes_per_thread * host_threads())
    K, W, T0 = a.steps, a.warmup, a.settle
    Wmax = max(W, 2 * a.sleep_steps) if any(m.endswith("_sleep") for m in modes) else W
    acts_np = (np.stack([S.arm_actions(1, n_scenes, t) for t in range(T0 + Wmax + K)]) if arm else None)

    import torch

    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd import train as TR
    from paper_2106_14405_amd.sim import Sim
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sim = Sim(batch, max_contacts=max_contacts, max_pairs=max_pairs, warm=L.PREV, tol=0.0, threads=a.threads,
              device=dev)
    acts = torch.as_tensor(acts_np, device=dev) if arm else None
    resets = None
    tuned = None
    persistent = a.workload in ("uneven", "scale") and a.launch != "plain"
    if persistent:
        sim.set_persistent(True)
        mask = sim.autotune(steps=3, dt=DT, iters=20)
        edges = ["1-16", "17-32", "33-64", "65-128", "129-256", "257-512", "513-1024", "1025-2046"]
        tuned = {e: ("wave" if (mask >> k) & 1 else "workgroup") for k, e in enumerate(edges)}
        progress(f"autotuned routing: {tuned}")
    if a.workload == "uneven":
        masks, index = reset_schedule(n_scenes, T0 + Wmax + K, a.pool)
        resets = torch.as_tensor(masks, device=dev)
        reset_index = torch.as_tensor(index, device=dev)
        pool_pose = torch.as_tensor(np.ascontiguousarray(pool[0].transpose(0, 2, 1)), device=dev)
        pool_vel = torch.as_tensor(np.ascontiguousarray(pool[1].transpose(0, 2, 1)), device=dev)
    net = None
    if "learned" in modes:
        wpath = os.path.join(ROOT, "paper_2106_14405_amd", "weights", "warmstart_drop.npz")
        net = TR.load(wpath, device=str(dev))
        net.attach(sim)

    def one(t, iters):
        if resets is not None:
            sim.reset(resets[t], pool_pose, pool_vel, None, reset_index[t])
        sim.step(acts[t] if arm else None, DT, iters)

    # settle (untimed): classic warm start, 20 sweeps per step
    sim.set_solver(L.PGS, L.PREV, 0.0)
    for t in range(T0):
        one(t, 20)
    torch.cuda.synchronize()
    settled = sim.save_state()
    contacts_settled = float(sim.stats["contacts"].float().mean().item())
    progress(f"settled {T0} steps, {contacts_settled:.1f} contacts per scene")

    results = {}
    for name in modes:
        sleep = name.endswith("_sleep")
        mode = {"cold": L.COLD, "prev": L.PREV, "learned": L.LEARNED}[name[:-6] if sleep else name]
        sim.load_state(settled)
        sim.set_sleep(0.0, 0)
        sim.set_solver(L.PGS, mode, a.tol)
        # sleeping: the rest counters start at zero after the settling, so the
        # untimed warm-up lasts long enough for islands to fall asleep
        Wm = max(W, 2 * a.sleep_steps) if sleep else W
        if sleep:
            sim.set_sleep(a.sleep_speed, a.sleep_steps)
        for t in range(Wm):
            one(T0 + t, cap)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        for t in range(K):
            one(T0 + Wm + t, cap)
        ev1.record(sim.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        r = dict(ms_per_step=ms / K, env_steps_per_s=n_scenes * K / (ms / 1e3))
        if not a.no_replay:
            # replay of the same W + K steps from the same state: bit-identical
            # to the timed steps; statistics of the K timed ones
            sim.load_state(settled)
            for t in range(Wm):
                one(T0 + t, cap)
            rec = {k: torch.zeros((K, n_scenes), dtype=v.dtype, device=dev)
                   for k, v in sim.stats.items() if k in ("sweeps", "residual", "flags", "contacts", "pairs", "colours")}
            for t in range(K):
                one(T0 + Wm + t, cap)
                for k in rec:
                    rec[k][t].copy_(sim.stats[k])
            torch.cuda.synchronize()
            rec = {k: v.cpu().numpy() for k, v in rec.items()}
            r.update(summarise(rec["sweeps"], rec["residual"], rec["flags"], rec["contacts"], a.tol))
            r["pairs_per_scene"] = float(rec["pairs"].mean())
            r["colours_per_scene"] = float(rec["colours"].mean())
        if sleep:
            r["sleep"] = dict(speed_m_per_s=a.sleep_speed, steps=a.sleep_steps, untimed_warmup=Wm)
        results[name] = r
        progress(f"{name}: {r['ms_per_step']:.3f} ms per step")
    sim.set_sleep(0.0, 0)
    sim.close()
    del sim
    torch.cuda.synchronize()
    for name, xb, desc in extra:
        results[name] = extra_mode(xb, acts, a, max_contacts, max_pairs, cap, dev, desc)
        progress(f"{name}: {results[name]['ms_per_step']:.3f} ms per step")

    head = results[a.headline]
    motion = batch.motion
    n_dyn = int(np.sum(motion == S.DYNAMIC))
    n_other = int(batch.n_bodies - n_dyn)
    contacts = head.get("contacts_per_scene", contacts_settled)
    bytes_launch = B_DYN * n_dyn + B_STATIC * n_other + B_CONTACT * contacts * n_scenes
    ms_step = head["ms_per_step"]
    achieved = bytes_launch / (ms_step / 1e3) / 1e9
    tag = window_tag(a.workload, a.headline, T0, a.tol, cap, n_scenes)
    traffic = measured_traffic(a.workload, tag)
    kname = "step_persistent" if persistent else "step_kernel"
    sweep_bytes = B_SWEEP * contacts * n_scenes * head.get("sweeps_mean", 0.0)
    out = {
        "metric": METRIC,
        "value": head["env_steps_per_s"],
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
            "dt": DT, "tolerance_m_per_s": a.tol, "sweep_cap": cap, "warm_start": a.headline, "solver": "pgs",
            "settle_steps": T0, "contacts_per_scene_settled": contacts_settled,
            "frac_scene_steps_at_tol": head.get("frac_at_tol"),
            "threads_per_scene": a.threads if not persistent else "autotuned: 64 (one wave) or 256",
            "max_contacts_per_scene": max_contacts, "max_pairs_per_scene": max_pairs,
            **({"launch": "persistent, HIP graph" if persistent else "one workgroup per scene",
                "routing_by_body_count": tuned,
                "resets": f"each scene after U[100, 300] steps, from a pool of {a.pool} fresh states per scene"}
               if a.workload == "uneven" else {}),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kname, "bytes_per_launch": bytes_launch, "window": tag,
            "sweep_equivalent_GBs": sweep_bytes / (ms_step / 1e3) / 1e9,
        },
        "modes": results,
        "solver_stats": {
            "sweeps_learned": results.get("learned", {}).get("sweeps_mean"),
            "sweeps_plain": results.get("cold", {}).get("sweeps_mean"),
            "sweeps_prev": results.get("prev", {}).get("sweeps_mean"),
        },
        "cpu_baseline": None,
    }
    if a.learned_eval:
        lv = learned_vs_plain(a.learned_scenes, a.learned_steps)
        if lv is not None:
            out["learned_vs_plain"] = lv
        progress("learned vs plain done")
    if cpu_batch is not None:
        out["cpu_baseline"] = cpu_baseline(cpu_batch, T0, a.cpu_steps, cap, a.tol, a.headline, arm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
