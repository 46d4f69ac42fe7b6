"""Python handle over the HIP library: torch owns the device memory and the
stream, the library does all the physics.

    sim = Sim(batch, max_contacts=512)
    sim.step(actions, dt=1/120, iters=20)
    pose = sim.pose          # [7, N] device tensor view (x y z qw qx qy qz)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from . import scenes

DEFAULT_CONSTS = dict(margin=0.02, baumgarte=0.2, slop=0.005, rest_thresh=0.5, ground_friction=0.5,
                      ground_restitution=0.0, gravity=(0.0, 0.0, -9.81), link_len=scenes.ARM_LINK_LENGTH,
                      arm_radius=scenes.ARM_RADIUS)


def _np_ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Sim:
    """A batch of scenes resident in one device workspace."""

    def __init__(self, batch: scenes.Batch, max_pairs: int | None = None, max_contacts: int | None = None,
                 solver: int = L.PGS, warm: int = L.COLD, tol: float = 0.0, threads: int = 64,
                 device: str | torch.device = "cuda", hbm_min_bodies: int = 0, **consts):
        lib = L.load()
        c = dict(DEFAULT_CONSTS)
        c.update(consts)
        self.consts = c
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.batch = batch
        self.S = batch.n_scenes
        self.N = batch.n_bodies
        nmax = int(np.max(batch.counts()))
        self.max_pairs = int(max_pairs or max(64, 6 * nmax))
        self.max_contacts = int(max_contacts or max(64, 6 * nmax))
        self._host = dict(
            off=np.ascontiguousarray(batch.body_offset, np.int32),
            shape=np.ascontiguousarray(batch.shape, np.uint8),
            motion=np.ascontiguousarray(batch.motion, np.uint8),
            param=np.ascontiguousarray(batch.param, np.float32).reshape(-1),
            mass=np.ascontiguousarray(batch.mass, np.float32),
            friction=np.ascontiguousarray(batch.friction, np.float32),
            restitution=np.ascontiguousarray(batch.restitution, np.float32),
            pose=np.ascontiguousarray(batch.pose, np.float32).reshape(-1),
            vel=np.ascontiguousarray(batch.vel, np.float32).reshape(-1),
            arm_base=np.ascontiguousarray(batch.arm_base, np.float32).reshape(-1),
            arm_theta=np.ascontiguousarray(batch.arm_theta, np.float32).reshape(-1),
        )
        self.has_parts = getattr(batch, "joint", None) is not None
        if self.has_parts:
            h2 = self._host
            h2["joint"] = np.ascontiguousarray(batch.joint, np.uint8)
            h2["joint_axis"] = np.ascontiguousarray(batch.joint_axis, np.float32).reshape(-1)
            h2["joint_anchor"] = np.ascontiguousarray(batch.joint_anchor, np.float32).reshape(-1)
            h2["joint_limits"] = np.ascontiguousarray(batch.joint_limits, np.float32).reshape(-1)
            h2["joint_parent"] = np.ascontiguousarray(batch.joint_parent, np.int32)
        self.has_hulls = getattr(batch, "hull_index", None) is not None
        if self.has_hulls:
            self._host["hull_index"] = np.ascontiguousarray(batch.hull_index, np.int32).reshape(-1)
            self._host["hull_vert"] = np.ascontiguousarray(batch.hull_vert, np.float32).reshape(-1)
            self._host["hull_face"] = np.ascontiguousarray(batch.hull_face, np.int32).reshape(-1)
        h = self._host
        d = L.BatchDesc()
        d.abi_version = L.SIM_ABI_VERSION
        d.num_scenes = self.S
        d.h_body_offset = _np_ptr(h["off"], C.c_int32)
        d.h_shape = _np_ptr(h["shape"], C.c_uint8)
        d.h_motion = _np_ptr(h["motion"], C.c_uint8)
        d.h_param = _np_ptr(h["param"], C.c_float)
        d.h_mass = _np_ptr(h["mass"], C.c_float)
        d.h_friction = _np_ptr(h["friction"], C.c_float)
        d.h_restitution = _np_ptr(h["restitution"], C.c_float)
        d.h_pose = _np_ptr(h["pose"], C.c_float)
        d.h_vel = _np_ptr(h["vel"], C.c_float)
        d.arm = int(batch.arm)
        d.h_arm_base = _np_ptr(h["arm_base"], C.c_float)
        d.h_arm_theta = _np_ptr(h["arm_theta"], C.c_float)
        for i in range(7):
            d.link_len[i] = c["link_len"][i]
        d.arm_radius = c["arm_radius"]
        for i in range(3):
            d.gravity[i] = c["gravity"][i]
        d.margin, d.baumgarte, d.slop = c["margin"], c["baumgarte"], c["slop"]
        d.rest_thresh, d.ground_friction, d.ground_restitution = (c["rest_thresh"], c["ground_friction"],
                                                                  c["ground_restitution"])
        d.max_pairs, d.max_contacts = self.max_pairs, self.max_contacts
        d.solver, d.warm_start, d.tolerance, d.threads = int(solver), int(warm), float(tol), int(threads)
        d.hbm_min_bodies = int(hbm_min_bodies)
        if self.has_hulls:
            d.n_hulls = int(len(h["hull_index"]) // 4)
            d.h_hull_index = _np_ptr(h["hull_index"], C.c_int32)
            d.h_hull_vert = _np_ptr(h["hull_vert"], C.c_float)
            d.h_hull_face = _np_ptr(h["hull_face"], C.c_int32)
        if self.has_parts:
            d.h_joint = _np_ptr(h["joint"], C.c_uint8)
            d.h_joint_axis = _np_ptr(h["joint_axis"], C.c_float)
            d.h_joint_anchor = _np_ptr(h["joint_anchor"], C.c_float)
            d.h_joint_limits = _np_ptr(h["joint_limits"], C.c_float)
            d.h_joint_parent = _np_ptr(h["joint_parent"], C.c_int32)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            d.stream = C.c_void_p(self.stream.cuda_stream)
            nbytes = lib.sim_workspace_bytes(C.byref(d))
            if nbytes == 0:
                raise L.SimError("invalid batch descriptor: " + lib.sim_last_error().decode())
            self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            handle = C.c_void_p()
            L.check(lib.sim_create(C.byref(d), C.c_void_p(self.ws.data_ptr()), C.c_size_t(nbytes),
                                   C.byref(handle)), "sim_create")
        self.h = handle
        self.desc = d
        self._mlp = None
        self._views()

    # ------------------------------------------------------------------ views
    def _view(self, ptr, dtype, shape):
        if not ptr:
            return None
        base = self.ws.data_ptr()
        off = int(ptr) - base
        n = int(np.prod(shape)) * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + n].view(dtype).view(*shape)

    def _views(self):
        lib = L.load()
        sv = L.StateView()
        L.check(lib.sim_state(self.h, C.byref(sv)), "sim_state")
        S, N, CM, PM = self.S, self.N, self.max_contacts, self.max_pairs
        self.pose = self._view(sv.pose, torch.float32, (7, N))
        self.vel = self._view(sv.vel, torch.float32, (6, N))
        self.rest = self._view(sv.rest, torch.int32, (N,))
        self.theta = self._view(sv.theta, torch.float32, (S, 7)) if self.batch.arm else None
        # articulated arm: [S, 3, 7] joint rates, motor targets, last motor impulses
        self.arm_state = self._view(sv.arm_state, torch.float32, (S, 3, 7)) if int(self.batch.arm) == 2 else None
        # container parts: [2, N] joint coordinates q and rates qd (0 for other bodies)
        self.joint_state = self._view(sv.joint_state, torch.float32, (2, N)) if self.has_parts else None
        st = L.StatsView()
        L.check(lib.sim_stats(self.h, C.byref(st)), "sim_stats")
        self.stats = dict(
            pairs=self._view(st.pairs, torch.int32, (S,)), contacts=self._view(st.contacts, torch.int32, (S,)),
            colours=self._view(st.colours, torch.int32, (S,)), sweeps=self._view(st.sweeps, torch.int32, (S,)),
            flags=self._view(st.flags, torch.int32, (S,)), residual=self._view(st.residual, torch.float32, (S,)),
            arm_force=self._view(st.arm_force, torch.float32, (S,)))

    def cache(self):
        """(count [S], key [S, CM], lam [4, S, CM]) of the contacts the next step warm-starts from."""
        lib = L.load()
        sv = L.StateView()
        L.check(lib.sim_state(self.h, C.byref(sv)), "sim_state")
        S, CM = self.S, self.max_contacts
        return (self._view(sv.cache_count, torch.int32, (S,)),
                self._view(sv.cache_key, torch.int32, (S, CM)),
                self._view(sv.cache_lam, torch.float32, (4, S, CM)))

    def contacts(self):
        """Views of the last step's contacts (exported fields need set_export(True))."""
        lib = L.load()
        cv = L.ContactView()
        L.check(lib.sim_contacts(self.h, C.byref(cv)), "sim_contacts")
        S, CM, PM = self.S, self.max_contacts, self.max_pairs
        return dict(
            count=self._view(cv.count, torch.int32, (S,)), key=self._view(cv.key, torch.int32, (S, CM)),
            normal=self._view(cv.normal, torch.float32, (3, S, CM)),
            point=self._view(cv.point, torch.float32, (3, S, CM)),
            phi=self._view(cv.phi, torch.float32, (S, CM)),
            lam=self._view(cv.lambda_, torch.float32, (3, S, CM)),
            colour=self._view(cv.colour, torch.int32, (S, CM)),
            features=self._view(cv.features, torch.float32, (16, S, CM)),
            n_pairs=self._view(cv.n_pairs, torch.int32, (S,)),
            pair_key=self._view(cv.pair_key, torch.int32, (S, PM)))

    # ------------------------------------------------------------------ calls
    def step(self, actions: torch.Tensor | None = None, dt: float = 1.0 / 120.0, iters: int = 10):
        ptr = None
        if actions is not None:
            if actions.device != self.device or actions.dtype != torch.float32 or not actions.is_contiguous():
                raise ValueError("actions must be a contiguous float32 tensor on the simulation device")
            if actions.numel() != 7 * self.S:
                raise ValueError("actions must hold 7 joint velocities per scene")
            ptr = C.c_void_p(actions.data_ptr())
        L.check(L.load().sim_step(self.h, ptr, float(dt), int(iters)), "sim_step")

    def query_arm(self, theta: torch.Tensor, clearance: float = 0.0, min_phi: bool = True):
        """Collision checks of arm configurations theta [S, M, 7] (float32, rad)
        against the current state: returns hit [S, M] uint8 and, if asked,
        the least separation [S, M] float32 (+inf when none is within the
        clearance)."""
        if theta.device != self.device or theta.dtype != torch.float32 or not theta.is_contiguous():
            raise ValueError("theta must be a contiguous float32 tensor on the simulation device")
        if theta.dim() != 3 or theta.shape[0] != self.S or theta.shape[2] != 7:
            raise ValueError("theta must be [S, M, 7]")
        M = int(theta.shape[1])
        hit = torch.empty((self.S, M), dtype=torch.uint8, device=self.device)
        phi = torch.empty((self.S, M), dtype=torch.float32, device=self.device) if min_phi else None
        L.check(L.load().sim_query_arm(self.h, C.c_void_p(theta.data_ptr()), M, float(clearance),
                                       C.c_void_p(hit.data_ptr()),
                                       C.c_void_p(phi.data_ptr()) if phi is not None else None),
                "sim_query_arm")
        return hit, phi

    def set_motors(self, kp: float = 0.3, max_impulse: float = 10.0):
        """Articulated arm: motor position gain and largest motor impulse per step (N m s)."""
        L.check(L.load().sim_set_motors(self.h, float(kp), float(max_impulse)), "sim_set_motors")

    def set_sleep(self, speed: float = 0.0, steps: int = 0):
        """Sleeping islands on (speed m/s > 0, steps >= 1) or off (speed 0)."""
        L.check(L.load().sim_set_sleep(self.h, float(speed), int(steps)), "sim_set_sleep")

    def set_trace(self, on: bool = True):
        """Per-scene phase timestamps ([S, 16] int64 device tensor) written by every later step."""
        if on:
            self.trace = torch.zeros((self.S, 16), dtype=torch.int64, device=self.device)
            ptr = C.c_void_p(self.trace.data_ptr())
        else:
            self.trace, ptr = None, None
        L.check(L.load().sim_set_trace(self.h, ptr), "sim_set_trace")

    def set_export(self, on: bool = True):
        L.check(L.load().sim_set_export(self.h, int(bool(on))), "sim_set_export")

    def set_solver(self, solver: int = L.PGS, warm: int = L.COLD, tol: float = 0.0):
        L.check(L.load().sim_set_solver(self.h, int(solver), int(warm), float(tol)), "sim_set_solver")

    def set_mlp(self, w1, w2, w3, b1, b2, b3, mean, std):
        """Device tensors: bf16 w1 [64,16], w2 [64,64], w3 [3,64]; fp32 biases, mean, std."""
        ts = [w1.contiguous(), w2.contiguous(), w3.contiguous(), b1.float().contiguous(), b2.float().contiguous(),
              b3.float().contiguous(), mean.float().contiguous(), std.float().contiguous()]
        for t in ts[:3]:
            if t.dtype != torch.bfloat16:
                raise ValueError("weights must be bfloat16")
        self._mlp = ts  # keep alive
        L.check(L.load().sim_set_mlp(self.h, *[C.c_void_p(t.data_ptr()) for t in ts]), "sim_set_mlp")

    def set_persistent(self, on: bool = True, wave_max_bodies: int = -1):
        """Persistent launch over two size-ordered scene queues, replayed from a HIP graph."""
        L.check(L.load().sim_set_persistent(self.h, int(bool(on)), int(wave_max_bodies)), "sim_set_persistent")

    def set_persistent_table(self, wave_buckets: int):
        """Persistent launch routed by a body-count bucket table (bit k: bucket k to single waves)."""
        L.check(L.load().sim_set_persistent_table(self.h, int(wave_buckets)), "sim_set_persistent_table")

    def autotune(self, steps: int = 5, dt: float = 1.0 / 120.0, iters: int = 10) -> int:
        """Times the persistent launch's routing, bucket by bucket, and keeps the
        fastest table (returned as its bit mask); state is unchanged."""
        lib = L.load()
        need = int(lib.sim_autotune_scratch_bytes(self.h))
        scratch = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        out = C.c_uint32(0)
        L.check(lib.sim_autotune(self.h, C.c_void_p(ptr), need, int(steps), float(dt), int(iters), C.byref(out)),
                "sim_autotune")
        return out.value

    def save_state(self) -> torch.Tensor:
        """Device blob of the state (pose, velocity, joint angles, contact caches)."""
        lib = L.load()
        blob = torch.empty(int(lib.sim_state_bytes(self.h)), dtype=torch.uint8, device=self.device)
        L.check(lib.sim_save_state(self.h, C.c_void_p(blob.data_ptr())), "sim_save_state")
        return blob

    def load_state(self, blob: torch.Tensor):
        """Restore a blob from save_state of a simulation with the same batch layout."""
        if blob.device != self.device or blob.dtype != torch.uint8 or not blob.is_contiguous():
            raise ValueError("blob must be a contiguous uint8 tensor on the simulation device")
        L.check(L.load().sim_load_state(self.h, C.c_void_p(blob.data_ptr())), "sim_load_state")

    def reset(self, mask: torch.Tensor, pose: torch.Tensor, vel: torch.Tensor, theta: torch.Tensor | None = None,
              index: torch.Tensor | None = None, joint_state: torch.Tensor | None = None):
        """Masked reset from a pool of K states: pose [K, 7, N], vel [K, 6, N],
        theta [K, S, 7] (arm batches), joint_state [K, 2, N] (batches with
        container parts); a single state may be given without the leading K.
        index: int32 [S] pool entry per scene (None: 0)."""
        pose = pose.reshape(-1, 7, self.N)
        K = pose.shape[0]
        ts = [mask.to(torch.uint8).contiguous(), pose.contiguous(), vel.reshape(K, 6, self.N).contiguous()]
        th = theta.reshape(K, self.S, 7).contiguous() if theta is not None else None
        ix = index.to(torch.int32).contiguous() if index is not None else None
        js = joint_state.reshape(K, 2, self.N).contiguous() if joint_state is not None else None
        self._reset_keep = ts + [th, ix, js]
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        pool = L.ResetPool(K, ptr(ts[1]), ptr(ts[2]), ptr(th), ptr(ix), ptr(js))
        L.check(L.load().sim_reset(self.h, ptr(ts[0]), C.byref(pool)), "sim_reset")

    def close(self):
        if getattr(self, "h", None):
            L.load().sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
