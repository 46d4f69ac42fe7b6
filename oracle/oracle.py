"""ctypes binding of the FP64 oracle (liborace.so built from rbo.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package's smoke() check
and bench.py's cpu_baseline leg; never by the product path.

All arrays handed to the oracle are float64 copies of the float32 inputs
(exact widening) or int32/uint8/uint32 index arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "rbo.c")

COLD, PREV, LEARNED = 0, 1, 2
PGS, JACOBI = 0, 1
F_NONFINITE, F_CAPACITY, F_NOT_CONVERGED, F_FELLBACK = 1, 2, 4, 8

# physics constants of the step (readings; the paper gives none)
DEFAULTS = dict(margin=0.02, baumgarte=0.2, slop=0.005, rest_thresh=0.5,
                ground_friction=0.5, ground_restitution=0.0,
                gravity=(0.0, 0.0, -9.81), link_len=(0.10, 0.30, 0.10, 0.30, 0.10, 0.20, 0.10),
                arm_radius=0.05, motor_kp=0.3, motor_max=10.0)


def build(force: bool = False) -> str:
    """Compile rbo.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O3", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_P = C.POINTER
_d = C.c_double


class Model(C.Structure):
    _fields_ = [("n_scenes", C.c_int), ("body_offset", _P(C.c_int32)), ("shape", _P(C.c_uint8)),
                ("motion", _P(C.c_uint8)), ("param", _P(_d)), ("mass", _P(_d)),
                ("friction", _P(_d)), ("restitution", _P(_d)), ("arm", C.c_int),
                ("arm_base", _P(_d)), ("link_len", _d * 7), ("arm_radius", _d),
                ("gravity", _d * 3), ("margin", _d), ("baumgarte", _d), ("slop", _d),
                ("rest_thresh", _d), ("ground_friction", _d), ("ground_restitution", _d),
                ("sleep_speed", _d), ("sleep_steps", C.c_int), ("motor_kp", _d), ("motor_max", _d),
                ("joint", _P(C.c_uint8)), ("joint_axis", _P(_d)), ("joint_anchor", _P(_d)),
                ("joint_limits", _P(_d)), ("joint_parent", _P(C.c_int32)),
                ("n_hulls", C.c_int), ("hull_index", _P(C.c_int32)), ("hull_vert", _P(_d)),
                ("hull_face", _P(C.c_int32))]


class Cache(C.Structure):
    _fields_ = [("cap", C.c_int), ("count", _P(C.c_int32)), ("key", _P(C.c_uint32)),
                ("lam", _P(_d))]


class Mlp(C.Structure):
    _fields_ = [("w1", _P(_d)), ("b1", _P(_d)), ("w2", _P(_d)), ("b2", _P(_d)),
                ("w3", _P(_d)), ("b3", _P(_d)), ("mean", _P(_d)), ("std", _P(_d)),
                ("bf16", C.c_int)]


class Out(C.Structure):
    _fields_ = [("max_pairs", C.c_int), ("max_contacts", C.c_int),
                ("n_pairs", _P(C.c_int32)), ("pair_key", _P(C.c_uint32)),
                ("n_contacts", _P(C.c_int32)), ("c_key", _P(C.c_uint32)),
                ("c_normal", _P(_d)), ("c_point", _P(_d)), ("c_phi", _P(_d)),
                ("c_lambda", _P(_d)), ("c_colour", _P(C.c_int32)), ("c_feat", _P(_d)),
                ("n_colours", _P(C.c_int32)), ("sweeps", _P(C.c_int32)),
                ("residual", _P(_d)), ("arm_force", _P(_d)), ("flags", _P(C.c_int32)),
                ("ambiguous", _P(C.c_int32)), ("tied", _P(C.c_uint8)), ("tol_gap", _P(_d))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        L.ora_step.argtypes = [_P(Model), _P(_d), _P(_d), _P(_d), _P(C.c_int32), _P(_d), _P(_d), _P(Cache), _P(_d), _d,
                               C.c_int,
                               _d, C.c_int, C.c_int, _P(Mlp), _P(Out), C.c_int, C.c_int]
        L.ora_step.restype = C.c_int
        L.ora_arm_pose.argtypes = [_P(Model), _P(_d), _P(_d)]
        L.ora_collide.argtypes = [C.c_int, _P(_d), _P(_d), C.c_int, _P(_d), _P(_d), C.c_int, _d,
                                  _P(C.c_int), _P(_d), _P(_d), _P(_d), _P(C.c_int)]
        L.ora_collide.restype = C.c_int
        L.ora_collide_hulls.argtypes = [_P(Model), C.c_int, _P(_d), _P(_d), C.c_int, _P(_d), _P(_d), C.c_int, _d,
                                        _P(C.c_int), _P(_d), _P(_d), _P(_d), _P(C.c_int)]
        L.ora_collide_hulls.restype = C.c_int
        L.ora_hull_mass.argtypes = [_P(Model), C.c_int, _d, _P(_d), _P(_d), _P(_d)]
        L.ora_hull_mass.restype = C.c_int
        L.ora_pairs.argtypes = [_P(Model), _P(_d), C.c_int, _P(C.c_uint32), C.c_int]
        L.ora_pairs.restype = C.c_int
        L.ora_arm_query.argtypes = [_P(Model), _P(_d), _P(_d), C.c_int, _d, _P(C.c_uint8), _P(_d),
                                    _P(C.c_int32), C.c_int, C.c_int]
        L.ora_arm_query.restype = C.c_int
        L.ora_mlp_forward.argtypes = [_P(Mlp), _P(_d), C.c_int, _P(_d)]
        L.ora_mlp_loss_grad.argtypes = [_P(Mlp), _P(_d), _P(_d), C.c_int] + [_P(_d)] * 6
        L.ora_mlp_loss_grad.restype = _d
        L.ora_bf16.argtypes = [_d]
        L.ora_bf16.restype = _d
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(_P(ct)) if a is not None else None


class OracleSim:
    """Batched FP64 simulation state driven by the oracle.

    ``batch`` is a packed scene batch (float32 arrays); everything is widened
    to float64 once.  ``cache_cap`` bounds the stored contacts per scene."""

    def __init__(self, batch, cache_cap: int = 4096, **consts):
        c = dict(DEFAULTS)
        c.update(consts)
        self.consts = c
        b = batch
        self.S = b.n_scenes
        self.off = np.ascontiguousarray(b.body_offset, np.int32)
        self.shape = np.ascontiguousarray(b.shape, np.uint8)
        self.motion = np.ascontiguousarray(b.motion, np.uint8)
        self.param = np.ascontiguousarray(b.param, np.float64).reshape(-1)
        self.mass = np.ascontiguousarray(b.mass, np.float64)
        self.friction = np.ascontiguousarray(b.friction, np.float64)
        self.restitution = np.ascontiguousarray(b.restitution, np.float64)
        self.arm = int(b.arm)            # 0 none, 1 kinematic, 2 dynamic with joint motors
        self.arm_base = np.ascontiguousarray(b.arm_base, np.float64).reshape(-1)
        self.pose = np.ascontiguousarray(b.pose, np.float64).reshape(-1).copy()
        self.vel = np.ascontiguousarray(b.vel, np.float64).reshape(-1).copy()
        self.theta = np.ascontiguousarray(b.arm_theta, np.float64).reshape(-1).copy()
        self.rest = np.zeros(int(self.off[-1]), np.int32)   # steps at rest per body (sleeping)
        # dynamic arm: per scene the joint rates, the motor targets and the
        # motor impulses of the last step (7 each); targets start at theta
        self.arm_state = np.zeros((self.S, 3, 7))
        self.arm_state[:, 1] = self.theta.reshape(self.S, 7)
        self.arm_state = self.arm_state.reshape(-1)
        # articulated container parts: per body the joint coordinate and its rate
        self.joint_state = np.zeros(2 * int(self.off[-1]))
        self.has_parts = getattr(b, "joint", None) is not None
        if self.has_parts:
            self.joint = np.ascontiguousarray(b.joint, np.uint8)
            self.joint_axis = np.ascontiguousarray(b.joint_axis, np.float64).reshape(-1)
            self.joint_anchor = np.ascontiguousarray(b.joint_anchor, np.float64).reshape(-1)
            self.joint_limits = np.ascontiguousarray(b.joint_limits, np.float64).reshape(-1)
            self.joint_parent = np.ascontiguousarray(b.joint_parent, np.int32)
        self.m = Model()
        self.m.n_scenes = self.S
        self.m.body_offset = _ptr(self.off, C.c_int32)
        self.m.shape = _ptr(self.shape, C.c_uint8)
        self.m.motion = _ptr(self.motion, C.c_uint8)
        self.m.param = _ptr(self.param, _d)
        self.m.mass = _ptr(self.mass, _d)
        self.m.friction = _ptr(self.friction, _d)
        self.m.restitution = _ptr(self.restitution, _d)
        self.m.arm = self.arm
        self.m.arm_base = _ptr(self.arm_base, _d)
        for i in range(7):
            self.m.link_len[i] = c["link_len"][i]
        self.m.arm_radius = c["arm_radius"]
        for i in range(3):
            self.m.gravity[i] = c["gravity"][i]
        for k in ("margin", "baumgarte", "slop", "rest_thresh", "ground_friction",
                  "ground_restitution", "motor_kp", "motor_max"):
            setattr(self.m, k, c[k])
        if self.has_parts:
            self.m.joint = _ptr(self.joint, C.c_uint8)
            self.m.joint_axis = _ptr(self.joint_axis, _d)
            self.m.joint_anchor = _ptr(self.joint_anchor, _d)
            self.m.joint_limits = _ptr(self.joint_limits, _d)
            self.m.joint_parent = _ptr(self.joint_parent, C.c_int32)
        self.has_hulls = getattr(b, "hull_index", None) is not None
        if self.has_hulls:
            self._hulls = set_hulls(self.m, b.hull_index, b.hull_vert, b.hull_face)
        self.cache_cap = cache_cap
        self.c_count = np.zeros(self.S, np.int32)
        self.c_key = np.zeros(self.S * cache_cap, np.uint32)
        self.c_lam = np.zeros(self.S * cache_cap * 4, np.float64)
        self.cache = Cache(cache_cap, _ptr(self.c_count, C.c_int32), _ptr(self.c_key, C.c_uint32),
                           _ptr(self.c_lam, _d))
        if self.arm:
            lib().ora_arm_pose(C.byref(self.m), _ptr(self.pose, _d), _ptr(self.theta, _d))
        self._mlp_keep = None

    def set_motors(self, kp: float, max_impulse: float):
        """Dynamic arm: motor position gain and largest impulse per step (N s)."""
        self.m.motor_kp = float(kp)
        self.m.motor_max = float(max_impulse)

    @property
    def q(self):
        """Container parts: joint coordinates [N] (a view; 0 for other bodies)."""
        return self.joint_state.reshape(-1, 2)[:, 0]

    @property
    def q_rate(self):
        """Container parts: joint rates [N] (a view)."""
        return self.joint_state.reshape(-1, 2)[:, 1]

    @property
    def qd(self):
        """Dynamic arm: joint rates [S, 7] (a view)."""
        return self.arm_state.reshape(self.S, 3, 7)[:, 0]

    @property
    def target(self):
        """Dynamic arm: motor targets [S, 7] (a view)."""
        return self.arm_state.reshape(self.S, 3, 7)[:, 1]

    @property
    def motor_impulse(self):
        """Dynamic arm: motor impulses of the last step [S, 7] (a view)."""
        return self.arm_state.reshape(self.S, 3, 7)[:, 2]

    def set_sleep(self, speed: float, steps: int):
        """Sleeping islands on (speed m/s > 0, steps >= 1) or off (speed 0)."""
        self.m.sleep_speed = float(speed)
        self.m.sleep_steps = int(steps)

    # ---------------------------------------------------------------- state
    def set_state(self, pose, vel, theta=None, cache=None, rest=None, arm_state=None, joint_state=None):
        """Overwrite the state with (float32) arrays, widened exactly."""
        self.pose[:] = np.asarray(pose, np.float64).reshape(-1)
        self.vel[:] = np.asarray(vel, np.float64).reshape(-1)
        if joint_state is not None:
            self.joint_state[:] = np.asarray(joint_state, np.float64).reshape(-1)
        if arm_state is not None:
            self.arm_state[:] = np.asarray(arm_state, np.float64).reshape(-1)
        if rest is not None:
            self.rest[:] = np.asarray(rest, np.int32).reshape(-1)
        if theta is not None:
            self.theta[:] = np.asarray(theta, np.float64).reshape(-1)
        if cache is not None:
            cnt, key, lam = cache
            self.c_count[:] = cnt
            self.c_key[:] = 0
            self.c_lam[:] = 0
            kk = self.c_key.reshape(self.S, -1)
            ll = self.c_lam.reshape(self.S, -1, 4)
            kk[:, :key.shape[1]] = key
            ll[:, :lam.shape[1]] = lam

    def set_theta(self, theta):
        """Set the arm joint angles (float64) and recompute the arm link poses."""
        self.theta[:] = np.asarray(theta, np.float64).reshape(-1)
        lib().ora_arm_pose(C.byref(self.m), _ptr(self.pose, _d), _ptr(self.theta, _d))

    def state32(self):
        return (self.pose.reshape(-1, 7).astype(np.float32), self.vel.reshape(-1, 6).astype(np.float32),
                self.theta.reshape(-1, 7).astype(np.float32))

    def cache_arrays(self):
        return (self.c_count.copy(), self.c_key.reshape(self.S, -1).copy(),
                self.c_lam.reshape(self.S, -1, 4).copy())

    def set_mlp(self, params: dict, bf16: bool = False):
        keep = {k: np.ascontiguousarray(np.asarray(params[k], np.float64).reshape(-1))
                for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mean", "std")}
        self._mlp_keep = keep
        self.mlp = Mlp(*[_ptr(keep[k], _d) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mean", "std")],
                       int(bf16))

    # ---------------------------------------------------------------- queries
    def arm_query(self, theta_q, clearance=0.0, scenes=None):
        """Collision checks of arm configurations theta_q [S, M, 7] (float64)
        against the current state.  Returns (hit [S, M] uint8, min_phi [S, M],
        ambiguous [S, M] int32)."""
        q = np.ascontiguousarray(np.asarray(theta_q, np.float64))
        if q.ndim != 3 or q.shape[0] != self.S or q.shape[2] != 7:
            raise ValueError("theta_q must be [S, M, 7]")
        M = q.shape[1]
        hit = np.zeros((self.S, M), np.uint8)
        phi = np.full((self.S, M), np.inf)
        amb = np.zeros((self.S, M), np.int32)
        s0, s1 = (0, self.S) if scenes is None else scenes
        rc = lib().ora_arm_query(C.byref(self.m), _ptr(self.pose, _d), _ptr(q, _d), int(M), float(clearance),
                                 _ptr(hit, C.c_uint8), _ptr(phi, _d), _ptr(amb, C.c_int32), int(s0), int(s1))
        if rc != 0:
            raise ValueError("oracle rejected the query arguments")
        return hit, phi, amb

    # ---------------------------------------------------------------- step
    def step(self, actions=None, dt=1.0 / 120.0, iters=10, tol=0.0, warm=COLD, solver=PGS,
             scenes=None, outputs=True, max_pairs=8192, max_contacts=8192, use_cache=True):
        s0, s1 = (0, self.S) if scenes is None else scenes
        out = None
        res = None
        if outputs:
            S = self.S
            res = dict(
                n_pairs=np.zeros(S, np.int32), pair_key=np.zeros(S * max_pairs, np.uint32),
                n_contacts=np.zeros(S, np.int32), c_key=np.zeros(S * max_contacts, np.uint32),
                c_normal=np.zeros(S * max_contacts * 3), c_point=np.zeros(S * max_contacts * 3),
                c_phi=np.zeros(S * max_contacts), c_lambda=np.zeros(S * max_contacts * 3),
                c_colour=np.zeros(S * max_contacts, np.int32),
                c_feat=np.zeros(S * max_contacts * 16),
                n_colours=np.zeros(S, np.int32), sweeps=np.zeros(S, np.int32),
                residual=np.zeros(S), arm_force=np.zeros(S), flags=np.zeros(S, np.int32),
                ambiguous=np.zeros(S, np.int32), tied=np.zeros(int(self.off[-1]), np.uint8),
                tol_gap=np.zeros(S))
            out = Out()
            out.max_pairs = max_pairs
            out.max_contacts = max_contacts
            for k, v in res.items():
                ct = {np.dtype(np.int32): C.c_int32, np.dtype(np.uint32): C.c_uint32,
                      np.dtype(np.uint8): C.c_uint8, np.dtype(np.float64): _d}[v.dtype]
                setattr(out, k, _ptr(v, ct))
        act = None
        if actions is not None:
            act = np.ascontiguousarray(np.asarray(actions, np.float64).reshape(-1))
        mlp = C.byref(self.mlp) if warm == LEARNED else None
        rc = lib().ora_step(C.byref(self.m), _ptr(self.pose, _d), _ptr(self.vel, _d),
                            _ptr(self.theta, _d), _ptr(self.rest, C.c_int32), _ptr(self.arm_state, _d),
                            _ptr(self.joint_state, _d),
                            C.byref(self.cache) if use_cache else None,
                            _ptr(act, _d) if act is not None else None, dt, int(iters), float(tol),
                            int(warm), int(solver), mlp, C.byref(out) if out is not None else None,
                            s0, s1)
        if rc != 0:
            raise ValueError("oracle rejected the step arguments")
        if res is None:
            return None
        mp, mc = max_pairs, max_contacts
        res["pair_key"] = res["pair_key"].reshape(self.S, mp)
        res["c_key"] = res["c_key"].reshape(self.S, mc)
        res["c_normal"] = res["c_normal"].reshape(self.S, mc, 3)
        res["c_point"] = res["c_point"].reshape(self.S, mc, 3)
        res["c_phi"] = res["c_phi"].reshape(self.S, mc)
        res["c_lambda"] = res["c_lambda"].reshape(self.S, mc, 3)
        res["c_colour"] = res["c_colour"].reshape(self.S, mc)
        res["c_feat"] = res["c_feat"].reshape(self.S, mc, 16)
        return res


def set_hulls(m, hull_index, hull_vert, hull_face):
    """Point the model's hull fields at float64 / int32 copies of a hull
    library; returns the arrays (keep them alive with the model)."""
    keep = (np.ascontiguousarray(hull_index, np.int32).reshape(-1),
            np.ascontiguousarray(hull_vert, np.float64).reshape(-1),
            np.ascontiguousarray(hull_face, np.int32).reshape(-1))
    m.n_hulls = len(keep[0]) // 4
    m.hull_index = _ptr(keep[0], C.c_int32)
    m.hull_vert = _ptr(keep[1], _d)
    m.hull_face = _ptr(keep[2], C.c_int32)
    return keep


def hull_library(hulls):
    """(index [H,4], vertices [V,3], faces [F,8]) of a list of (vertices, face loops)."""
    idx, vs, fs = [], [], []
    nv = nf = 0
    for V, F in hulls:
        idx.append((nv, len(V), nf, len(F)))
        vs.append(np.asarray(V, np.float64))
        for f in F:
            row = np.full(8, -1, np.int32)
            row[:len(f)] = f
            fs.append(row)
        nv += len(V)
        nf += len(F)
    return np.asarray(idx, np.int32), np.concatenate(vs), np.asarray(fs, np.int32)


def hull_mass(hulls, h, mass):
    """(inertia [3,3] about the body origin, centre of mass [3], volume) of hull h."""
    m = Model()
    keep = set_hulls(m, *hull_library(hulls))
    I = np.zeros(9)
    c = np.zeros(3)
    v = C.c_double(0.0)
    if lib().ora_hull_mass(C.byref(m), int(h), float(mass), _ptr(I, _d), _ptr(c, _d), C.byref(v)) != 0:
        raise ValueError("unusable hull")
    del keep
    return I.reshape(3, 3), c, v.value


def collide(shape_a, param_a, pose_a, shape_b=None, param_b=None, pose_b=None, margin=0.02, hulls=None):
    """Contacts of one pair (b = ground when shape_b is None).  Returns a list
    of (feature, normal[3], point[3], phi) and the ambiguity count.  hulls:
    a list of (vertices, face loops) that HULL shapes index by param[0]."""
    L = lib()
    pa = np.ascontiguousarray(param_a, np.float64)
    xa = np.ascontiguousarray(pose_a, np.float64)
    ground = shape_b is None
    pb = np.ascontiguousarray(param_b if not ground else np.zeros(3), np.float64)
    xb = np.ascontiguousarray(pose_b if not ground else [0, 0, 0, 1, 0, 0, 0], np.float64)
    f = np.zeros(4, np.int32)
    n = np.zeros(12)
    p = np.zeros(12)
    ph = np.zeros(4)
    amb = C.c_int(0)
    m = Model()
    keep = set_hulls(m, *hull_library(hulls)) if hulls else None
    k = L.ora_collide_hulls(C.byref(m), int(shape_a), _ptr(pa, _d), _ptr(xa, _d), int(shape_b or 0), _ptr(pb, _d),
                            _ptr(xb, _d), int(ground), float(margin), f.ctypes.data_as(_P(C.c_int)),
                            _ptr(n, _d), _ptr(p, _d), _ptr(ph, _d), C.byref(amb))
    del keep
    if k < 0:
        raise ValueError("oracle rejected the pair")
    return [(int(f[i]), n[3 * i:3 * i + 3].copy(), p[3 * i:3 * i + 3].copy(), float(ph[i]))
            for i in range(k)], amb.value


def bf16(x: float) -> float:
    return lib().ora_bf16(float(x))


def mlp_struct(params: dict, bf16: bool = False):
    keep = {k: np.ascontiguousarray(np.asarray(params[k], np.float64).reshape(-1))
            for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mean", "std")}
    s = Mlp(*[_ptr(keep[k], _d) for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mean", "std")],
            int(bf16))
    return s, keep


def mlp_forward(params: dict, x, bf16: bool = False):
    s, keep = mlp_struct(params, bf16)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros((x.shape[0], 3))
    lib().ora_mlp_forward(C.byref(s), _ptr(x, _d), x.shape[0], _ptr(y, _d))
    return y


def mlp_loss_grad(params: dict, x, t, bf16: bool = False):
    s, keep = mlp_struct(params, bf16)
    x = np.ascontiguousarray(x, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = dict(w1=np.zeros(64 * 16), b1=np.zeros(64), w2=np.zeros(64 * 64), b2=np.zeros(64),
             w3=np.zeros(3 * 64), b3=np.zeros(3))
    loss = lib().ora_mlp_loss_grad(C.byref(s), _ptr(x, _d), _ptr(t, _d), x.shape[0],
                                   *[_ptr(g[k], _d) for k in ("w1", "b1", "w2", "b2", "w3", "b3")])
    g = {k: v.reshape(np.shape(params[k])) for k, v in g.items()}
    return loss, g


def adam_step(params, m, v, grad, step: int, lr: float, clip: float = 0.0, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1: bias-corrected first
    and second moments) applied after rescaling the whole gradient to global
    L2 norm at most `clip` (gradient-norm clipping, Pascanu et al. 2013;
    clip 0 disables it).  The clip and lr defaults the trainer uses are the
    paper's monolithic-policy setup (appendix B.2).  float64 in and out:
    returns (params, m, v, clipped gradient, norm before clipping)."""
    g = np.asarray(grad, np.float64)
    norm = float(np.sqrt(np.sum(g * g)))
    if clip > 0.0 and norm > clip:
        g = g * (clip / norm)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    p = np.asarray(params, np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v, g, norm
