"""CPU checks of the boundary: the library loads, exports every function
that include/rbsim.h declares, and rejects bad descriptors on the host
(no device calls)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from helpers import ROOT, S

HEADER = os.path.join(ROOT, "include", "rbsim.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sim_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sim_create", "sim_step", "sim_contacts", "sim_workspace_bytes", "sim_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2106_14405_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sim_[a-z_]+)", out))
    assert set(declared_functions()) <= exported


def test_python_names_match_header():
    from paper_2106_14405_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def _desc(batch, **kw):
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import DEFAULT_CONSTS
    keep = dict(off=np.ascontiguousarray(batch.body_offset, np.int32),
                shape=np.ascontiguousarray(batch.shape, np.uint8),
                motion=np.ascontiguousarray(batch.motion, np.uint8),
                param=np.ascontiguousarray(batch.param, np.float32).reshape(-1),
                mass=np.ascontiguousarray(batch.mass, np.float32),
                fr=np.ascontiguousarray(batch.friction, np.float32),
                re=np.ascontiguousarray(batch.restitution, np.float32),
                pose=np.ascontiguousarray(batch.pose, np.float32).reshape(-1),
                vel=np.ascontiguousarray(batch.vel, np.float32).reshape(-1),
                base=np.ascontiguousarray(batch.arm_base, np.float32).reshape(-1),
                th=np.ascontiguousarray(batch.arm_theta, np.float32).reshape(-1))
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    d = L.BatchDesc()
    d.abi_version = L.SIM_ABI_VERSION
    d.num_scenes = batch.n_scenes
    d.h_body_offset = P(keep["off"], C.c_int32)
    d.h_shape = P(keep["shape"], C.c_uint8)
    d.h_motion = P(keep["motion"], C.c_uint8)
    d.h_param = P(keep["param"], C.c_float)
    d.h_mass = P(keep["mass"], C.c_float)
    d.h_friction = P(keep["fr"], C.c_float)
    d.h_restitution = P(keep["re"], C.c_float)
    d.h_pose = P(keep["pose"], C.c_float)
    d.h_vel = P(keep["vel"], C.c_float)
    d.arm = int(batch.arm)
    d.h_arm_base = P(keep["base"], C.c_float)
    d.h_arm_theta = P(keep["th"], C.c_float)
    for i in range(7):
        d.link_len[i] = DEFAULT_CONSTS["link_len"][i]
    d.arm_radius = 0.05
    d.gravity[2] = -9.81
    d.margin, d.baumgarte, d.slop, d.rest_thresh = 0.02, 0.2, 0.005, 0.5
    d.ground_friction = 0.5
    d.max_pairs = 256
    d.max_contacts = 256
    d.threads = 128
    for k, v in kw.items():
        setattr(d, k, v)
    return d, keep


def test_workspace_bytes_and_validation():
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.batch_drop(2)
    d, keep = _desc(b)
    n = lib.sim_workspace_bytes(C.byref(d))
    assert n > 0 and n % 256 == 0
    # the workspace grows with the contact capacity
    d2, keep2 = _desc(b, max_contacts=512)
    assert lib.sim_workspace_bytes(C.byref(d2)) > n
    for bad in (dict(abi_version=99), dict(num_scenes=0), dict(max_contacts=0), dict(threads=96),
                dict(solver=5), dict(warm_start=7), dict(tolerance=-1.0), dict(max_pairs=0),
                dict(max_pairs=(1 << 20) + 1)):
        db, kb = _desc(b, **bad)
        assert lib.sim_workspace_bytes(C.byref(db)) == 0, bad
        h = C.c_void_p()
        rc = lib.sim_create(C.byref(db), None, 0, C.byref(h))
        assert rc < 0 and not h.value
        assert lib.sim_last_error()


def test_workspace_holds_narrowphase_staging():
    """The narrowphase stages up to 4 contacts (2 float4 each) per pair in a
    scene's solver-record block, so that block must grow with the pair
    capacity even when the contact capacity is small."""
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.batch_drop(3)
    S_ = b.n_scenes
    small, k1 = _desc(b, max_pairs=128, max_contacts=256)
    big, k2 = _desc(b, max_pairs=1024, max_contacts=256)
    grow = lib.sim_workspace_bytes(C.byref(big)) - lib.sim_workspace_bytes(C.byref(small))
    # record block per scene: max(5 * 256, 8 * pairs) float4 of 16 bytes
    assert grow >= S_ * (8 * 1024 - 5 * 256) * 16


def test_bad_bodies_rejected():
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.batch_drop(1)
    b.mass = b.mass.copy()
    b.mass[3] = 0.0
    d, keep = _desc(b)
    assert lib.sim_workspace_bytes(C.byref(d)) == 0
    assert b"mass" in lib.sim_last_error()
    b = S.batch_drop(1)
    b.param = b.param.copy()
    b.param[0, 0] = -1.0
    d, keep = _desc(b)
    assert lib.sim_workspace_bytes(C.byref(d)) == 0


def test_create_rejects_small_workspace_without_device_calls():
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.batch_drop(1)
    d, keep = _desc(b)
    h = C.c_void_p()
    assert lib.sim_create(C.byref(d), None, 16, C.byref(h)) == L.SIM_EWORKSPACE
    assert lib.sim_step(None, None, C.c_float(1 / 120), 10) == L.SIM_EINVAL


def test_arm_layout_validated():
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.batch_clutter(1)
    b.motion = b.motion.copy()
    b.motion[-1] = S.DYNAMIC
    b.mass = b.mass.copy()
    b.mass[-1] = 1.0
    d, keep = _desc(b)
    assert lib.sim_workspace_bytes(C.byref(d)) == 0
    assert b"kinematic" in lib.sim_last_error()


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    """The binding raises instead of falling back when the library is absent."""
    from paper_2106_14405_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L.load()


def _with_hulls(d, keep, b):
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    keep["hi"] = np.ascontiguousarray(b.hull_index, np.int32).reshape(-1).copy()
    keep["hv"] = np.ascontiguousarray(b.hull_vert, np.float32).reshape(-1).copy()
    keep["hf"] = np.ascontiguousarray(b.hull_face, np.int32).reshape(-1).copy()
    d.n_hulls = len(keep["hi"]) // 4
    d.h_hull_index = P(keep["hi"], C.c_int32)
    d.h_hull_vert = P(keep["hv"], C.c_float)
    d.h_hull_face = P(keep["hf"], C.c_int32)


def test_hull_library_validated():
    """The host's checks of a hull library (convexity, closed surface,
    principal frame about the centre of mass, index range, no learned
    start), without a GPU: sim_workspace_bytes validates first."""
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.pack([S.drop_scene(3, n_spheres=2, n_boxes=2, n_hulls=4)])
    d, keep = _desc(b)
    _with_hulls(d, keep, b)
    assert lib.sim_workspace_bytes(C.byref(d)) > 0, lib.sim_last_error()
    v0, nv, f0, nf = b.hull_index[0]
    cases = [("not convex", lambda: keep["hv"].__setitem__(slice(3 * v0, 3 * v0 + 3), 0.4 * keep["hv"][3 * v0:3 * v0 + 3])),
             ("centre of mass", lambda: keep["hv"].__setitem__(slice(3 * v0, 3 * (v0 + nv)), keep["hv"][3 * v0:3 * (v0 + nv)] + 0.01)),
             ("close the surface", lambda: keep["hf"].__setitem__(slice(8 * f0, 8 * f0 + 3), keep["hf"][8 * f0:8 * f0 + 3][::-1].copy())),
             ("index of a hull", lambda: keep["param"].__setitem__(3 * int(np.nonzero(b.shape == S.HULL)[0][0]), 99.0))]
    for why, spoil in cases:
        d, keep = _desc(b)
        keep["param"] = keep["param"].copy()
        d.h_param = keep["param"].ctypes.data_as(C.POINTER(C.c_float))
        _with_hulls(d, keep, b)
        spoil()
        assert lib.sim_workspace_bytes(C.byref(d)) == 0, why
        msg = lib.sim_last_error().decode()
        assert why in msg or (why == "not convex" and "centre of mass" in msg), (why, msg)
    d, keep = _desc(b, warm_start=L.LEARNED)
    _with_hulls(d, keep, b)
    assert lib.sim_workspace_bytes(C.byref(d)) == 0
    assert b"learned" in lib.sim_last_error()


def test_container_parts_validated():
    """The host's checks of container parts without a GPU: kinds, dynamic
    bodies only, unit axes, ordered limits, parent range, 16 a scene, PGS
    without the learned start."""
    from paper_2106_14405_amd import _lib as L
    lib = L.load()
    b = S.batch_clutter(1, seed0=10000, arm=True, cabinets=2)
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))

    def desc(spoil=None, **kw):
        d, keep = _desc(b, **kw)
        keep["j"] = np.ascontiguousarray(b.joint, np.uint8).copy()
        keep["ja"] = np.ascontiguousarray(b.joint_axis, np.float32).reshape(-1).copy()
        keep["jo"] = np.ascontiguousarray(b.joint_anchor, np.float32).reshape(-1).copy()
        keep["jl"] = np.ascontiguousarray(b.joint_limits, np.float32).reshape(-1).copy()
        keep["jp"] = np.ascontiguousarray(b.joint_parent, np.int32).copy()
        if spoil:
            spoil(keep)
        d.h_joint = P(keep["j"], C.c_uint8)
        d.h_joint_axis = P(keep["ja"], C.c_float)
        d.h_joint_anchor = P(keep["jo"], C.c_float)
        d.h_joint_limits = P(keep["jl"], C.c_float)
        d.h_joint_parent = P(keep["jp"], C.c_int32)
        return d, keep
    d, keep = desc()
    assert lib.sim_workspace_bytes(C.byref(d)) > 0, lib.sim_last_error()
    p0 = int(np.nonzero(b.joint)[0][0])
    dyn = [i for i in range(len(b.joint) - 7) if b.motion[i] == S.DYNAMIC and b.joint[i] == 0][:13]

    def many(k):
        k["j"][dyn] = 2
        for i in dyn:
            k["ja"][3 * i:3 * i + 3] = (1.0, 0.0, 0.0)
    cases = [("joint kind", lambda k: k["j"].__setitem__(p0, 3)),
             ("dynamic body", lambda k: k["j"].__setitem__(0, 1)),
             ("unit vector", lambda k: k["ja"].__setitem__(slice(3 * p0, 3 * p0 + 3), (1.0, 1.0, 0.0))),
             ("lower <= upper", lambda k: k["jl"].__setitem__(slice(2 * p0, 2 * p0 + 2), (0.5, -0.5))),
             ("parent", lambda k: k["jp"].__setitem__(p0, 9999)),
             ("16 container parts", many)]
    for why, spoil in cases:
        d, keep = desc(spoil)
        assert lib.sim_workspace_bytes(C.byref(d)) == 0, why
        assert why in lib.sim_last_error().decode(), (why, lib.sim_last_error())
    for kw in (dict(solver=L.JACOBI), dict(warm_start=L.LEARNED)):
        d, keep = desc(**kw)
        assert lib.sim_workspace_bytes(C.byref(d)) == 0
        assert b"container parts" in lib.sim_last_error()


def test_generated_hulls_pass_the_library_checks():
    """Every hull the scene generator draws (prisms, bipyramids, cut boxes of
    every size) is convex, closed and in its principal frame about its
    centre of mass, as the library requires."""
    lib = __import__("paper_2106_14405_amd._lib", fromlist=["load"]).load()
    b = S.pack([S.drop_scene(50 + k, n_spheres=1, n_boxes=1, n_hulls=25, size=(0.03, 0.3), edge=4.0)
                for k in range(8)])
    assert len(b.hull_index) == 200
    d, keep = _desc(b)
    _with_hulls(d, keep, b)
    assert lib.sim_workspace_bytes(C.byref(d)) > 0, lib.sim_last_error()
