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
