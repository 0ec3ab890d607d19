"""Host-side parts of the reference schedule in the library (no GPU):
Eq. 5-6 pose extrapolation and Eq. 2's relative transform against the
oracle's independent float64 versions, and render_sequence's argument
checks."""
import ctypes as C
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import sequence as seq


@pytest.fixture(scope="module")
def L():
    from paper_2404_11852_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2404_11852_amd import build
        build.build()
    return _lib


def _f32(p):
    return np.asarray(p, np.float64).reshape(12).astype(np.float32)


def test_extrapolate_pose_matches_oracle(L):
    rng = np.random.default_rng(4)
    cases = [(synth.orbit_pose(k - 1), synth.orbit_pose(k)) for k in (1, 17, 200)]
    for _ in range(40):
        R0 = Rotation.random(random_state=rng)
        R1 = Rotation.from_rotvec(rng.normal(0, 0.2, 3)) * R0
        cases.append((np.concatenate([R0.as_matrix(), rng.normal(0, 3, (3, 1))], 1),
                      np.concatenate([R1.as_matrix(), rng.normal(0, 3, (3, 1))], 1)))
    # a half turn between the poses and a pose that does not move
    cases.append((np.concatenate([np.eye(3), np.zeros((3, 1))], 1),
                  np.concatenate([np.diag([1.0, -1.0, -1.0]), np.ones((3, 1))], 1)))
    cases.append((synth.orbit_pose(3), synth.orbit_pose(3)))
    for P, Q in cases:
        P32, Q32 = _f32(P), _f32(Q)
        for steps in (0.0, 0.5, 3.0, 8.0, 13.0, -1.0):
            got = np.array(L.extrapolate_pose(P32, Q32, steps), np.float64)
            ref = seq.extrapolate_pose(P32.reshape(3, 4), Q32.reshape(3, 4), steps, as_float32=False).reshape(12)
            assert np.allclose(got, ref, rtol=0, atol=2e-6 * max(1.0, abs(steps))), (steps, got - ref)


def test_relative_pose_matches_oracle(L):
    rng = np.random.default_rng(5)
    for k in range(30):
        A = _f32(synth.orbit_pose(k, step_deg=11.0))
        B = _f32(synth.look_at(rng.normal(0, 1, 3) * 3 + np.array([0, 0, 4.0])))
        got = np.array(L.relative_pose(A, B), np.float32)
        ref = seq.relative_pose(A, B)
        assert np.allclose(got, ref, rtol=0, atol=1e-6)


def test_pose_arguments_rejected(L):
    lib = L.lib()
    good = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    bad = (C.c_float * 12)(1, 0, 0, float("inf"), 0, 1, 0, 0, 0, 0, 1, 0)
    out = (C.c_float * 12)()
    assert lib.cic_extrapolate_pose(good, bad, C.c_float(1.0), out) == -1
    assert lib.cic_extrapolate_pose(good, good, C.c_float(float("nan")), out) == -1
    assert lib.cic_extrapolate_pose(None, good, C.c_float(1.0), out) == -1
    assert lib.cic_relative_pose(good, bad, out) == -1


def test_render_sequence_validation(L):
    lib = L.lib()
    g = L.Grid((C.c_int32 * 3)(32, 32, 32), 12, L.CIC_F32, (C.c_float * 3)(-1.5, -1.5, -1.5),
               (C.c_float * 3)(1.5, 1.5, 1.5), -6.9, 0x1000, 0x2000, None)
    m = L.MLP(L.CIC_F32, 39, 128, 4, 0x3000, 0x3100, 0x3200, 0x3300, 0x3400, 0x3500)
    o = L.make_opts(64)
    pose = [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 4]
    cams = (L.Camera * 3)(L.make_camera(32, 32, 40.0, 16.0, 16.0, pose), L.make_camera(32, 32, 40.0, 16.0, 16.0, pose),
                          L.make_camera(32, 24, 40.0, 16.0, 12.0, pose))
    p = C.c_void_p(0x5000)
    big = C.c_size_t(1 << 40)

    def call(n=2, window=4, lead=-1.0, flags=1, cams_=cams, ws_bytes=big, part=0, stream=None,
             ref=C.c_void_p(0x7000)):
        return lib.render_sequence(C.byref(g), C.byref(m), C.byref(o), cams_, C.c_int32(n), C.c_int32(window),
                                   C.c_float(lead), C.c_int32(flags), C.c_int32(part), p, p, p, None, None, None, p,
                                   ws_bytes, stream, ref)

    assert call(n=0) == 0
    assert call(window=0) == -1 and "window" in L.last_error()
    assert call(lead=float("nan")) == -1
    assert call(flags=4) == -1 and "flags" in L.last_error()
    assert call(n=3) == -1 and "size" in L.last_error()
    assert call(cams_=None) == -1
    assert call(ws_bytes=C.c_size_t(64)) == -2
    assert call(n=-1) == -1
    assert call(part=4, flags=0) == -1 and "target_cus_per_xcd" in L.last_error()
    assert call(part=-1) == -1
    # the overlapped schedule needs a caller-owned reference stream distinct from the target stream
    assert call(ref=None) == -1 and "reference stream" in L.last_error()
    assert call(stream=C.c_void_p(0x7000)) == -1 and "reference stream" in L.last_error()
    per_frame = L.workspace_bytes(L.OP_RENDER_SEQUENCE, 1024, g, o)
    assert per_frame > 2 * L.workspace_bytes(L.OP_RENDER_FRAME, 1024, g, o)


def test_cu_masked_stream_validation(L):
    """cic_stream_create_cu_masked rejects bad arguments before touching the
    runtime, and destroying a NULL stream is a no-op."""
    lib = L.lib()
    h = C.c_void_p(0x1234)
    assert lib.cic_stream_create_cu_masked(C.c_int32(8), C.c_int32(2), C.byref(h)) == -1
    assert h.value is None and "role" in L.last_error()
    assert lib.cic_stream_create_cu_masked(C.c_int32(8), C.c_int32(0), None) == -1
    assert lib.cic_stream_destroy(None) == 0
