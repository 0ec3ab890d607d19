"""Pins of the oracle's reference-frame schedule (Sec. III-C, Eq. 5-6):
pose extrapolation against closed forms and an independent rotation library,
the relative transform of Eq. 2 against a second formula, and the schedule
on a camera that does not move."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import sequence as seq


def _pose(R, c):
    return np.concatenate([np.asarray(R, np.float64), np.asarray(c, np.float64)[:, None]], axis=1)


def test_zero_and_minus_one_steps():
    rng = np.random.default_rng(0)
    for _ in range(20):
        R0 = Rotation.random(random_state=rng).as_matrix()
        R1 = Rotation.from_rotvec(rng.normal(0, 0.05, 3)).as_matrix() @ R0
        c0, c1 = rng.normal(0, 2, 3), rng.normal(0, 2, 3)
        P, Q = _pose(R0, c0), _pose(R1, c1)
        assert np.allclose(seq.extrapolate_pose(P, Q, 0.0, as_float32=False), Q, atol=1e-12)
        assert np.allclose(seq.extrapolate_pose(P, Q, -1.0, as_float32=False), P, atol=1e-12)


def test_translation_is_a_straight_line():
    rng = np.random.default_rng(1)
    R = Rotation.random(random_state=rng).as_matrix()
    c0 = np.array([0.3, -1.0, 2.0])
    step = np.array([0.05, 0.02, -0.01])
    P, Q = _pose(R, c0), _pose(R, c0 + step)
    for s in (0.5, 3.0, 8.0):
        out = seq.extrapolate_pose(P, Q, s, as_float32=False)
        assert np.allclose(out[:, :3], R, atol=1e-12)
        assert np.allclose(out[:, 3], c0 + (1.0 + s) * step, atol=1e-12)


def test_constant_angular_velocity_matches_rotation_library():
    """Orientation R_k = exp(k w) R_0: extrapolating from k = 0, 1 by s steps
    gives exp((1 + s) w) R_0 (scipy's rotation vectors)."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        R0 = Rotation.random(random_state=rng)
        w = rng.normal(0, 0.1, 3)
        R1 = Rotation.from_rotvec(w) * R0
        s = float(rng.uniform(0.5, 12.0))
        out = seq.extrapolate_pose(_pose(R0.as_matrix(), np.zeros(3)), _pose(R1.as_matrix(), np.zeros(3)), s,
                                   as_float32=False)
        expect = (Rotation.from_rotvec((1.0 + s) * w) * R0).as_matrix()
        assert np.allclose(out[:, :3], expect, atol=1e-12)
        assert np.allclose(out[:, :3] @ out[:, :3].T, np.eye(3), atol=1e-12)


def test_orbit_orientation_and_chord():
    """On the orbit about z (1 degree per frame) the extrapolated orientation
    is the orbit's own orientation `s` frames ahead, while the centre runs
    along the chord, off the circle (the reference is off the trajectory)."""
    a = 10
    P, Q = synth.orbit_pose(a - 1), synth.orbit_pose(a)
    for s in (2.0, 8.0, 13.0):
        out = seq.extrapolate_pose(P, Q, s, as_float32=False)
        assert np.allclose(out[:, :3], synth.orbit_pose(a + s)[:, :3], atol=1e-12)
        assert np.allclose(out[:, 3], Q[:, 3] + s * (Q[:, 3] - P[:, 3]), atol=1e-12)
        assert np.linalg.norm(out[:, 3]) > 4.0 + 1e-6
    # the default lead of half a window puts the reference near the window's middle frame
    out = seq.extrapolate_pose(P, Q, 8.0, as_float32=False)
    assert np.linalg.norm(out[:, 3] - synth.orbit_pose(a + 8)[:, 3]) < 0.05


def test_relative_pose_two_formulas():
    rng = np.random.default_rng(3)
    for k in range(10):
        A = synth.as_f32(synth.orbit_pose(k, step_deg=7.0))
        B = synth.as_f32(synth.look_at(rng.normal(0, 1, 3) * 3 + np.array([0, 0, 4.0])))
        T = seq.relative_pose(A, B)
        assert np.allclose(T, synth.relative_pose(A, B), rtol=0, atol=1e-6)
        # a world point seen from camera A, moved by T, is the same point seen from camera B
        X = rng.normal(0, 1, 3)
        Am, Bm = A.reshape(3, 4).astype(np.float64), B.reshape(3, 4).astype(np.float64)
        xa = Am[:, :3].T @ (X - Am[:, 3])
        xb = Bm[:, :3].T @ (X - Bm[:, 3])
        Tm = T.reshape(3, 4).astype(np.float64)
        assert np.allclose(Tm[:, :3] @ xa + Tm[:, 3], xb, atol=1e-5)
    I = seq.relative_pose(synth.as_f32(synth.orbit_pose(3)), synth.as_f32(synth.orbit_pose(3)))
    assert np.allclose(I.reshape(3, 4), np.eye(3, 4), atol=1e-6)


def test_schedule_indices():
    assert seq.window_starts(1, 4) == []
    assert seq.window_starts(2, 4) == [1]
    assert seq.window_starts(10, 4) == [1, 5, 9]
    poses = [synth.as_f32(synth.orbit_pose(k)).reshape(3, 4) for k in range(10)]
    refs = seq.reference_poses(poses, 4)
    assert len(refs) == 2
    assert np.array_equal(refs[0], seq.extrapolate_pose(poses[0], poses[1], 2.0))
    assert np.array_equal(refs[1], seq.extrapolate_pose(poses[4], poses[5], 2.0))
    assert np.array_equal(seq.reference_poses(poses, 4, lead=6.0)[1], seq.extrapolate_pose(poses[4], poses[5], 6.0))


@pytest.fixture(scope="module")
def small_model():
    density, features = synth.make_scene(32, seed=0)
    return oracle.Model(density, features, synth.make_mlp(seed=1), density_shift=float(synth.DENSITY_SHIFT))


def test_static_camera_sequence_repeats_frame_zero(small_model):
    """A camera that does not move: every reference is frame 0's pose, every
    target is an identity warp of frame 0 with no holes."""
    W = H = 24
    f = synth.intrinsics(W, H)[0]
    pose = synth.as_f32(synth.orbit_pose(0)).reshape(3, 4)
    op = oracle.opts(64, 1e-4)
    frames, refs = seq.render_sequence(small_model, op, W, H, f, W / 2, H / 2, [pose] * 8, window=3)
    assert len(refs) == 2 and all(np.allclose(r, pose, rtol=0, atol=1e-7) for r in refs)
    rgb0, dz0 = frames[0][0], frames[0][1]
    for k in range(1, 8):
        rgb, dz, mask, nm = frames[k]
        assert nm == 0 and mask.sum() == 0
        assert np.array_equal(rgb, rgb0.astype(np.float32).astype(np.float64))
        assert np.array_equal(dz, dz0.astype(np.float32).astype(np.float64))


def test_upsample_matches_torch_and_affine():
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(6)
    for (w, h, s) in ((5, 4, 2), (8, 8, 2), (7, 3, 3)):
        img = rng.uniform(0, 1, (h * w, 3))
        W, H = w * s, h * s
        got = seq.upsample_bilinear(img, w, h, W, H, s)
        t = torch.from_numpy(img.reshape(h, w, 3).transpose(2, 0, 1)[None].copy())
        ref = F.interpolate(t, size=(H, W), mode="bilinear", align_corners=False)[0].numpy()
        assert np.allclose(got.reshape(H, W, 3), ref.transpose(1, 2, 0), atol=1e-12)
    # an affine image is reproduced exactly away from the clamped border
    w, h, s = 9, 7, 2
    jj, ii = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    img = (0.3 + 0.1 * ii - 0.05 * jj).reshape(-1, 1)
    up = seq.upsample_bilinear(img, w, h, w * s, h * s, s).reshape(h * s, w * s)
    J, I = np.meshgrid(np.arange(h * s), np.arange(w * s), indexing="ij")
    x, y = (I + 0.5) / s - 0.5, (J + 0.5) / s - 0.5
    inner = (x >= 0) & (x <= w - 1) & (y >= 0) & (y <= h - 1)
    assert np.allclose(up[inner], (0.3 + 0.1 * x - 0.05 * y)[inner], atol=1e-12)
    # factor 1 is the identity
    assert np.array_equal(seq.upsample_bilinear(img, w, h, w, h, 1), img)


def test_low_res_camera_covers_the_same_view():
    """The low-resolution pixel centre k + 1/2 and the full-resolution pixel
    centres it covers see the same ray direction on average: pixel (k) of the
    small camera looks where pixels (s k .. s k + s - 1) look."""
    W, H = 64, 48
    f, cx, cy = synth.intrinsics(W, H)
    w, h, fl, cxl, cyl = seq.low_res_camera(W, H, f, cx, cy, 2)
    assert (w, h) == (32, 24)
    k = np.arange(w)
    a_low = (k + 0.5 - cxl) / fl
    a_full = ((2 * k + 0.5 - cx) / f + (2 * k + 1.5 - cx) / f) / 2
    assert np.allclose(a_low, a_full, atol=1e-6)
    assert seq.low_res_camera(65, 49, f, cx, cy, 2)[:2] == (33, 25)


def test_temporal_static_camera(small_model):
    """Temp-N with a camera that does not move: every frame repeats the last
    full render and nothing is re-rendered between full renders."""
    W = H = 24
    f = synth.intrinsics(W, H)[0]
    pose = synth.as_f32(synth.orbit_pose(0)).reshape(3, 4)
    op = oracle.opts(64, 1e-4)
    frames = seq.render_temporal(small_model, op, W, H, f, W / 2, H / 2, [pose] * 7, window=3)
    for k in range(7):
        rgb, dz, mask, nm = frames[k]
        if k % 3 == 0:
            assert nm == W * H
        else:
            assert nm == 0
            assert np.array_equal(rgb, frames[k - 1][0].astype(np.float32).astype(np.float64))


def test_temporal_window_one_is_full_rendering(small_model):
    W = H = 16
    f = synth.intrinsics(W, H)[0]
    poses = [synth.as_f32(synth.orbit_pose(k, step_deg=5.0)).reshape(3, 4) for k in range(3)]
    op = oracle.opts(64, 1e-4)
    frames = seq.render_temporal(small_model, op, W, H, f, W / 2, H / 2, poses, window=1)
    for k in range(3):
        rgb, _, _, _ = oracle.render_pixels(small_model, op, oracle.camera(W, H, f, W / 2, H / 2, poses[k].reshape(12)))
        assert np.array_equal(frames[k][0], rgb)
