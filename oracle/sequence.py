"""Oracle for the reference-frame schedule of Sec. III-C: references placed
off the trajectory by extrapolating the camera motion (Eq. 5-6), targets
warped from the latest reference and their holes rendered (Sec. III-B, Eq. 4).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: used by the tests, never
by the product package.  Plain float64 numpy; the rendering and warping are
the oracle's own C routines.

Readings the paper leaves open:
* Eq. 5-6 treat the pose as a vector.  The camera centre is extrapolated
  linearly; the orientation is extrapolated at constant angular velocity,
  i.e. the world-frame rotation that takes the older orientation to the newer
  one is applied `steps` more times (fractional powers by spherical
  interpolation of unit quaternions).  steps = t_r / dt.
* Schedule: frame 0 is rendered in full and is the first reference.  The
  other frames form windows of N consecutive targets, window w starting at
  frame s_w = 1 + w N.  Window w is warped from reference w.  Reference w + 1
  is extrapolated from the two newest poses known when window w starts,
  frames s_w - 1 and s_w, with t_r = N/2 dt by default, so that it can render
  while window w is being warped.
"""
import numpy as np

from . import camera, render_pixels, sparw


# ---------------------------------------------------------------------------
# unit quaternions (w, x, y, z)
# ---------------------------------------------------------------------------
def _quat_from_matrix(R):
    """Rotation matrix -> unit quaternion (largest-pivot branch for accuracy)."""
    R = np.asarray(R, dtype=np.float64)
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    if tr > 0.0:
        s = 2.0 * np.sqrt(tr + 1.0)
        q = np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s])
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        q = np.array([(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s])
    elif R[1, 1] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2])
        q = np.array([(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s])
    else:
        s = 2.0 * np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1])
        q = np.array([(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s])
    return q / np.linalg.norm(q)


def _quat_mul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _quat_conj(q):
    return np.array([q[0], -q[1], -q[2], -q[3]])


def _quat_pow(q, s):
    """q^s for a unit quaternion on the short arc (w >= 0)."""
    if q[0] < 0.0:
        q = -q
    v = np.linalg.norm(q[1:])
    if v == 0.0:
        return np.array([1.0, 0.0, 0.0, 0.0])
    half = np.arctan2(v, q[0])
    axis = q[1:] / v
    return np.concatenate([[np.cos(s * half)], np.sin(s * half) * axis])


def _matrix_from_quat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def extrapolate_pose(c2w_prev, c2w_cur, steps, as_float32=True):
    """Eq. 5-6: v = (T2 - T1)/dt, R = T2 + v t_r with t_r = steps * dt, for
    camera-to-world poses [R | c] (row-major 3x4).  Returns the 3x4 pose,
    rounded once to float32 unless as_float32 is False."""
    P = np.asarray(c2w_prev, dtype=np.float64).reshape(3, 4)
    Q = np.asarray(c2w_cur, dtype=np.float64).reshape(3, 4)
    c = Q[:, 3] + steps * (Q[:, 3] - P[:, 3])
    q_prev, q_cur = _quat_from_matrix(P[:, :3]), _quat_from_matrix(Q[:, :3])
    q_step = _quat_mul(q_cur, _quat_conj(q_prev))          # world-frame rotation prev -> cur
    R = _matrix_from_quat(_quat_mul(_quat_pow(q_step, steps), q_cur))
    out = np.concatenate([R, c[:, None]], axis=1)
    return out.astype(np.float32) if as_float32 else out


def relative_pose(c2w_ref, c2w_tgt):
    """Eq. 2's rigid transform from reference-camera to target-camera
    coordinates, T = inverse(C2W_tgt) C2W_ref, in float64 from the float32
    poses, rounded once to float32 (row-major 3x4)."""
    A = np.eye(4)
    A[:3, :] = np.asarray(c2w_ref, dtype=np.float64).reshape(3, 4)
    B = np.eye(4)
    B[:3, :] = np.asarray(c2w_tgt, dtype=np.float64).reshape(3, 4)
    T = np.linalg.inv(B) @ A
    return np.ascontiguousarray(T[:3, :].reshape(12).astype(np.float32))


def window_starts(n_frames, window):
    return list(range(1, n_frames, window))


def reference_poses(c2ws, window, lead=None):
    """Poses of references 1, 2, ... (reference 0 is frame 0) for a trajectory
    of camera-to-world poses."""
    lead = window / 2.0 if lead is None or lead < 0 else float(lead)
    starts = window_starts(len(c2ws), window)
    return [extrapolate_pose(c2ws[s - 1], c2ws[s], lead) for s in starts[:-1]]


def render_sequence(model, op, width, height, f, cx, cy, c2ws, window, lead=None):
    """Render a trajectory (list of float32 3x4 camera-to-world poses) under
    the schedule above.  Returns per-frame (rgb float64 [P,3], z-depth
    float64 [P], mask uint8 [P], n_masked) and the reference poses."""
    cams = [camera(width, height, f, cx, cy, np.asarray(p, np.float32).reshape(12)) for p in c2ws]
    n_frames = len(cams)
    out = [None] * n_frames
    rgb0, dz0, _, _ = render_pixels(model, op, cams[0])
    out[0] = (rgb0, dz0, np.ones(width * height, np.uint8), width * height)   # every pixel rendered
    ref = (np.asarray(c2ws[0], np.float32).reshape(12), rgb0.astype(np.float32), dz0.astype(np.float32))
    poses = reference_poses(c2ws, window, lead)
    for w, s in enumerate(window_starts(n_frames, window)):
        if w > 0:
            pose = poses[w - 1].reshape(12)
            rr, rd, _, _ = render_pixels(model, op, camera(width, height, f, cx, cy, pose))
            ref = (pose, rr.astype(np.float32), rd.astype(np.float32))
        ref_cam = camera(width, height, f, cx, cy, ref[0])
        for k in range(s, min(s + window, n_frames)):
            T = relative_pose(ref[0], c2ws[k])
            out[k] = sparw(model, op, ref_cam, ref[1], ref[2], cams[k], T)
    return out, poses


# ---------------------------------------------------------------------------
# comparison variants of the paper's evaluation
# ---------------------------------------------------------------------------
def low_res_camera(width, height, f, cx, cy, factor):
    """Camera of the same pose whose pixels are `factor` times larger:
    ceil(W/s) x ceil(H/s) pixels, f/s, principal point /s (float32)."""
    s = np.float32(factor)
    return ((width + factor - 1) // factor, (height + factor - 1) // factor,
            float(np.float32(f) / s), float(np.float32(cx) / s), float(np.float32(cy) / s))


def upsample_bilinear(img, w, h, width, height, factor):
    """Bilinear upsampling of a [h*w, C] image to [height*width, C]: output
    pixel centre i + 1/2 sits at (i + 1/2)/s - 1/2 in low-resolution pixel
    index space; neighbours outside the image are clamped to the border."""
    img = np.asarray(img, np.float64).reshape(h, w, -1)
    x = (np.arange(width) + 0.5) / factor - 0.5
    y = (np.arange(height) + 0.5) / factor - 0.5
    x0, y0 = np.floor(x).astype(int), np.floor(y).astype(int)
    fx, fy = x - x0, y - y0
    xa, xb = np.clip(x0, 0, w - 1), np.clip(x0 + 1, 0, w - 1)
    ya, yb = np.clip(y0, 0, h - 1), np.clip(y0 + 1, 0, h - 1)
    top = img[ya][:, xa] * (1 - fx)[None, :, None] + img[ya][:, xb] * fx[None, :, None]
    bot = img[yb][:, xa] * (1 - fx)[None, :, None] + img[yb][:, xb] * fx[None, :, None]
    out = top * (1 - fy)[:, None, None] + bot * fy[:, None, None]
    return out.reshape(height * width, -1)


def render_downsampled(model, op, width, height, f, cx, cy, c2w, factor=2):
    """DS-s variant: render at 1/s resolution, upsample bilinearly (rgb)."""
    w, h, fl, cxl, cyl = low_res_camera(width, height, f, cx, cy, factor)
    rgb, _, _, diag = render_pixels(model, op, camera(w, h, fl, cxl, cyl, np.asarray(c2w, np.float32).reshape(12)))
    return upsample_bilinear(rgb, w, h, width, height, factor), rgb, diag


def render_temporal(model, op, width, height, f, cx, cy, c2ws, window):
    """Temp-N variant: frames 0, N, 2N, ... are rendered in full; every other
    frame is warped from the previous output frame (its colour and z-depth,
    as float32) with the holes rendered, so warping errors carry forward."""
    cams = [camera(width, height, f, cx, cy, np.asarray(p, np.float32).reshape(12)) for p in c2ws]
    out = []
    for k, cam in enumerate(cams):
        if k % window == 0:
            rgb, dz, _, _ = render_pixels(model, op, cam)
            out.append((rgb, dz, np.ones(width * height, np.uint8), width * height))
        else:
            prgb, pdz = out[k - 1][0].astype(np.float32), out[k - 1][1].astype(np.float32)
            T = relative_pose(c2ws[k - 1], c2ws[k])
            out.append(sparw(model, op, cams[k - 1], prgb, pdz, cam, T))
    return out
