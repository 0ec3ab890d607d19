"""Camera intrinsics and poses (inputs, not method arithmetic).

Axes follow the OpenCV convention: camera x right, y down, z forward.  A pose
is the 3x4 row-major camera-to-world matrix [R | eye] whose columns are the
camera's right, down and forward axes in world coordinates.  Poses are built
in float64 and handed to both sides as float32.
"""
from dataclasses import dataclass
import numpy as np


@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    f: float
    cx: float
    cy: float
    c2w: np.ndarray  # float32 [12], row-major 3x4

    def as_tuple(self):
        return (self.width, self.height, self.f, self.cx, self.cy, self.c2w)


def intrinsics(width, height, fov_deg=40.0):
    """Pinhole intrinsics with horizontal field of view fov_deg, principal
    point at the image centre; returns float32-rounded (f, cx, cy)."""
    f = (width / 2.0) / np.tan(np.deg2rad(fov_deg) / 2.0)
    return float(np.float32(f)), float(np.float32(width / 2.0)), float(np.float32(height / 2.0))


def look_at(eye, up=(0.0, 0.0, 1.0)):
    """float64 3x4 camera-to-world looking at the origin from `eye`."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = -eye / np.linalg.norm(eye)
    up = np.asarray(up, dtype=np.float64)
    if abs(np.dot(fwd, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    m = np.zeros((3, 4))
    m[:, 0] = right
    m[:, 1] = down
    m[:, 2] = fwd
    m[:, 3] = eye
    return m


def orbit_pose(k, radius=4.0, elev_deg=30.0, az0_deg=0.0, step_deg=1.0):
    """Pose k of an orbit about the world z axis at fixed elevation."""
    az = np.deg2rad(az0_deg + step_deg * k)
    el = np.deg2rad(elev_deg)
    eye = radius * np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
    return look_at(eye)


def orbit_poses(n, **kw):
    return [orbit_pose(k, **kw) for k in range(n)]


def sphere_poses(n=8, seed=2, radius=4.0):
    """n poses looking at the origin from directions drawn as normalised
    N(0, I3) vectors."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        out.append(look_at(radius * v))
    return out


def as_f32(pose):
    return np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(12).astype(np.float32))


def make_camera(width, height, pose, fov_deg=40.0):
    f, cx, cy = intrinsics(width, height, fov_deg)
    return Camera(width, height, f, cx, cy, as_f32(pose))


def relative_pose(c2w_ref, c2w_tgt):
    """T_ref->tgt = W2C_tgt * C2W_ref as a float32 row-major 3x4 [R | t].

    Computed in float64 from the float32 pose bits both sides received, then
    rounded once to float32, so every consumer sees identical bits."""
    a = np.asarray(c2w_ref, dtype=np.float64).reshape(3, 4)
    b = np.asarray(c2w_tgt, dtype=np.float64).reshape(3, 4)
    ra, ea = a[:, :3], a[:, 3]
    rb, eb = b[:, :3], b[:, 3]
    r = rb.T @ ra
    t = rb.T @ (ea - eb)
    m = np.concatenate([r, t[:, None]], axis=1)
    return np.ascontiguousarray(m.reshape(12).astype(np.float32))
