"""Pins for the oracle's depth outputs and their adjoint, independent of the
oracle's own formulas.

* Frame z-depth (the depth that Eq. 1 back-projects, Sec. III-B): a camera
  looking straight down at the box's top face sees a fronto-parallel opaque
  surface at camera depth h - 1.5 in every pixel.  The expected z-depth is
  fixed by plane geometry (entry distance (h - 1.5)/cos, exit distance
  (h + 1.5)/cos along a ray at angle theta to the optical axis, with cos
  taken from the pixel's camera-space direction (a, b, 1)) and the geometric
  series of the constant-density quadrature.
* Expected distance and opacity gradients: central finite differences of a
  loss on depth_t and on acc over every density vertex of a small model, and
  the closed-form derivative of the constant box's expected distance.
* Ray/box interval: entry and exit points lie on the box faces; rays that
  miss never pass through the box.
"""
import math

import numpy as np
import pytest

import synth

H_CAM = 4.0


def _down_camera(W, H, eye_xy=(0.0, 0.0)):
    """c2w of a camera at height H_CAM looking along -z (OpenCV axes: x right,
    y down, z forward): columns r = (1, 0, 0), d = (0, -1, 0), f = (0, 0, -1)."""
    c2w = np.array([[1.0, 0.0, 0.0, eye_xy[0]],
                    [0.0, -1.0, 0.0, eye_xy[1]],
                    [0.0, 0.0, -1.0, H_CAM]], np.float32)
    f, cx, cy = synth.intrinsics(W, H)
    return f, cx, cy, c2w


def _const_model(orc, raw, shift, R=6, nf=12, beta=0.4):
    dens = np.full((R, R, R), raw, np.float32)
    feats = np.random.default_rng(5).standard_normal((R, R, R, nf)).astype(np.float32)
    mlp = synth.make_mlp(6, in_dim=nf + 27)
    mlp["w2"][:] = 0.0
    mlp["b2"][:] = np.float32(beta)
    return orc.Model(dens, feats, mlp, density_shift=shift)


def _plane_geometry(W, H, f, cx, cy, eye_xy):
    """Per pixel: cos(theta) to the optical axis and whether the ray enters
    through the top face z = 1.5 and leaves through the bottom face z = -1.5
    (well inside the side faces)."""
    j, i = np.mgrid[0:H, 0:W]
    a = (i + 0.5 - cx) / f
    b = (j + 0.5 - cy) / f
    cos = 1.0 / np.sqrt(a * a + b * b + 1.0)
    # world x, y of the ray at the two faces (camera y axis is world -y)
    top = np.stack([eye_xy[0] + a * (H_CAM - 1.5), eye_xy[1] - b * (H_CAM - 1.5)], -1)
    bot = np.stack([eye_xy[0] + a * (H_CAM + 1.5), eye_xy[1] - b * (H_CAM + 1.5)], -1)
    inside = (np.abs(top) < 1.49).all(-1) & (np.abs(bot) < 1.49).all(-1)
    return cos.ravel(), inside.ravel()


@pytest.mark.parametrize("n_samples,raw", [(64, 0.5), (256, 3.0), (32, 200.0)])
def test_frame_depth_fronto_parallel_box(orc, n_samples, raw):
    """Constant density sigma inside the box, camera looking down -z from
    height h: a ray at angle theta enters at t_n = (h - 1.5)/cos theta, crosses
    L = 3/cos theta, and its expected distance over its opacity is t_n + delta
    (1/2 + S) with delta = L/N, q = exp(-sigma delta) and S = sum_k k q^k /
    sum_k q^k (k < N).  The z-depth of that point is cos theta times it: for
    large sigma every pixel sees the top face at camera depth h - 1.5."""
    W = H = 40
    eye = (0.2, -0.1)
    f, cx, cy, c2w = _down_camera(W, H, eye)
    shift = -0.3
    m = _const_model(orc, raw, shift)
    cam = orc.camera(W, H, f, cx, cy, c2w)
    op = orc.opts(n_samples)
    rgb, dz, acc, _ = orc.render_pixels(m, op, cam)
    cos, inside = _plane_geometry(W, H, f, cx, cy, eye)
    assert inside.sum() > 600 and (~inside).sum() > 50
    sigma = math.log1p(math.exp(float(np.float32(raw)) + float(np.float32(shift))))
    N = n_samples
    k = np.arange(N, dtype=np.float64)
    want = np.empty(W * H)
    for p in np.nonzero(inside)[0]:
        tn = (H_CAM - 1.5) / cos[p]
        delta = 3.0 / cos[p] / N
        qk = np.exp(-sigma * delta * k)
        S = float(np.sum(k * qk) / np.sum(qk))
        want[p] = cos[p] * (tn + delta * (0.5 + S))
    # sample positions are float32 (relative ulp ~6e-8 at t ~ 4)
    np.testing.assert_allclose(dz[inside], want[inside], rtol=0, atol=2e-5)
    if raw >= 100.0:
        # opaque: the top face at camera depth h - 1.5, to within half a step
        assert np.all(np.abs(dz[inside] - (H_CAM - 1.5)) <= 0.5 * 3.0 / N + 1e-5)
        # the corner pixels are ~10 degrees off axis: distance along the ray
        # differs from the z-depth there by far more than the tolerance
        assert np.max(1.0 / cos[inside] - 1.0) * (H_CAM - 1.5) > 0.02


def test_frame_depth_void_rule(orc):
    """Pixels whose rays miss the box, and rays whose opacity stays below the
    void threshold, have infinite z-depth; opaque ones are finite."""
    W = H = 24
    f, cx, cy, c2w = _down_camera(W, H)
    cam = orc.camera(W, H, f, cx, cy, c2w)
    # very thin density: acc ~ 3e-5 < 1e-4 everywhere
    m = _const_model(orc, -12.0, 0.0)
    _, dz, acc, _ = orc.render_pixels(m, orc.opts(32), cam)
    assert np.all(acc < 1e-4) and np.all(np.isinf(dz))
    # the camera sees the whole box from above: pixels outside its footprint miss
    m = _const_model(orc, 4.0, 0.0)
    c2w_far = c2w.copy()
    c2w_far[2, 3] = 12.0
    cam = orc.camera(W, H, f, cx, cy, c2w_far)
    _, dz, acc, _ = orc.render_pixels(m, orc.opts(32), cam)
    o, d = orc.generate_rays(cam)
    miss = ~orc.ray_box(o, d)[2]
    assert miss.sum() > 20 and (~miss).sum() > 20
    assert np.all(np.isinf(dz[miss])) and np.all(acc[miss] == 0.0)
    assert np.all(np.isfinite(dz[~miss]))


def test_ray_box_interval_on_faces(orc):
    """Entry and exit points o + t d lie on faces of the box, with the other
    two coordinates inside it; points between them are inside; rays that miss
    never pass through the box.  Rays start outside, inside and on an axis."""
    rng = np.random.default_rng(70)
    n = 4000
    o = rng.uniform(-4.0, 4.0, (n, 3)).astype(np.float32)
    o[:300] = rng.uniform(-1.4, 1.4, (300, 3))             # starting inside
    d = rng.standard_normal((n, 3))
    d[300:400, 1:] = 0.0                                    # axis-aligned directions
    d[400:500, 0] = 0.0
    aim = rng.uniform(-2.0, 2.0, (2000, 3))                 # aimed near the box
    d[500:2500] = aim - o[500:2500]
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    tn, tf, hit = orc.ray_box(o, d)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    tol = 2e-5 * (1.0 + np.abs(tf.astype(np.float64)))
    for r in np.nonzero(hit)[0]:
        p_in = o64[r] + float(tn[r]) * d64[r]
        p_out = o64[r] + float(tf[r]) * d64[r]
        assert np.all(np.abs(p_out) <= 1.5 + tol[r])
        assert abs(np.max(np.abs(p_out)) - 1.5) <= tol[r]
        assert np.all(np.abs(p_in) <= 1.5 + tol[r])
        if tn[r] > 0.0:
            # entered from outside: on a face
            assert abs(np.max(np.abs(p_in)) - 1.5) <= tol[r]
        else:
            # starts inside the box
            assert np.all(np.abs(o64[r]) <= 1.5)
        mid = o64[r] + 0.5 * (float(tn[r]) + float(tf[r])) * d64[r]
        assert np.all(np.abs(mid) <= 1.5 + tol[r])
    miss = ~hit
    assert miss.sum() > 500 and hit.sum() > 1500
    assert not np.any(_passes_inside(o[miss], d[miss]))


def _passes_inside(o, d, margin=1e-3):
    """Brute force: does some point o + t d (t >= 0, steps of 2e-3) lie inside
    the box shrunk by a rounding margin?"""
    t = np.arange(0.0, 16.0, 2e-3)
    out = np.zeros(o.shape[0], bool)
    for s in range(0, o.shape[0], 64):
        pts = o[s:s + 64, None, :].astype(np.float64) + t[None, :, None] * d[s:s + 64, None, :].astype(np.float64)
        out[s:s + 64] = (np.abs(pts) <= 1.5 - margin).all(-1).any(-1)
    return out


def _small_model(orc, seed=30, R=8, n_feat=4):
    rng = np.random.default_rng(seed)
    dens = rng.normal(0.0, 1.0, (R, R, R)).astype(np.float32) + 1.0
    feats = rng.normal(0.0, 1.0, (R, R, R, n_feat)).astype(np.float32)
    mlp = synth.make_mlp(seed + 1, in_dim=n_feat + 27, hidden=32, bias_std=0.1)
    m = orc.Model(dens, feats, mlp, density_shift=-2.0)
    f, cx, cy = synth.intrinsics(64, 64)
    cam = orc.camera(64, 64, f, cx, cy, synth.as_f32(synth.orbit_pose(10)))
    pix = synth.pixel_subset(64, 64, 16, seed=seed + 2)
    o, d = orc.generate_rays(cam, pix)
    return m, o, d


@pytest.mark.parametrize("which", ["depth", "acc", "both"])
def test_depth_and_opacity_gradients_finite_differences(orc, which):
    """Loss L = sum_r a_r (E_t,r - e_r)^2 + b_r (acc_r - s_r)^2 with no colour
    term: the adjoint's density gradient matches central differences (eps
    1e-3, float64 forward) on every vertex, and the feature and MLP
    gradients are zero (neither E_t nor acc depends on them)."""
    m, o, d = _small_model(orc)
    op = orc.opts(64)
    rng = np.random.default_rng(33)
    n = o.shape[0]
    a = rng.uniform(0.5, 1.5, n) if which in ("depth", "both") else np.zeros(n)
    b = rng.uniform(0.5, 1.5, n) * 4.0 if which in ("acc", "both") else np.zeros(n)
    _, dep0, acc0 = orc.render_rays(m, op, o, d)
    e_t = dep0 + rng.normal(0, 0.5, n)
    s_t = np.clip(acc0 + rng.normal(0, 0.2, n), 0, 1)

    def loss():
        _, dep, acc = orc.render_rays(m, op, o, d)
        return float(np.sum(a * (dep - e_t) ** 2 + b * (acc - s_t) ** 2))

    g, (_, dep, acc) = orc.render_backward(m, op, o, d, np.zeros((n, 3)),
                                           d_depth_t=2 * a * (dep0 - e_t), d_acc=2 * b * (acc0 - s_t))
    np.testing.assert_array_equal(dep, dep0)
    assert np.all(g["features"] == 0.0)
    for k in ("w0", "b0", "w1", "b1", "w2", "b2"):
        assert np.all(g[k] == 0.0), k
    eps = 1e-3
    dens = m.density
    scale = np.abs(g["density"]).max()
    assert scale > 1e-3
    bad = []
    touched = 0
    for idx in np.ndindex(dens.shape):
        old = dens[idx]
        up = float(np.float32(old + eps) - old)
        dn = float(old - np.float32(old - eps))
        dens[idx] = old + np.float32(up)
        lp = loss()
        dens[idx] = old - np.float32(dn)
        lm = loss()
        dens[idx] = old
        gf = (lp - lm) / (up + dn)
        ga = g["density"][idx]
        touched += ga != 0.0
        if abs(gf - ga) > 2e-7 * scale + 1e-5 * abs(ga):
            bad.append((idx, gf, ga))
    assert touched > 40
    assert not bad, bad[:10]


@pytest.mark.parametrize("n_samples", [16, 64])
def test_constant_box_expected_distance_derivative(orc, n_samples):
    """Constant raw density r on every vertex: the density gradient summed
    over vertices is dL/dr.  With d_depth_t = 1 that is dE_t/dsigma times
    sigmoid(r + b), where E_t(sigma) = delta sum_k (k + 1/2) q^k (1 - q) +
    t_n (1 - q^N), q = exp(-sigma delta), is the constant-density quadrature;
    its sigma-derivative is taken by central differences of that closed form
    in float64."""
    R, nf = 6, 12
    raw, shift = 0.8, -0.5
    m = _const_model(orc, raw, shift, R=R, nf=nf)
    o, d = synth.random_rays(64, seed=44)
    op = orc.opts(n_samples)
    tn, tf, hit = orc.ray_box(o, d)
    r = float(np.float32(raw)) + float(np.float32(shift))
    sigma = math.log1p(math.exp(r))
    sgm = 1 / (1 + math.exp(-r))
    N = n_samples
    k = np.arange(N, dtype=np.float64)
    checked = 0
    for i in np.nonzero(hit)[0][:12]:
        delta = float(np.float32((tf[i] - tn[i]) / np.float32(N)))
        t_k = np.float32(tn[i]) + (k.astype(np.float32) + np.float32(0.5)) * np.float32(delta)
        t_k = t_k.astype(np.float64)

        def E(s):
            q = math.exp(-s * delta)
            return float(np.sum(t_k * q ** k * (1.0 - q)))

        h = 1e-6
        dE = (E(sigma + h) - E(sigma - h)) / (2 * h)
        g, _ = orc.render_backward(m, op, o[i:i + 1], d[i:i + 1], np.zeros((1, 3)), d_depth_t=np.ones(1))
        want = dE * sgm
        assert abs(g["density"].sum() - want) <= 1e-7 * max(1.0, abs(want)), (g["density"].sum(), want)
        assert np.all(g["features"] == 0.0)
        checked += 1
    assert checked == 12
