"""Pins for the oracle's sparse radiance warping (Eq. 1-4) against closed
forms: identity warp, pure rotation (a homography independent of depth),
fronto-parallel translation (an exact pixel shift), equal-depth collisions
(smallest source index wins), points at infinity, and the two limits of the
merge (all pixels holes / no holes)."""
import numpy as np

import synth


def _cam(orc, W, H, pose, f=None):
    ff, cx, cy = synth.intrinsics(W, H)
    if f is not None:
        ff = f
    return orc.camera(W, H, ff, cx, cy, synth.as_f32(pose))


def _ident():
    return np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)


def test_identity_warp_reproduces_reference(orc):
    W, H = 48, 40
    rng = np.random.default_rng(0)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    dep = rng.uniform(2.0, 6.0, W * H).astype(np.float32)
    dep[rng.choice(W * H, 200, replace=False)] = np.inf  # void pixels
    cam = _cam(orc, W, H, synth.orbit_pose(0))
    out, od, mask, src = orc.warp(cam, cam, _ident(), rgb, dep)
    assert mask.sum() == 0
    assert np.array_equal(src, np.arange(W * H))
    assert np.array_equal(out, rgb)
    assert np.array_equal(od, dep)


def test_pure_rotation_is_a_depth_independent_homography(orc):
    W, H = 64, 48
    ang = np.deg2rad(2.0)
    Rz = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(ang), -np.sin(ang)], [0, np.sin(ang), np.cos(ang)]])
    R = Rz @ Rx
    T = np.concatenate([R, np.zeros((3, 1))], 1).reshape(12).astype(np.float32)
    cam = _cam(orc, W, H, synth.orbit_pose(0))
    rng = np.random.default_rng(1)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    masks = []
    for seed in (2, 3):
        dep = np.random.default_rng(seed).uniform(1.0, 9.0, W * H).astype(np.float32)
        _, od, mask, src = orc.warp(cam, cam, T, rgb, dep)
        masks.append(mask)
        # each winner lands where the float64 homography K R K^-1 puts it
        f, cx, cy = cam.f, cam.cx, cam.cy
        ok = src >= 0
        s = src[ok]
        i, j = s % W, s // W
        v = np.stack([(i + 0.5 - cx) / f, (j + 0.5 - cy) / f, np.ones_like(i, dtype=float)], 0)
        p = R.astype(np.float32).astype(np.float64) @ v
        u = f * p[0] / p[2] + cx
        vv = f * p[1] / p[2] + cy
        tgt = np.nonzero(ok)[0]
        ti, tj = tgt % W, tgt // W
        clear = (np.abs(u - np.round(u)) > 1e-3) & (np.abs(vv - np.round(vv)) > 1e-3)
        assert np.array_equal(np.floor(u[clear]).astype(int), ti[clear])
        assert np.array_equal(np.floor(vv[clear]).astype(int), tj[clear])
    assert np.array_equal(masks[0], masks[1])
    assert 0 < masks[0].sum() < W * H // 4


def test_fronto_parallel_translation_shifts_by_k_pixels(orc):
    """Plane at depth D, camera moved right by k*D/f: every pixel moves k
    pixels left and the hole mask is the k-pixel strip at the right edge."""
    W, H, D, f, k = 64, 32, 2.0, 64.0, 3
    cam = _cam(orc, W, H, synth.orbit_pose(0), f=f)
    tx = k * D / f
    T = _ident()
    T[3] = -tx
    rng = np.random.default_rng(4)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    dep = np.full(W * H, D, np.float32)
    out, od, mask, src = orc.warp(cam, cam, T, rgb, dep)
    m2 = mask.reshape(H, W)
    assert np.all(m2[:, W - k:] == 1) and np.all(m2[:, :W - k] == 0)
    img = rgb.reshape(H, W, 3)
    assert np.array_equal(out.reshape(H, W, 3)[:, :W - k], img[:, k:])
    assert np.all(od.reshape(H, W)[:, :W - k] == np.float32(D))


def test_equal_depth_collisions_keep_smallest_source(orc):
    """Camera moved back by D along its axis while looking at a plane at
    depth D: every 2x2 block of reference pixels lands in one target pixel
    at equal depth 2D; the top-left (smallest index) source must win."""
    W, H, D = 32, 32, 2.0
    cam = _cam(orc, W, H, synth.orbit_pose(0), f=32.0)
    T = _ident()
    T[11] = D
    rgb = np.random.default_rng(5).uniform(0, 1, (W * H, 3)).astype(np.float32)
    dep = np.full(W * H, D, np.float32)
    out, od, mask, src = orc.warp(cam, cam, T, rgb, dep)
    # u_t = (i + 1/2 - cx)/2 + cx  ->  floor((i + 1/2)/2 + cx/2)
    cx = cam.cx
    for ti in range(W):
        for tj in range(H):
            p = tj * W + ti
            cand = [(j * W + i) for i in range(W) for j in range(H)
                    if int(np.floor((i + 0.5 - cx) / 2 + cx)) == ti
                    and int(np.floor((j + 0.5 - cx) / 2 + cx)) == tj]
            if cand:
                assert src[p] == min(cand) and mask[p] == 0
                assert od[p] == np.float32(2 * D)
            else:
                assert mask[p] == 1 and src[p] == -1


def test_points_at_infinity_rotate_only(orc):
    """Void reference pixels (depth +inf) ignore translation, keep depth
    +inf and lose to any finite splat on the same target pixel."""
    W, H = 40, 40
    cam = _cam(orc, W, H, synth.orbit_pose(0))
    rgb = np.random.default_rng(6).uniform(0, 1, (W * H, 3)).astype(np.float32)
    dep = np.full(W * H, np.inf, np.float32)
    T = _ident()
    T[3], T[7], T[11] = 0.5, -0.3, 0.7
    out, od, mask, src = orc.warp(cam, cam, T, rgb, dep)
    assert mask.sum() == 0 and np.all(np.isinf(od))
    assert np.array_equal(out, rgb)
    dep2 = dep.copy()
    dep2[5 * W + 7] = 3.0   # one finite point; it lands somewhere else
    out2, od2, mask2, src2 = orc.warp(cam, cam, T, rgb, dep2)
    hit = np.nonzero(src2 == 5 * W + 7)[0]
    assert len(hit) == 1 and np.isfinite(od2[hit[0]])


def test_sparw_limits(orc):
    """Eq. 4 merge: with every pixel a hole the result is the full render;
    with the identity pose it is the reference frame and no pixel is
    rendered."""
    dens, feats = synth.make_scene(16, seed=8)
    m = orc.Model(dens, feats, synth.make_mlp(9), density_shift=synth.DENSITY_SHIFT)
    m.set_occupancy(orc.build_occupancy(m))
    op = orc.opts(32, et_threshold=1e-4, use_occupancy=True)
    W, H = 24, 24
    cam = _cam(orc, W, H, synth.orbit_pose(0))
    rgb, dz, acc, _ = orc.render_pixels(m, op, cam)
    rgb32, dz32 = rgb.astype(np.float32), dz.astype(np.float32)
    out, od, mask, nm = orc.sparw(m, op, cam, rgb32, dz32, cam, _ident())
    assert nm == 0 and mask.sum() == 0
    assert np.array_equal(out, rgb32.astype(np.float64))
    far = _ident()
    far[0], far[10] = -1.0, -1.0   # half-turn about y: every point and direction behind
    out, od, mask, nm = orc.sparw(m, op, cam, rgb32, dz32, cam, far)
    assert nm == W * H and mask.all()
    assert np.array_equal(out, rgb)
    np.testing.assert_array_equal(od, dz)


def test_mask_shrinks_as_target_approaches_reference(orc):
    W, H = 64, 64
    dens, feats = synth.make_scene(24, seed=0)
    m = orc.Model(dens, feats, synth.make_mlp(1), density_shift=synth.DENSITY_SHIFT)
    m.set_occupancy(orc.build_occupancy(m))
    op = orc.opts(64, et_threshold=1e-4, use_occupancy=True)
    ref_pose = synth.orbit_pose(0)
    cam = _cam(orc, W, H, ref_pose)
    rgb, dz, _, _ = orc.render_pixels(m, op, cam)
    fr = []
    for step in (8.0, 4.0, 2.0, 1.0, 0.0):
        tp = synth.orbit_pose(1, step_deg=step)
        T = synth.relative_pose(synth.as_f32(ref_pose), synth.as_f32(tp))
        tcam = _cam(orc, W, H, tp)
        _, _, mask, _ = orc.warp(cam, tcam, T, rgb.astype(np.float32), dz.astype(np.float32))
        fr.append(mask.mean())
    assert fr[-1] == 0.0
    assert all(a >= b for a, b in zip(fr, fr[1:])), fr


def test_angle_threshold_limits(orc):
    """Sec. III-C warp-angle test: 180 degrees equals no test; an identity
    warp subtends no angle; points at infinity always pass."""
    W, H = 48, 40
    rng = np.random.default_rng(9)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    dep = rng.uniform(2.0, 6.0, W * H).astype(np.float32)
    dep[:100] = np.inf
    rp, tp = synth.orbit_pose(0), synth.orbit_pose(1, step_deg=6.0)
    cr, ct = _cam(orc, W, H, rp), _cam(orc, W, H, tp)
    T = synth.relative_pose(synth.as_f32(rp), synth.as_f32(tp))
    a = orc.warp(cr, ct, T, rgb, dep)
    b = orc.warp(cr, ct, T, rgb, dep, max_angle_deg=180.0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    c = orc.warp(cr, cr, _ident(), rgb, dep, max_angle_deg=0.5)
    assert c[2].sum() == 0
    allvoid = np.full(W * H, np.inf, np.float32)
    d = orc.warp(cr, ct, T, rgb, allvoid, max_angle_deg=0.5)
    e = orc.warp(cr, ct, T, rgb, allvoid)
    assert np.array_equal(d[2], e[2])


def test_angle_threshold_closed_form(orc):
    """Plane at depth D seen by two cameras a baseline b apart along x: the
    reference pixel whose point lies at x (reference camera frame) subtends
    the angle between (x, y, D) and (x - b, y, D) at the point.  A target
    pixel keeps the point the plain warp puts there when that point's angle
    is below the threshold and becomes a hole otherwise.  Checked against
    the float64 angle away from the boundary."""
    W, H, D, f = 64, 48, 2.0, 40.0
    cam = _cam(orc, W, H, synth.orbit_pose(0), f=f)
    b = 0.25
    T = _ident()
    T[3] = -b          # target camera moved by +b along x
    rng = np.random.default_rng(10)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    dep = np.full(W * H, D, np.float32)
    phi = 6.0
    _, _, m_plain, src_plain = orc.warp(cam, cam, T, rgb, dep)
    r_phi, _, m_phi, src_phi = orc.warp(cam, cam, T, rgb, dep, max_angle_deg=phi)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    x = (ii.ravel() + 0.5 - cam.cx) / f * D
    y = (jj.ravel() + 0.5 - cam.cy) / f * D
    # in target coordinates the point is (x - b, y, D), the reference centre (-b, 0, 0)
    vt = np.stack([x - b, y, np.full_like(x, D)], 1)
    vr = np.stack([x, y, np.full_like(x, D)], 1)
    cosang = (vt * vr).sum(1) / (np.linalg.norm(vt, axis=1) * np.linalg.norm(vr, axis=1))
    ang = np.degrees(np.arccos(np.clip(cosang, -1, 1)))
    passes = ang < phi
    covered = src_plain >= 0
    s = src_plain[covered]
    clear = np.abs(ang[s] - phi) > 1e-3
    expect = np.where(passes[s], s, -1)
    assert np.array_equal(src_phi[covered][clear], expect[clear])
    assert np.all(src_phi[~covered] == -1)
    assert 0 < passes[s].mean() < 1
    hole = src_phi < 0
    assert np.array_equal(m_phi.astype(bool), hole)
    assert np.all(r_phi[hole] == 0)
    assert np.array_equal(r_phi[~hole], rgb[src_phi[~hole]])


def test_angle_threshold_nests(orc):
    """A smaller threshold only adds holes: every pixel warped under the
    smaller threshold is warped, from the same reference pixel, under the
    larger one and without the test (quality can only rise as the threshold
    falls, the trend of the paper's threshold sweep)."""
    W, H = 64, 48
    rng = np.random.default_rng(11)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    # two depth layers so that near points occlude far ones in the target
    dep = np.where((ii // 8 + jj // 8) % 2 == 0, 2.0, 4.5).astype(np.float32).ravel()
    dep[rng.uniform(size=W * H) < 0.05] = np.inf
    rp, tp = synth.orbit_pose(0), synth.orbit_pose(1, step_deg=12.0)
    cr, ct = _cam(orc, W, H, rp), _cam(orc, W, H, tp)
    T = synth.relative_pose(synth.as_f32(rp), synth.as_f32(tp))
    prev = orc.warp(cr, ct, T, rgb, dep)[3]
    counts = [int((prev < 0).sum())]
    for phi in (8.0, 5.0, 3.0, 1.0):
        cur = orc.warp(cr, ct, T, rgb, dep, max_angle_deg=phi)[3]
        kept = cur >= 0
        assert np.array_equal(cur[kept], prev[kept])
        counts.append(int((cur < 0).sum()))
        prev = cur
    assert counts == sorted(counts) and counts[-1] > counts[0]
