"""Pins for the oracle's rendering path, independent of the oracle itself.

Each test checks the oracle against something the paper or mathematics fixes:
closed forms of the rendering quadrature on a constant-density box, exactness
of trilinear interpolation on multilinear fields, a library interpolator and a
library MLP, an independent brute-force renderer built from numpy/scipy/torch
primitives, and invariants (opacity in [0,1], weights summing to opacity,
empty grids rendering the background).
"""
import math

import numpy as np
import pytest

import synth

LO, HI = np.array(synth.BOX_LO), np.array(synth.BOX_HI)


def _model(orc, dens, feats, mlp, shift=0.0, occ=None):
    return orc.Model(dens, feats, mlp, density_shift=shift, occ=occ)


def _const_mlp(n_feat, beta, seed=3):
    """MLP whose output is the constant sigmoid(beta) (W2 = 0)."""
    m = synth.make_mlp(seed, in_dim=n_feat + 27)
    m["w2"][:] = 0.0
    m["b2"][:] = np.float32(beta)
    return m


def _slab64(o, d):
    """float64 slab interval of rays against the box."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d.astype(np.float64)
        t0 = (LO - o) * inv
        t1 = (HI - o) * inv
    tn = np.nanmax(np.minimum(t0, t1), axis=1)
    tf = np.nanmin(np.maximum(t0, t1), axis=1)
    tn = np.maximum(tn, 0.0)
    return tn, tf


def _softplus(x):
    return np.logaddexp(0.0, x)


@pytest.mark.parametrize("n_samples", [1, 7, 64, 256])
def test_constant_box_opacity_colour_depth(orc, n_samples):
    """Constant density sigma on the box: opacity is exactly 1-exp(-sigma L)
    for any N (sum of steps equals L); a constant MLP colour s gives
    C = s*acc + bg*(1-acc); expected distance is the geometric-series
    closed form."""
    R, nf = 9, 12
    raw = 1.3
    shift = -0.4
    dens = np.full((R, R, R), raw, np.float32)
    feats = np.random.default_rng(0).standard_normal((R, R, R, nf)).astype(np.float32)
    beta = 0.7
    m = _model(orc, dens, feats, _const_mlp(nf, beta), shift=shift)
    o, d = synth.random_rays(300, seed=11)
    bg = (1.0, 0.25, 0.5)
    op = orc.opts(n_samples, bg=bg)
    rgb, dep, acc, diag = orc.render_rays(m, op, o, d, diagnostics=True)
    sigma = _softplus(np.float64(np.float32(raw) + np.float32(shift)))
    tn, tf = _slab64(o, d)
    hit = tn < tf
    L = np.where(hit, tf - tn, 0.0)
    acc_cf = 1.0 - np.exp(-sigma * L)
    np.testing.assert_allclose(acc, acc_cf, rtol=0, atol=2e-6)
    s = 1.0 / (1.0 + math.exp(-float(np.float32(beta))))
    for ch in range(3):
        np.testing.assert_allclose(rgb[:, ch], s * acc + bg[ch] * (1 - acc), rtol=0, atol=1e-12)
    # expected distance, geometric series with q = exp(-sigma*delta)
    N = n_samples
    delta = L / N
    q = np.exp(-sigma * delta)
    geo = np.where(hit, q * (1 - N * q ** (N - 1) + (N - 1) * q ** N) / np.maximum((1 - q) ** 2, 1e-300), 0.0)
    et_cf = (1 - q ** N) * (tn + delta / 2) + delta * (1 - q) * geo
    et_cf = np.where(hit, et_cf, 0.0)
    # sample distances are float32 (ulp ~5e-7 at t ~ 5): allow a few ulps
    np.testing.assert_allclose(dep, et_cf, rtol=0, atol=1e-5)
    assert np.all(diag["n_eval"][hit] == N) and np.all(diag["n_eval"][~hit] == 0)
    assert np.all(acc[~hit] == 0.0)


def test_termination_index_closed_form(orc):
    """Early termination: sample k is evaluated iff exp(-sigma k delta) >=
    thr, so the count is the first k with exp(-sigma k delta) < thr."""
    R, nf = 5, 12
    dens = np.full((R, R, R), 4.0, np.float32)
    feats = np.zeros((R, R, R, nf), np.float32)
    m = _model(orc, dens, feats, _const_mlp(nf, 0.0), shift=0.0)
    o, d = synth.random_rays(200, seed=12)
    thr = 1e-4
    op = orc.opts(256, et_threshold=thr)
    rgb, dep, acc, diag = orc.render_rays(m, op, o, d, diagnostics=True)
    sigma = _softplus(4.0)
    tn, tf = _slab64(o, d)
    hit = tn < tf
    delta = np.where(hit, (tf - tn) / 256, 1.0)
    ratio = math.log(1 / thr) / (sigma * delta)
    kstar = np.minimum(np.floor(ratio).astype(int) + 1, 256)
    safe = hit & (np.abs(ratio - np.round(ratio)) > 1e-3)
    assert safe.sum() > 50
    np.testing.assert_array_equal(diag["n_eval"][safe], kstar[safe])
    acc_cf = 1 - np.exp(-sigma * kstar * delta)
    np.testing.assert_allclose(acc[safe], acc_cf[safe], rtol=0, atol=5e-6)  # float32 step


def test_trilinear_exact_on_multilinear_fields(orc):
    """Trilinear interpolation reproduces any multilinear field exactly and
    returns vertex values at vertices (align-corners grid)."""
    rng = np.random.default_rng(3)
    R = (7, 9, 6)
    coef = rng.standard_normal((8, 2))
    ax = [np.linspace(LO[a], HI[a], R[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")

    def field(x, y, z, c):
        return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z
                + c[6] * y * z + c[7] * x * y * z)

    vals = np.stack([field(X, Y, Z, coef[:, ch]) for ch in range(2)], -1).astype(np.float32)
    dens = vals[..., 0].copy()
    m = _model(orc, dens, vals, synth.make_mlp(1, in_dim=2 + 27))
    pos = rng.uniform(-1.5, 1.5, (500, 3)).astype(np.float32)
    got = orc.trilerp(m, vals, pos)
    # exact field from the float32 vertex values: interpolate in float64
    # through the per-cell multilinear form evaluated at the float64 position
    want = np.stack([field(pos[:, 0].astype(np.float64), pos[:, 1].astype(np.float64),
                           pos[:, 2].astype(np.float64), coef[:, ch]) for ch in range(2)], -1)
    np.testing.assert_allclose(got, want, rtol=0, atol=5e-5)  # float32 vertex storage
    # vertices
    ii = rng.integers(0, R[0], 50), rng.integers(0, R[1], 50), rng.integers(0, R[2], 50)
    vp = np.stack([ax[0][ii[0]], ax[1][ii[1]], ax[2][ii[2]]], -1).astype(np.float32)
    gv = orc.trilerp(m, vals, vp)
    np.testing.assert_allclose(gv, vals[ii[0], ii[1], ii[2]], rtol=0, atol=1e-5)


def test_trilinear_matches_scipy(orc):
    """The gather equals scipy's RegularGridInterpolator (linear) on the
    vertex lattice spanning the box corners."""
    from scipy.interpolate import RegularGridInterpolator
    rng = np.random.default_rng(4)
    R = 11
    vals = rng.standard_normal((R, R, R, 3)).astype(np.float32)
    m = _model(orc, vals[..., 0].copy(), vals, synth.make_mlp(1, in_dim=3 + 27))
    pos = rng.uniform(-1.5, 1.5, (400, 3)).astype(np.float32)
    got = orc.trilerp(m, vals, pos)
    ax = np.linspace(-1.5, 1.5, R)
    ref = RegularGridInterpolator((ax, ax, ax), vals.astype(np.float64))(pos.astype(np.float64))
    # float32 voxel coordinate (ulp ~1e-6 at u ~ 10) times slopes of O(1)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-5)


def test_mlp_matches_torch(orc):
    """The per-sample MLP equals torch.nn Linear/ReLU/Sigmoid in float64."""
    import torch
    mlp = synth.make_mlp(7, bias_std=0.3)
    m = _model(orc, np.zeros((2, 2, 2), np.float32), np.zeros((2, 2, 2, 12), np.float32), mlp)
    x = np.random.default_rng(8).standard_normal((64, 39))
    got = orc.mlp_forward(m, x)
    net = torch.nn.Sequential(torch.nn.Linear(39, 128), torch.nn.ReLU(), torch.nn.Linear(128, 128),
                              torch.nn.ReLU(), torch.nn.Linear(128, 3), torch.nn.Sigmoid()).double()
    with torch.no_grad():
        for li, k in zip((0, 2, 4), ("0", "1", "2")):
            net[li].weight.copy_(torch.from_numpy(mlp["w" + k].astype(np.float64)))
            net[li].bias.copy_(torch.from_numpy(mlp["b" + k].astype(np.float64)))
        ref = net(torch.from_numpy(x)).numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_mlp_input_layout_worked_example(orc):
    """Input vector for d = (1, 0, 0) and features 0..11: features, then d,
    then sin(2^m d_c) (c outer, m inner), then cos(2^m d_c)."""
    m = _model(orc, np.zeros((2, 2, 2), np.float32), np.zeros((2, 2, 2, 12), np.float32), synth.make_mlp(1))
    feat = np.arange(12, dtype=np.float64)[None]
    x = orc.mlp_input(m, feat, np.array([[1.0, 0.0, 0.0]], np.float32))[0]
    want = list(range(12)) + [1.0, 0.0, 0.0]
    want += [math.sin(1), math.sin(2), math.sin(4), math.sin(8)] + [0.0] * 8
    want += [math.cos(1), math.cos(2), math.cos(4), math.cos(8)] + [1.0] * 8
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-15)


def _brute_render(dens, feats, mlp, shift, o, d, N, bg):
    """Independent renderer from library primitives: float64 slab and
    samples, scipy trilinear interpolation, numpy softplus and cumulative
    product for transmittance, torch MLP."""
    import torch
    from scipy.interpolate import RegularGridInterpolator
    R = dens.shape[0]
    ax = np.linspace(-1.5, 1.5, R)
    fd = RegularGridInterpolator((ax, ax, ax), dens.astype(np.float64))
    ff = RegularGridInterpolator((ax, ax, ax), feats.astype(np.float64))
    n_feat = feats.shape[-1]
    net = torch.nn.Sequential(torch.nn.Linear(n_feat + 27, 128), torch.nn.ReLU(), torch.nn.Linear(128, 128),
                              torch.nn.ReLU(), torch.nn.Linear(128, 3), torch.nn.Sigmoid()).double()
    with torch.no_grad():
        for li, k in zip((0, 2, 4), ("0", "1", "2")):
            net[li].weight.copy_(torch.from_numpy(mlp["w" + k].astype(np.float64)))
            net[li].bias.copy_(torch.from_numpy(mlp["b" + k].astype(np.float64)))
    tn, tf = _slab64(o.astype(np.float64), d.astype(np.float64))
    out = np.zeros((len(o), 3))
    for r in range(len(o)):
        if not tn[r] < tf[r]:
            out[r] = bg
            continue
        delta = (tf[r] - tn[r]) / N
        t = tn[r] + (np.arange(N) + 0.5) * delta
        pts = np.clip(o[r].astype(np.float64) + t[:, None] * d[r].astype(np.float64), -1.5, 1.5)
        sigma = np.logaddexp(0.0, fd(pts) + shift)
        alpha = 1 - np.exp(-sigma * delta)
        trans = np.concatenate([[1.0], np.cumprod(1 - alpha)])
        w = trans[:-1] * alpha
        dd = d[r].astype(np.float64)
        pe = [dd] + [np.sin(2.0 ** k * dd[c]) for c in range(3) for k in range(4)]
        pe = np.concatenate([np.atleast_1d(v) for v in pe])
        pe_cos = np.array([np.cos(2.0 ** k * dd[c]) for c in range(3) for k in range(4)])
        x = np.concatenate([ff(pts), np.tile(np.concatenate([pe, pe_cos]), (N, 1))], axis=1)
        with torch.no_grad():
            c = net(torch.from_numpy(x)).numpy()
        out[r] = (w[:, None] * c).sum(0) + trans[-1] * np.asarray(bg)
    return out


def test_brute_force_8x8(orc):
    """An 8x8 frame from the oracle agrees with the brute-force renderer."""
    dens, feats = synth.make_scene(16, seed=21)
    mlp = synth.make_mlp(22, bias_std=0.1)
    shift = synth.DENSITY_SHIFT
    m = _model(orc, dens, feats, mlp, shift=shift)
    f, cx, cy = synth.intrinsics(8, 8)
    cam = orc.camera(8, 8, f, cx, cy, synth.as_f32(synth.orbit_pose(17)))
    o, d = orc.generate_rays(cam)
    bg = (1.0, 1.0, 1.0)
    rgb, _, _ = orc.render_rays(m, orc.opts(48, bg=bg), o, d)
    ref = _brute_render(dens, feats, mlp, np.float64(np.float32(shift)), o, d, 48, bg)
    np.testing.assert_allclose(rgb, ref, rtol=0, atol=2e-5)


def test_weights_nonnegative_and_sum_to_opacity(orc):
    """With a constant MLP colour, C = s*sum(w) + bg*T_stop: sum(w) equals
    the opacity 1-T_stop, and opacity stays in [0, 1] (all weights are
    non-negative products of transmittance and alpha)."""
    dens, feats = synth.make_scene(24, seed=5)
    beta = 1.1
    m = _model(orc, dens, feats, _const_mlp(12, beta), shift=synth.DENSITY_SHIFT)
    o, d = synth.random_rays(500, seed=13)
    bg = (0.0, 0.0, 0.0)
    rgb, dep, acc = orc.render_rays(m, orc.opts(128, et_threshold=1e-4, bg=bg), o, d)
    s = 1 / (1 + math.exp(-float(np.float32(beta))))
    np.testing.assert_allclose(rgb[:, 0] / s, acc, rtol=1e-12, atol=1e-15)
    assert np.all(acc >= 0.0) and np.all(acc <= 1.0)
    tn, tf = _slab64(o, d)
    assert np.all(dep >= 0.0) and np.all(dep <= np.where(tn < tf, tf, 0.0) * acc + 1e-9)


def test_ray_generation(orc):
    """Pixel rays: unit length, origin at the camera centre, camera-space
    direction proportional to (i+1/2-cx, j+1/2-cy, f)."""
    pose = synth.orbit_pose(5)
    W, H = 40, 30
    f, cx, cy = synth.intrinsics(W, H)
    c2w = synth.as_f32(pose)
    cam = orc.camera(W, H, f, cx, cy, c2w)
    o, d = orc.generate_rays(cam)
    np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=1), 1.0, atol=3e-7)
    Rm = c2w.reshape(3, 4)[:, :3].astype(np.float64)
    assert np.all(o == c2w.reshape(3, 4)[:, 3])
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    v = np.stack([ii.ravel() + 0.5 - cx, jj.ravel() + 0.5 - cy, np.full(W * H, f)], -1)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    np.testing.assert_allclose(d @ Rm, v, atol=1e-6)  # R^T d back in camera space
    # subset selection picks the same rays
    pix = synth.pixel_subset(W, H, 50, seed=3)
    o2, d2 = orc.generate_rays(cam, pix)
    assert np.array_equal(d2, d[pix]) and np.array_equal(o2, o[pix])


def test_ray_box(orc):
    o, d = synth.random_rays(2000, seed=14)
    tn, tf, hit = orc.ray_box(o, d)
    tn64, tf64 = _slab64(o, d)
    hit64 = tn64 < tf64
    clear = np.abs(tf64 - tn64) > 1e-4
    assert np.array_equal(hit[clear], hit64[clear])
    np.testing.assert_allclose(tn[hit & clear], tn64[hit & clear], atol=2e-6)
    np.testing.assert_allclose(tf[hit & clear], tf64[hit & clear], atol=2e-6)
    assert hit.sum() > 500 and (~hit).sum() > 50


def test_occupancy_conservative_and_empty_grid(orc):
    """A voxel is skipped only if all eight vertex densities are <= the cut;
    a grid below the cut everywhere renders the background with opacity 0
    when skipping is on."""
    dens, feats = synth.make_scene(20, seed=6)
    shift = np.float32(synth.DENSITY_SHIFT)
    m = _model(orc, dens, feats, synth.make_mlp(1), shift=shift)
    occ = orc.build_occupancy(m, 1e-2)
    sig = _softplus(dens.astype(np.float64) + np.float64(shift))
    above = sig > 1e-2
    cell_any = np.zeros(occ.shape, bool)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                cell_any |= above[dx:dx + 19, dy:dy + 19, dz:dz + 19]
    near = np.abs(sig - 1e-2) < 1e-7
    near_cell = np.zeros(occ.shape, bool)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                near_cell |= near[dx:dx + 19, dy:dy + 19, dz:dz + 19]
    assert np.array_equal(occ.astype(bool)[~near_cell], cell_any[~near_cell])
    assert 0.05 < occ.mean() < 0.95
    # empty grid
    empty = np.full_like(dens, -20.0)
    m2 = _model(orc, empty, feats, synth.make_mlp(1), shift=shift)
    occ2 = orc.build_occupancy(m2, 1e-2)
    assert occ2.sum() == 0
    m2.set_occupancy(occ2)
    o, d = synth.random_rays(100, seed=15)
    bg = (0.2, 0.4, 0.6)
    rgb, dep, acc = orc.render_rays(m2, orc.opts(64, use_occupancy=True, bg=bg), o, d)
    assert np.all(acc == 0.0) and np.all(dep == 0.0)
    assert np.all(rgb == np.array(bg, np.float32).astype(np.float64))


def test_occupancy_skip_error_bound(orc):
    """Skipping changes a ray's colour by at most the density cut times the
    ray length (each skipped sample has sigma <= cut)."""
    dens, feats = synth.make_scene(24, seed=7)
    shift = synth.DENSITY_SHIFT
    m = _model(orc, dens, feats, synth.make_mlp(1), shift=shift)
    occ = orc.build_occupancy(m, 1e-2)
    o, d = synth.random_rays(300, seed=16)
    a = orc.render_rays(m, orc.opts(128), o, d)[0]
    m.set_occupancy(occ)
    b = orc.render_rays(m, orc.opts(128, use_occupancy=True), o, d)[0]
    tn, tf = _slab64(o, d)
    L = np.where(tn < tf, tf - tn, 0.0)
    bound = 2 * 1e-2 * L + 1e-12
    assert np.all(np.abs(a - b).max(1) <= bound)


def test_bf16_mode_matches_torch_bfloat16(orc):
    """Precision mode: every layer's inputs and weights rounded to bfloat16
    (round to nearest even) with float64 accumulation equals torch's
    bfloat16 conversion followed by float64 Linear/ReLU/Sigmoid."""
    import torch
    mlp = synth.make_mlp(11, bias_std=0.2)
    m = orc.Model(np.zeros((2, 2, 2), np.float32), np.zeros((2, 2, 2, 12), np.float32), mlp, round_bf16=True)
    x = np.random.default_rng(12).standard_normal((128, 39)) * 2.0
    got = orc.mlp_forward(m, x)

    def r(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    with torch.no_grad():
        h = torch.from_numpy(x)
        for k, act in (("0", torch.relu), ("1", torch.relu), ("2", torch.sigmoid)):
            w = r(torch.from_numpy(mlp["w" + k]))
            b = torch.from_numpy(mlp["b" + k].astype(np.float64))
            h = act(r(h) @ w.T + b)
    np.testing.assert_allclose(got, h.numpy(), rtol=0, atol=1e-13)
    # and it is a different function from the float64 one
    m64 = orc.Model(np.zeros((2, 2, 2), np.float32), np.zeros((2, 2, 2, 12), np.float32), mlp)
    assert np.abs(orc.mlp_forward(m64, x) - got).max() > 1e-4
