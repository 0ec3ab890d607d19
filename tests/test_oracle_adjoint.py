"""Pins for the oracle's adjoint: central finite differences of the float64
forward on a small model (8^3 grid, 4 feature channels, 16 rays, 64 samples,
no skipping or termination), the adjoint identity of the trilinear
gather/scatter pair, and the closed-form derivative of a constant-density
box's opacity and colour."""
import math

import numpy as np
import pytest

import synth


def _setup(orc, n_feat=4, R=8, seed=30):
    rng = np.random.default_rng(seed)
    dens = rng.normal(0.0, 1.0, (R, R, R)).astype(np.float32) + 3.0
    feats = rng.normal(0.0, 1.0, (R, R, R, n_feat)).astype(np.float32)
    # hidden width 32 keeps the ~6000 forward evaluations cheap; the adjoint
    # formulas do not depend on the width
    mlp = synth.make_mlp(seed + 1, in_dim=n_feat + 27, hidden=32, bias_std=0.1)
    m = orc.Model(dens, feats, mlp, density_shift=-2.0)
    f, cx, cy = synth.intrinsics(64, 64)
    cam = orc.camera(64, 64, f, cx, cy, synth.as_f32(synth.orbit_pose(10)))
    pix = synth.pixel_subset(64, 64, 16, seed=seed + 2)
    o, d = orc.generate_rays(cam, pix)
    gt = rng.uniform(0, 1, (16, 3))
    return m, o, d, gt


def _loss(orc, m, op, o, d, gt):
    rgb, _, _, diag = orc.render_rays(m, op, o, d, diagnostics=True)
    return float(np.mean((rgb - gt) ** 2)), diag["relu_sig"].copy(), rgb


def test_finite_differences(orc):
    m, o, d, gt = _setup(orc)
    op = orc.opts(64)
    L0, sig0, rgb = _loss(orc, m, op, o, d, gt)
    d_rgb = 2.0 * (rgb - gt) / rgb.size
    g, _ = orc.render_backward(m, op, o, d, d_rgb)
    eps = 1e-3
    rng = np.random.default_rng(31)

    def fd(arr, idx):
        old = arr[idx]
        arr[idx] = old + eps
        lp, sp, _ = _loss(orc, m, op, o, d, gt)
        arr[idx] = old - eps
        lm, sm, _ = _loss(orc, m, op, o, d, gt)
        arr[idx] = old
        flip = not (np.array_equal(sp, sig0) and np.array_equal(sm, sig0))
        return (lp - lm) / (2 * eps), flip

    # Finite differences of float32 parameters: perturb the float32 array in
    # place (the oracle reads it through a pointer), steps are exact in
    # float32 for values of this magnitude up to ~1e-7 relative.
    checks = []
    dens = m.density
    for idx in np.ndindex(dens.shape):
        checks.append(("density", dens, idx, g["density"][idx]))
    feats = m.features
    for idx in np.ndindex(feats.shape):
        checks.append(("features", feats, idx, g["features"][idx]))
    for k in ("w0", "b0", "w1", "b1", "w2", "b2"):
        arr = m.w[k]
        n = arr.size
        take = rng.choice(n, size=min(n, 420), replace=False)
        for t in take:
            idx = np.unravel_index(t, arr.shape)
            checks.append((k, arr, idx, g[k][idx]))
    n_grid = 8 ** 3 * 5
    assert sum(c[0] in ("density", "features") for c in checks) == n_grid
    scale = max(np.abs(g["density"]).max(), np.abs(g["features"]).max(), np.abs(g["w1"]).max())
    bad, flips, mlp_checked = [], 0, 0
    for name, arr, idx, ga in checks:
        # the actual float32 step
        old = arr[idx]
        up = np.float32(old + eps) - old
        dn = old - np.float32(old - eps)
        gf, flip = fd(arr, idx)
        gf = gf * (2 * eps) / (float(up) + float(dn))
        if flip:
            # a ReLU crossing inside [-eps, eps] makes the difference quotient
            # first-order accurate only; such entries are excluded and counted
            flips += 1
            continue
        mlp_checked += name not in ("density", "features")
        if abs(gf - ga) > 1e-7 * scale + 1e-5 * abs(ga):
            bad.append((name, idx, gf, ga))
    assert not bad, bad[:10]
    assert mlp_checked >= 512, (mlp_checked, flips)
    assert flips < len(checks) // 4, flips


def test_gather_scatter_adjoint_identity(orc):
    """<gather(G), y> == <G, scatter(y)> for random G, y and positions."""
    rng = np.random.default_rng(40)
    R, C = 9, 5
    G = rng.standard_normal((R, R, R, C)).astype(np.float32)
    m = orc.Model(G[..., 0].copy(), G, synth.make_mlp(1, in_dim=C + 27))
    pos = rng.uniform(-1.6, 1.6, (700, 3)).astype(np.float32)   # some outside: clamped
    y = rng.standard_normal((700, C))
    lhs = float(np.sum(orc.trilerp(m, G, pos) * y))
    rhs = float(np.sum(G.astype(np.float64) * orc.trilerp_scatter(m, C, pos, y)))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


@pytest.mark.parametrize("n_samples", [16, 64])
def test_constant_box_derivatives(orc, n_samples):
    """Constant raw density r on every vertex: the sum of the density
    gradient over vertices is d/dr of the loss, since a uniform shift of all
    vertices shifts the interpolated value uniformly.  With d_acc = 1 that
    is L exp(-sigma L) sigmoid(r + b); with a constant colour s and d_rgb =
    (1, 0, 0) it is (s - bg) L exp(-sigma L) sigmoid(r + b)."""
    R, nf = 6, 12
    raw, shift = 0.8, -0.5
    dens = np.full((R, R, R), raw, np.float32)
    feats = np.random.default_rng(41).standard_normal((R, R, R, nf)).astype(np.float32)
    mlp = synth.make_mlp(42)
    mlp["w2"][:] = 0.0
    mlp["b2"][:] = np.float32(0.3)
    m = orc.Model(dens, feats, mlp, density_shift=shift)
    o, d = synth.random_rays(64, seed=43)
    bg = (0.1, 0.2, 0.3)
    op = orc.opts(n_samples, bg=bg)
    tn, tf, hit = orc.ray_box(o, d)
    r = float(np.float32(raw)) + float(np.float32(shift))
    sigma = math.log1p(math.exp(r))
    sgm = 1 / (1 + math.exp(-r))
    s = 1 / (1 + math.exp(-float(np.float32(0.3))))
    for k in np.nonzero(hit)[0][:12]:
        L = float(n_samples * np.float32((tf[k] - tn[k]) / np.float32(n_samples)))
        g, _ = orc.render_backward(m, op, o[k:k + 1], d[k:k + 1], np.zeros((1, 3)), d_acc=np.ones(1))
        want = L * math.exp(-sigma * L) * sgm
        assert abs(g["density"].sum() - want) <= 1e-9 * max(1, abs(want))
        assert np.all(g["features"] == 0.0)
        g, _ = orc.render_backward(m, op, o[k:k + 1], d[k:k + 1], np.array([[1.0, 0.0, 0.0]]))
        want = (s - bg[0]) * L * math.exp(-sigma * L) * sgm
        assert abs(g["density"].sum() - want) <= 1e-9 * max(1, abs(want))
