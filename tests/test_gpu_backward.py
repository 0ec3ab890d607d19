"""GPU adjoint (render_backward) against the oracle's float64 adjoint: per
tensor, ||g_gpu - g_oracle|| / ||g_oracle|| <= 1e-4, on a small case, on a
pass of several chunks with densely sampled bricks, and on the full
training-step size (160^3 grids, 8192 rays x 256 samples)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import Pair, print_case, to_np

pytestmark = pytest.mark.gpu

NAMES = ("density", "features", "w0", "b0", "w1", "b1", "w2", "b2")


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / max(nb, 1e-300)


def _training_rays(cfg_views=8, W=800, H=800, n=8192, pose_seed=3, ray_seed=12):
    poses = synth.sphere_poses(cfg_views, seed=pose_seed)
    view, pix = synth.training_pixels(cfg_views, W, H, n, seed=ray_seed)
    f, cx, cy = synth.intrinsics(W, H)
    o = np.empty((n, 3), np.float32)
    d = np.empty((n, 3), np.float32)
    for v in range(cfg_views):
        sel = np.nonzero(view == v)[0]
        oc = oracle.camera(W, H, f, cx, cy, synth.as_f32(poses[v]))
        oo, dd = oracle.generate_rays(oc, pix[sel])
        o[sel], d[sel] = oo, dd
    return o, d


def _run(p, n_samples, et, o, d, gt, with_depth=False):
    import paper_2404_11852_amd as cic
    op = oracle.opts(n_samples, et)
    rgb, dep, acc = oracle.render_rays(p.orc, op, o, d)
    d_rgb = (2.0 * (rgb - gt) / rgb.size).astype(np.float32)
    d_dep = (np.linspace(-1e-3, 1e-3, len(o))).astype(np.float32) if with_depth else None
    d_acc = (np.linspace(2e-3, -1e-3, len(o))).astype(np.float32) if with_depth else None
    go = cic.make_opts(n_samples, et)
    g = cic.render_backward(p.gpu, go, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(),
                            torch.from_numpy(d_rgb).cuda(),
                            None if d_dep is None else torch.from_numpy(d_dep).cuda(),
                            None if d_acc is None else torch.from_numpy(d_acc).cuda())
    torch.cuda.synchronize()
    og, _ = oracle.render_backward(p.orc, op, o, d, d_rgb.astype(np.float64),
                                   None if d_dep is None else d_dep.astype(np.float64),
                                   None if d_acc is None else d_acc.astype(np.float64))
    return g, og


def test_backward_small_matches_oracle():
    print_case("backward small 24^3, 700 rays, N=64")
    p = Pair(24, seed=4, mlp_seed=5, bias_std=0.1)
    o, d = synth.random_rays(700, seed=9)
    gt = np.random.default_rng(1).uniform(0, 1, (700, 3))
    g, og = _run(p, 64, 0.0, o, d, gt, with_depth=True)
    for k in NAMES:
        r = _rel(to_np(g[k]), og[k])
        print("%s rel %.2e" % (k, r))
        assert r <= 1e-4, (k, r)


def test_backward_multichunk_dense_bricks():
    """18000 parallel rays through a narrow beam of a 24^3 grid: three chunks
    of the pass (8192 rays each at most), gradients accumulated across them,
    and a few bricks holding thousands of samples each, so every such brick
    is cut into several segments whose tiles the vertex gather adds up."""
    print_case("backward 24^3, 18000 beam rays, N=128")
    p = Pair(24, seed=6, mlp_seed=8, bias_std=0.1)
    n = 18000
    rng = np.random.default_rng(21)
    o = np.zeros((n, 3), np.float32)
    o[:, 0] = rng.uniform(-0.3, 0.3, n)
    o[:, 1] = rng.uniform(-0.3, 0.3, n)
    o[:, 2] = -3.0
    d = np.tile(np.array([[0.05, -0.03, 1.0]], np.float32), (n, 1))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    gt = rng.uniform(0, 1, (n, 3))
    g, og = _run(p, 128, 0.0, o, d, gt, with_depth=True)
    for k in NAMES:
        r = _rel(to_np(g[k]), og[k])
        print("%s rel %.2e" % (k, r))
        assert r <= 1e-4, (k, r)


def test_backward_non_cubic_grid():
    """A 41 x 25 x 57 grid: bricks cut short differently on each axis, so the
    owned vertex ranges and the tiles of the last bricks differ per axis."""
    print_case("backward 41x25x57, 3000 rays, N=96")
    dens, feats = synth.make_scene(64, seed=3)
    dens = np.ascontiguousarray(dens[:41, :25, :57])
    feats = np.ascontiguousarray(feats[:41, :25, :57])
    p = Pair(0, dens=dens, feats=feats, mlp=synth.make_mlp(2, bias_std=0.1))
    o, d = synth.random_rays(3000, seed=14)
    gt = np.random.default_rng(4).uniform(0, 1, (3000, 3))
    g, og = _run(p, 96, 0.0, o, d, gt, with_depth=True)
    for k in NAMES:
        r = _rel(to_np(g[k]), og[k])
        print("%s rel %.2e" % (k, r))
        assert r <= 1e-4, (k, r)


def test_backward_full_size_training_step():
    """One MSE step: GT from the seed-10 scene rendered by the oracle, model
    grids N(0, 0.01) (seed 11), MLP seed 21, 8192 rays from 8 views,
    256 samples, termination at 1e-4."""
    print_case("backward full size 160^3, 8192 rays, N=256")
    cfg = synth.get_config("train8192_views8")
    ex = cfg.extra
    o, d = _training_rays()
    gd, gf = synth.make_scene(160, seed=ex["gt_scene_seed"])
    gt_model = oracle.Model(gd, gf, synth.make_mlp(ex["gt_mlp_seed"]), density_shift=synth.DENSITY_SHIFT)
    gt, _, _ = oracle.render_rays(gt_model, oracle.opts(256, 1e-4), o, d)
    md, mf = synth.make_model_grid(160, seed=ex["model_grid_seed"])
    p = Pair(160, dens=md, feats=mf, mlp=synth.make_mlp(ex["model_mlp_seed"]))
    g, og = _run(p, 256, 1e-4, o, d, gt)
    for k in NAMES:
        r = _rel(to_np(g[k]), og[k])
        print("%s rel %.2e" % (k, r))
        assert r <= 1e-4, (k, r)


def test_autograd_function_matches_direct_call():
    import paper_2404_11852_amd as cic
    print_case("autograd wrapper")
    p = Pair(16, seed=6, mlp_seed=7)
    o, d = synth.random_rays(300, seed=10)
    to_, td = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    go = cic.make_opts(48)
    params = [p.gpu.density, p.gpu.features] + [p.gpu.w[k] for k in ("w0", "b0", "w1", "b1", "w2", "b2")]
    leaves = [t.detach().clone().requires_grad_(True) for t in params]
    rgb, dep, acc = cic.RenderRays.apply(*leaves, to_, td, p.gpu, go)
    target = torch.rand_like(rgb)
    loss = ((rgb - target) ** 2).mean() + 0.1 * acc.sum()
    loss.backward()
    d_rgb = (2.0 * (rgb.detach() - target) / rgb.numel()).contiguous()
    d_acc = torch.full_like(acc, 0.1)
    g = cic.render_backward(p.gpu, go, to_, td, d_rgb, None, d_acc)
    for leaf, k in zip(leaves, NAMES):
        ref = g[k]
        assert torch.allclose(leaf.grad, ref, rtol=1e-5, atol=1e-7 * float(ref.abs().max()) + 1e-12), k


def test_autograd_function_uses_the_leaves_it_is_given():
    """RenderRays renders with the tensors passed in, not the model's own
    copies: after an SGD step on the leaves, the next forward equals a plain
    render of a model holding the updated values (same bits), its gradients
    equal render_backward on that model, and a leaf modified in place
    between forward and backward is refused."""
    import paper_2404_11852_amd as cic
    print_case("autograd leaves updated between calls")
    p = Pair(16, seed=6, mlp_seed=7, bias_std=0.1)
    o, d = synth.random_rays(400, seed=11)
    to_, td = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    go = cic.make_opts(48)
    params = [p.gpu.density, p.gpu.features] + [p.gpu.w[k] for k in ("w0", "b0", "w1", "b1", "w2", "b2")]
    leaves = [t.detach().clone().requires_grad_(True) for t in params]
    target = torch.rand((400, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    rgb0, _, _ = cic.RenderRays.apply(*leaves, to_, td, p.gpu, go)
    ((rgb0 - target) ** 2).mean().backward()
    with torch.no_grad():
        for t in leaves:
            t -= 50.0 * t.grad
            t.grad = None
    rgb1, dep1, acc1 = cic.RenderRays.apply(*leaves, to_, td, p.gpu, go)
    assert float((rgb1 - rgb0).detach().abs().max()) > 1e-4      # the step changed the image
    fresh = cic.Model(leaves[0].detach().cpu().numpy(), leaves[1].detach().cpu().numpy(),
                      {k: leaves[2 + i].detach().cpu().numpy() for i, k in enumerate(NAMES[2:])},
                      device="cuda", density_shift=synth.DENSITY_SHIFT)
    ref_rgb, ref_dep, ref_acc = cic.render_rays(fresh, go, to_, td)
    assert torch.equal(rgb1, ref_rgb) and torch.equal(dep1, ref_dep) and torch.equal(acc1, ref_acc)
    loss = ((rgb1 - target) ** 2).mean()
    loss.backward()
    d_rgb = (2.0 * (rgb1.detach() - target) / rgb1.numel()).contiguous()
    g = cic.render_backward(fresh, go, to_, td, d_rgb)
    for leaf, k in zip(leaves, NAMES):
        ref = g[k]
        assert torch.allclose(leaf.grad, ref, rtol=1e-5, atol=1e-7 * float(ref.abs().max()) + 1e-12), k
    rgb2, _, _ = cic.RenderRays.apply(*leaves, to_, td, p.gpu, go)
    with torch.no_grad():
        leaves[3].add_(1.0)
    with pytest.raises(RuntimeError):
        ((rgb2 - target) ** 2).mean().backward()


def test_backward_degenerate_inputs():
    """No rays, and rays that all miss the grid (no live samples, so no brick
    segments): the accumulated gradients stay exactly zero; a zero upstream
    gradient on rays that hit gives zero gradients too."""
    import paper_2404_11852_amd as cic
    print_case("backward degenerate inputs")
    p = Pair(24, seed=4, mlp_seed=5, bias_std=0.1)
    go = cic.make_opts(64)
    z = torch.empty((0, 3), device="cuda")
    g = cic.render_backward(p.gpu, go, z, z, z)
    torch.cuda.synchronize()
    assert all(float(v.abs().max()) == 0.0 for v in g.values() if v.numel())
    o = torch.tensor([[5.0, 5.0, 5.0]] * 40, device="cuda")
    d = torch.tensor([[1.0, 0.0, 0.0]] * 40, device="cuda")
    g = cic.render_backward(p.gpu, go, o, d, torch.ones((40, 3), device="cuda"))
    torch.cuda.synchronize()
    assert all(float(v.abs().max()) == 0.0 for v in g.values())
    o2, d2 = synth.random_rays(100, seed=3)
    g = cic.render_backward(p.gpu, go, torch.from_numpy(o2).cuda(), torch.from_numpy(d2).cuda(),
                            torch.zeros((100, 3), device="cuda"))
    torch.cuda.synchronize()
    assert all(float(v.abs().max()) == 0.0 for v in g.values())


def test_backward_repeat_mlp_gradients_same_bits():
    """Two identical calls on a beam of 12000 rays through a 24^3 grid (bricks
    cut into several segments): the MLP gradients are fixed-order sums, so
    they are the same bits; the grid gradients follow the bucketing's atomic
    order and agree to float32 rounding (measured 4e-7 and 6e-7 relative;
    bound 1e-5)."""
    import paper_2404_11852_amd as cic
    print_case("backward repeat, 24^3, 12000 beam rays, N=96")
    p = Pair(24, seed=6, mlp_seed=8, bias_std=0.1)
    n = 12000
    rng = np.random.default_rng(31)
    o = np.zeros((n, 3), np.float32)
    o[:, 0] = rng.uniform(-0.4, 0.4, n)
    o[:, 1] = rng.uniform(-0.4, 0.4, n)
    o[:, 2] = -3.0
    d = np.tile(np.array([[0.04, 0.02, 1.0]], np.float32), (n, 1))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d_rgb = torch.from_numpy(rng.normal(0, 1e-3, (n, 3)).astype(np.float32)).cuda()
    go = cic.make_opts(96, 0.0)
    ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    g1 = cic.render_backward(p.gpu, go, ot, dt, d_rgb)
    g2 = cic.render_backward(p.gpu, go, ot, dt, d_rgb)
    torch.cuda.synchronize()
    for k in ("w0", "b0", "w1", "b1", "w2", "b2"):
        assert torch.equal(g1[k], g2[k]), k
        assert torch.count_nonzero(g1[k]) > 0, k
    for k in ("density", "features"):
        r = _rel(to_np(g2[k]), to_np(g1[k]))
        print("%s repeat rel %.2e" % (k, r))
        assert r <= 1e-5, (k, r)
