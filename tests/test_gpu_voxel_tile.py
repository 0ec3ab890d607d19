"""BF16 MLP in voxel order, where workgroups stage each brick's feature
vertices in LDS and gather every sample of the brick from there (the
memory-centric rendering of Sec. IV-A).  A sample's colour depends only on
its own inputs, and the compositing reads samples in ray order, so voxel
order must reproduce ray order bit for bit: the tests hold the tiled path to
exact equality with the ray-ordered one (whose parity with the oracle the
precision tests establish), for both grid storage types, on ragged sizes,
on rays with no live samples, on launches partitioned to a few CUs, and on
the full eight-view 800x800 workload."""
import numpy as np
import pytest
import torch

import synth
from helpers import cams, print_case

pytestmark = pytest.mark.gpu


def _model(res, storage, seed=0, mlp_seed=1):
    import paper_2404_11852_amd as cic
    dens, feats = synth.make_scene(res, seed=seed)
    mlp = synth.make_mlp(mlp_seed, bias_std=0.1)
    m = cic.Model(dens, feats, mlp, device="cuda", storage=storage, density_shift=synth.DENSITY_SHIFT,
                  compute=cic.CIC_BF16)
    m.build_occupancy(synth.OCC_SIGMA)
    return m


def _both_orders(m, n_samples, o, d, et=1e-4):
    import paper_2404_11852_amd as cic
    out = []
    for order in (cic.CIC_ORDER_RAY, cic.CIC_ORDER_VOXEL):
        n = torch.zeros(1, dtype=torch.int64, device="cuda")
        rgb, dt, acc = cic.render_rays(m, cic.make_opts(n_samples, et, True, order=order), o, d, n_eval=n)
        out.append((rgb, dt, acc, int(n.item())))
    torch.cuda.synchronize()
    return out


def _assert_equal(a, b):
    for x, y, name in zip(a[:3], b[:3], ("rgb", "depth", "acc")):
        assert torch.equal(torch.nan_to_num(x, posinf=-1.0), torch.nan_to_num(y, posinf=-1.0)), name
    assert a[3] == b[3]


@pytest.mark.parametrize("storage", [torch.float32, torch.float16])
@pytest.mark.parametrize("n_rays", [1, 7, 1000, 4099, 256 * 512 + 77])
def test_voxel_tiles_equal_ray_order_ragged(storage, n_rays):
    """Ragged ray counts through a 48^3 grid (6^3 bricks): segments of
    several bricks, partial last segments, bricks shared by workgroups.  The
    largest count takes the LDS-histogram compaction (blocks of 256 rays,
    used from 512 blocks up) with a ragged last block; the others take the
    per-run global counters."""
    print_case("voxel tiles vs ray order, 48^3, %d rays, %s" % (n_rays, storage))
    m = _model(48, storage)
    rng = np.random.default_rng(n_rays)
    o = rng.normal(0.0, 0.3, (n_rays, 3)) + np.array([0.0, 0.0, -3.0])
    d = np.array([0.0, 0.0, 1.0]) + rng.normal(0.0, 0.15, (n_rays, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = torch.tensor(o, dtype=torch.float32, device="cuda")
    d = torch.tensor(d, dtype=torch.float32, device="cuda")
    ray, vox = _both_orders(m, 192, o, d)
    _assert_equal(ray, vox)
    assert vox[3] > 0


def test_voxel_tiles_no_live_samples():
    """Rays that miss the grid: no segments at all; every workgroup must
    find its XCD's range empty and leave the background."""
    print_case("voxel tiles, rays missing the grid")
    m = _model(32, torch.float32)
    o = torch.tensor([[10.0, 10.0, 10.0]] * 50, dtype=torch.float32, device="cuda")
    d = torch.tensor([[0.0, 0.0, 1.0]] * 50, dtype=torch.float32, device="cuda")
    ray, vox = _both_orders(m, 64, o, d)
    _assert_equal(ray, vox)
    assert vox[3] == 0
    assert torch.equal(vox[0], torch.ones_like(vox[0]))


@pytest.mark.parametrize("storage", [torch.float32, torch.float16])
def test_voxel_tiles_full_size_eight_views(storage):
    """The eight-view 800x800 workload of the precision path, 160^3 grid."""
    import paper_2404_11852_amd as cic
    print_case("voxel tiles vs ray order, 8 x 800x800, %s" % storage)
    W = H = 800
    m = _model(160, storage)
    f, cx, cy = synth.intrinsics(W, H)
    rays = [cic.generate_rays(cic.make_camera(W, H, f, cx, cy, synth.as_f32(p))) for p in synth.sphere_poses(8, 2)]
    o = torch.cat([r[0] for r in rays]).contiguous()
    d = torch.cat([r[1] for r in rays]).contiguous()
    ray, vox = _both_orders(m, 256, o, d)
    _assert_equal(ray, vox)
    print("live samples %d" % vox[3])


@pytest.mark.parametrize("cus", [1, 3])
def test_voxel_tiles_partitioned_launch(cus):
    """render_sequence with the targets confined to a few CUs per XCD: the
    tiled MLP then runs on a grid of 8 * cus workgroups and must give the
    same frames as the serial schedule on the whole chip."""
    import paper_2404_11852_amd as cic
    print_case("voxel tiles, partitioned sequence, %d CUs per XCD" % cus)
    W = H = 96
    m = _model(64, torch.float16)
    gcams = [cams(W, H, synth.orbit_pose(k, step_deg=2.0))[0] for k in range(9)]
    opts = cic.make_opts(128, 1e-4, True, order=cic.CIC_ORDER_VOXEL)
    part = cic.render_sequence(m, opts, gcams, 4, overlap=True, target_cus_per_xcd=cus)
    ser = cic.render_sequence(m, opts, gcams, 4, overlap=False)
    ray = cic.render_sequence(m, cic.make_opts(128, 1e-4, True, order=cic.CIC_ORDER_RAY), gcams, 4, overlap=False)
    torch.cuda.synchronize()
    for a, b, c, name in zip(part[:4], ser[:4], ray[:4], ("rgb", "depth", "mask", "n_masked")):
        a, b, c = (torch.nan_to_num(t, posinf=-1.0) for t in (a, b, c))
        assert torch.equal(a, b), name
        assert torch.equal(b, c), name


def test_voxel_tiles_non_cubic_grid():
    """A 41 x 25 x 57 grid (partial last bricks of different sizes on each
    axis): the tiled BF16 path against ray order for both storage types."""
    import paper_2404_11852_amd as cic
    print_case("voxel tiles, 41x25x57 grid")
    dens, feats = synth.make_scene(64, seed=3)
    dens = np.ascontiguousarray(dens[:41, :25, :57])
    feats = np.ascontiguousarray(feats[:41, :25, :57])
    mlp = synth.make_mlp(2, bias_std=0.1)
    rng = np.random.default_rng(5)
    n = 20000
    o = rng.normal(0.0, 0.4, (n, 3)) + np.array([0.2, -0.1, -3.0])
    d = np.array([0.1, 0.05, 1.0]) + rng.normal(0.0, 0.2, (n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = torch.tensor(o, dtype=torch.float32, device="cuda")
    d = torch.tensor(d, dtype=torch.float32, device="cuda")
    for storage in (torch.float32, torch.float16):
        m = cic.Model(dens, feats, mlp, device="cuda", storage=storage, density_shift=synth.DENSITY_SHIFT,
                      compute=cic.CIC_BF16)
        m.build_occupancy(synth.OCC_SIGMA)
        ray, vox = _both_orders(m, 160, o, d)
        _assert_equal(ray, vox)
        assert vox[3] > 0
