"""GPU parity of the multi-level (hash-grid) encoding path (hierarchical
encodings, Sec. IV-A): rendering with the encoding against the oracle, in
ray and voxel order, float32 and float16 tables, all-hashed small tables,
and an 800x800 frame on sampled pixels."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import cams, compare, print_case, to_np

pytestmark = pytest.mark.gpu


class HashPair:
    def __init__(self, res=160, seed=0, mlp_seed=1, hres=synth.HASH_RES, log2_size=synth.HASH_LOG2_SIZE,
                 hseed=30, storage=torch.float32, occupancy=True, compute=None):
        import paper_2404_11852_amd as cic
        dens, _ = synth.make_scene(res, seed=seed)
        h = synth.make_hash_tables(hseed, res=hres, log2_size=log2_size)
        mlp = synth.make_mlp(mlp_seed)
        kw = {} if compute is None else {"compute": compute}
        self.gpu = cic.Model(dens, None, mlp, storage=storage, density_shift=synth.DENSITY_SHIFT, hash_enc=h, **kw)
        if storage == torch.float16:
            dens = dens.astype(np.float16).astype(np.float32)
            h = dict(h, tables=h["tables"].astype(np.float16).astype(np.float32))
        self.orc = oracle.Model(dens, None, mlp, density_shift=synth.DENSITY_SHIFT, hash_enc=h,
                                round_bf16=compute is not None)
        if occupancy:
            self.gpu.build_occupancy(synth.OCC_SIGMA)
            self.orc.set_occupancy(oracle.build_occupancy(self.orc, synth.OCC_SIGMA))


def _bf16_check(p, rgb, o, d, oop, what):
    """BF16 colours against the BF16-rounding oracle: per ray within 2e-5
    plus the colour change one bfloat16 rounding flip of one MLP input could
    cause (the oracle's flip diagnostic, weighted by compositing weight)."""
    orgb, _, _, diag = oracle.render_rays(p.orc, oop, o, d, flip=True)
    err = np.abs(to_np(rgb).astype(np.float64) - orgb).max(axis=1)
    flip = diag["flip"]
    print("%s: p99.5 %.2e max %.2e, flip bound median %.2e max %.2e"
          % (what, np.quantile(err, 0.995), err.max(), np.median(flip), flip.max()))
    assert np.quantile(err, 0.995) <= 2e-5
    assert np.all(err <= 2e-5 + flip), int(np.argmax(err - flip))


def _rays_check(p, n=4000, order=None, et=1e-4):
    import paper_2404_11852_amd as cic
    o, d = synth.random_rays(n, seed=8)
    kw = {} if order is None else {"order": order}
    go = cic.make_opts(256, et, True, **kw)
    rgb, dep, acc = cic.render_rays(p.gpu, go, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    orgb, odep, oacc, diag = oracle.render_rays(p.orc, oracle.opts(256, et, True), o, d, diagnostics=True)
    e1, nf = compare(to_np(rgb), orgb, margin=diag["margin"])
    compare(to_np(dep), odep, margin=diag["margin"], what="depth_t")
    compare(to_np(acc), oacc, margin=diag["margin"], what="acc")
    print("max err %.2e, flagged %d" % (e1, nf))
    return rgb, dep, acc


@pytest.mark.parametrize("storage", [torch.float32, torch.float16])
def test_hash_render_rays_matches_oracle(storage):
    import paper_2404_11852_amd as cic
    print_case("hash render_rays %s" % storage)
    p = HashPair(storage=storage)
    a = _rays_check(p)
    b = _rays_check(p, order=cic.CIC_ORDER_VOXEL)
    assert torch.equal(a[2], b[2]) and torch.equal(a[1], b[1])
    assert float((a[0] - b[0]).abs().max()) <= 2e-6


def test_hash_all_levels_hashed_small_table():
    print_case("hash render_rays, 2^12 tables")
    p = HashPair(res=64, hres=(24, 48, 96, 192), log2_size=12, hseed=31)
    _rays_check(p, n=2000)


def test_hash_frame_800_sampled():
    import paper_2404_11852_amd as cic
    print_case("hash frame 800x800")
    W = H = 800
    p = HashPair()
    pose = synth.orbit_pose(4)
    gc, oc = cams(W, H, pose)
    go = cic.make_opts(256, 1e-4, True)
    n_eval = torch.zeros(1, dtype=torch.int64, device="cuda")
    rgb, dz, acc = cic.render_frame(p.gpu, go, gc, n_eval=n_eval)
    pix = synth.pixel_subset(W, H, 1500, seed=9)
    orgb, odz, oacc, diag = oracle.render_pixels(p.orc, oracle.opts(256, 1e-4, True), oc, pix)
    compare(to_np(rgb)[pix], orgb, margin=diag["margin"])
    compare(to_np(acc)[pix], oacc, margin=diag["margin"], what="acc")
    assert int(n_eval.item()) > 10_000_000


def test_hash_bf16_against_bf16_oracle():
    import paper_2404_11852_amd as cic
    print_case("hash BF16 render_rays")
    p = HashPair(compute=cic.CIC_BF16)
    o, d = synth.random_rays(3000, seed=10)
    go = cic.make_opts(256, 0.0, True)
    rgb, _, _ = cic.render_rays(p.gpu, go, torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    _bf16_check(p, rgb, o, d, oracle.opts(256, 0.0, True), "bf16 hash")


@pytest.mark.parametrize("storage", [torch.float16, torch.float32])
def test_hash_bf16_voxel_levels_staged_equal_ray_order(storage):
    """BF16 voxel order stages each segment's boxes of level vertices in LDS
    (all four levels with 2^19 tables on the 160^3 grid: FP16 boxes always
    fit, FP32 boxes of the finest level only for segments that do not span
    their brick) and interpolates from there: the colours equal the ray-order
    gather bit for bit."""
    import paper_2404_11852_amd as cic
    print_case("hash BF16 voxel vs ray, %s tables" % storage)
    p = HashPair(storage=storage, compute=cic.CIC_BF16)
    o, d = synth.random_rays(30000, seed=12)
    o, d = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    a = cic.render_rays(p.gpu, cic.make_opts(256, 1e-4, True), o, d)
    b = cic.render_rays(p.gpu, cic.make_opts(256, 1e-4, True, order=cic.CIC_ORDER_VOXEL), o, d)
    for x, y, name in zip(a, b, ("rgb", "depth_t", "acc")):
        assert torch.equal(x, y), name


def test_hash_bf16_voxel_coarse_density_grid_falls_back():
    """A 32^3 density grid: a brick spans about 8, 17, 33 and 66 cells of
    the four levels, so the finer levels' boxes exceed the LDS and are
    gathered from the tables, the coarse one staged where the segment's
    samples use its vertices often enough; colours bit-exact with ray order,
    and against the BF16 oracle."""
    import paper_2404_11852_amd as cic
    print_case("hash BF16 voxel vs ray, 32^3 density grid")
    p = HashPair(res=32, compute=cic.CIC_BF16)
    o, d = synth.random_rays(6000, seed=13)
    go = cic.make_opts(256, 0.0, True)
    gv = cic.make_opts(256, 0.0, True, order=cic.CIC_ORDER_VOXEL)
    ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    a = cic.render_rays(p.gpu, go, ot, dt)
    b = cic.render_rays(p.gpu, gv, ot, dt)
    for x, y, name in zip(a, b, ("rgb", "depth_t", "acc")):
        assert torch.equal(x, y), name
    _bf16_check(p, b[0][:1500], o[:1500], d[:1500], oracle.opts(256, 0.0, True), "bf16 hash voxel")


def test_hash_bf16_voxel_extreme_levels_and_max_samples():
    """Degenerate and extreme levels: 1 and 2 cells per axis (one or two
    cells cover the box, every segment's box is the whole level) and 4096
    cells on 2^12-entry tables (every segment's box is far over the LDS and
    the level is gathered per sample), at the maximum 1024 samples per ray:
    voxel order equals ray order bit for bit and matches the BF16 oracle."""
    import paper_2404_11852_amd as cic
    print_case("hash BF16 voxel, levels (1, 2, 4096, 4096), N=1024")
    p = HashPair(res=64, hres=(1, 2, 4096, 4096), log2_size=12, hseed=32, compute=cic.CIC_BF16)
    o, d = synth.random_rays(3000, seed=14)
    ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    a = cic.render_rays(p.gpu, cic.make_opts(1024, 1e-4, True), ot, dt)
    b = cic.render_rays(p.gpu, cic.make_opts(1024, 1e-4, True, order=cic.CIC_ORDER_VOXEL), ot, dt)
    for x, y, name in zip(a, b, ("rgb", "depth_t", "acc")):
        assert torch.equal(x, y), name
    _bf16_check(p, b[0][:400], o[:400], d[:400], oracle.opts(1024, 1e-4, True), "bf16 hash extreme")


def test_hash_bf16_voxel_frame_800():
    """800x800 frame, FP16 tables + BF16 MLP: voxel order with staged level
    boxes equals ray order on every pixel."""
    import paper_2404_11852_amd as cic
    print_case("hash BF16 frame 800x800 voxel vs ray")
    p = HashPair(storage=torch.float16, compute=cic.CIC_BF16)
    gc, _ = cams(800, 800, synth.orbit_pose(2))
    a = cic.render_frame(p.gpu, cic.make_opts(256, 1e-4, True), gc)
    b = cic.render_frame(p.gpu, cic.make_opts(256, 1e-4, True, order=cic.CIC_ORDER_VOXEL), gc)
    assert torch.equal(a[0], b[0]) and torch.equal(a[2], b[2])
    assert torch.equal(torch.nan_to_num(a[1], posinf=-1), torch.nan_to_num(b[1], posinf=-1))


def test_hash_backward_rejected():
    import paper_2404_11852_amd as cic
    p = HashPair(res=32, occupancy=False)
    o, d = synth.random_rays(16, seed=1)
    with pytest.raises(cic.CicError):
        cic.render_backward(p.gpu, cic.make_opts(32), torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(),
                            torch.zeros(16, 3, device="cuda"))
