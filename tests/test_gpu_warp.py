"""GPU parity of sparse radiance warping: warp_frame bit-exact against the
oracle (same float32 expression order, same tie rule), and
render_frame_sparw against the oracle's warp + sparse render + merge on the
same reference frame."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import Pair, cams, compare, print_case, to_np

pytestmark = pytest.mark.gpu


def _synthetic_ref(W, H, seed, void_frac=0.1):
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 1, (W * H, 3)).astype(np.float32)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    dep = (3.0 + 0.8 * np.sin(ii / 7.0) * np.cos(jj / 11.0) + 0.05 * rng.standard_normal((H, W))).astype(np.float32)
    dep = dep.reshape(-1)
    dep[rng.uniform(size=W * H) < void_frac] = np.inf
    return rgb, dep


def _T(ref_pose, tgt_pose):
    return synth.relative_pose(synth.as_f32(ref_pose), synth.as_f32(tgt_pose))


@pytest.mark.parametrize("W,H,step", [(64, 48, 1.0), (64, 48, 8.0), (800, 800, 1.0), (800, 800, 15.0)])
def test_warp_bit_exact(W, H, step):
    import paper_2404_11852_amd as cic
    print_case("warp %dx%d step %.0f" % (W, H, step))
    rgb, dep = _synthetic_ref(W, H, seed=int(step) + W)
    rp, tp = synth.orbit_pose(0), synth.orbit_pose(1, step_deg=step)
    gr, orr = cams(W, H, rp)
    gt, ot = cams(W, H, tp)
    T = _T(rp, tp)
    g = cic.warp_frame(gr, gt, torch.from_numpy(T), torch.from_numpy(rgb).cuda(), torch.from_numpy(dep).cuda(),
                       with_src=True)
    o = oracle.warp(orr, ot, T, rgb, dep)
    for a, b, name in zip(g, o, ("rgb", "depth", "mask", "src")):
        assert np.array_equal(to_np(a), b), name
    assert 0 < o[2].sum() < W * H


def test_warp_identity_and_translation():
    import paper_2404_11852_amd as cic
    print_case("warp identity/translation")
    W, H = 128, 96
    rgb, dep = _synthetic_ref(W, H, seed=1)
    gr, orr = cams(W, H, synth.orbit_pose(0))
    I = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    r, dz, m = cic.warp_frame(gr, gr, torch.from_numpy(I), torch.from_numpy(rgb).cuda(), torch.from_numpy(dep).cuda())
    assert int(m.sum()) == 0 and np.array_equal(to_np(r), rgb) and np.array_equal(to_np(dz), dep)
    T = I.copy()
    T[3], T[7], T[11] = 0.21, -0.13, 0.4
    g = cic.warp_frame(gr, gr, torch.from_numpy(T), torch.from_numpy(rgb).cuda(), torch.from_numpy(dep).cuda(),
                       with_src=True)
    o = oracle.warp(orr, orr, T, rgb, dep)
    for a, b in zip(g, o):
        assert np.array_equal(to_np(a), b)


def test_sparw_matches_oracle():
    """Same reference frame (rendered by the oracle) on both sides: mask and
    warped pixels bit-exact, re-rendered pixels within tolerance."""
    import paper_2404_11852_amd as cic
    print_case("sparw 96x96")
    W = H = 96
    p = Pair(160, seed=0, mlp_seed=1, occupancy=True)
    rp, tp = synth.orbit_pose(0), synth.orbit_pose(6)
    gr, orr = cams(W, H, rp)
    gt, ot = cams(W, H, tp)
    oop = oracle.opts(256, 1e-4, True)
    ref_rgb, ref_dz, _, _ = oracle.render_pixels(p.orc, oop, orr)
    ref_rgb32, ref_dz32 = ref_rgb.astype(np.float32), ref_dz.astype(np.float32)
    T = _T(rp, tp)
    go = cic.make_opts(256, 1e-4, True)
    n_eval = torch.zeros(1, dtype=torch.int64, device="cuda")
    rgb, dz, mask, nm = cic.render_frame_sparw(p.gpu, go, gr, torch.from_numpy(ref_rgb32).cuda(),
                                               torch.from_numpy(ref_dz32).cuda(), gt, torch.from_numpy(T),
                                               n_eval=n_eval)
    orgb, odz, omask, onm = oracle.sparw(p.orc, oop, orr, ref_rgb32, ref_dz32, ot, T)
    assert np.array_equal(to_np(mask), omask)
    assert int(nm.item()) == onm and onm > 0
    keep = omask == 0
    assert np.array_equal(to_np(rgb)[keep].astype(np.float64), orgb[keep])
    holes = np.nonzero(omask)[0]
    _, _, _, diag = oracle.render_pixels(p.orc, oop, ot, holes)
    compare(to_np(rgb)[holes], orgb[holes], margin=diag["margin"])
    assert int(n_eval.item()) > 0


def test_sparw_identity_renders_nothing_and_full_mask_renders_frame():
    import paper_2404_11852_amd as cic
    print_case("sparw limits")
    W = H = 64
    p = Pair(64, seed=1, occupancy=True)
    gc, oc = cams(W, H, synth.orbit_pose(3))
    go = cic.make_opts(128, 1e-4, True)
    ref_rgb, ref_dz, _ = cic.render_frame(p.gpu, go, gc)
    I = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    n_eval = torch.zeros(1, dtype=torch.int64, device="cuda")
    rgb, dz, mask, nm = cic.render_frame_sparw(p.gpu, go, gc, ref_rgb, ref_dz, gc, torch.from_numpy(I), n_eval=n_eval)
    assert int(nm.item()) == 0 and int(n_eval.item()) == 0
    assert torch.equal(rgb, ref_rgb)
    half_turn = I.copy()
    half_turn[0], half_turn[10] = -1.0, -1.0
    rgb, dz, mask, nm = cic.render_frame_sparw(p.gpu, go, gc, ref_rgb, ref_dz, gc, torch.from_numpy(half_turn))
    assert int(nm.item()) == W * H
    assert torch.equal(rgb, ref_rgb)
    assert torch.equal(torch.nan_to_num(dz, posinf=-1), torch.nan_to_num(ref_dz, posinf=-1))


@pytest.mark.parametrize("W,H,step,phi", [(64, 48, 8.0, 2.0), (800, 800, 6.0, 4.0), (800, 800, 15.0, 10.0)])
def test_warp_angle_threshold_bit_exact(W, H, step, phi):
    """Warp-angle test of Sec. III-C on: same float32 decision on both sides."""
    import paper_2404_11852_amd as cic
    print_case("warp angle %dx%d step %.0f phi %.1f" % (W, H, step, phi))
    rgb, dep = _synthetic_ref(W, H, seed=int(step) + 3 * W)
    rp, tp = synth.orbit_pose(0), synth.orbit_pose(1, step_deg=step)
    gr, orr = cams(W, H, rp)
    gt, ot = cams(W, H, tp)
    T = _T(rp, tp)
    g = cic.warp_frame(gr, gt, torch.from_numpy(T), torch.from_numpy(rgb).cuda(), torch.from_numpy(dep).cuda(),
                       with_src=True, max_angle_deg=phi)
    o = oracle.warp(orr, ot, T, rgb, dep, max_angle_deg=phi)
    for a, b, name in zip(g, o, ("rgb", "depth", "mask", "src")):
        assert np.array_equal(to_np(a), b), name
    # the threshold removes splats (more holes than without it) but not all of them
    o_off = oracle.warp(orr, ot, T, rgb, dep)
    assert o[2].sum() >= o_off[2].sum()
    assert o[2].sum() < W * H


def test_sparw_angle_threshold_matches_oracle():
    import paper_2404_11852_amd as cic
    print_case("sparw angle 96x96")
    W = H = 96
    p = Pair(160, seed=2, mlp_seed=3, occupancy=True)
    rp, tp = synth.orbit_pose(0), synth.orbit_pose(10)
    gr, orr = cams(W, H, rp)
    gt, ot = cams(W, H, tp)
    oop = oracle.opts(256, 1e-4, True, warp_max_angle=3.0)
    oop_off = oracle.opts(256, 1e-4, True)
    ref_rgb, ref_dz, _, _ = oracle.render_pixels(p.orc, oop, orr)
    ref_rgb32, ref_dz32 = ref_rgb.astype(np.float32), ref_dz.astype(np.float32)
    T = _T(rp, tp)
    go = cic.make_opts(256, 1e-4, True, warp_max_angle=3.0)
    rgb, dz, mask, nm = cic.render_frame_sparw(p.gpu, go, gr, torch.from_numpy(ref_rgb32).cuda(),
                                               torch.from_numpy(ref_dz32).cuda(), gt, torch.from_numpy(T))
    orgb, odz, omask, onm = oracle.sparw(p.orc, oop, orr, ref_rgb32, ref_dz32, ot, T)
    _, _, omask_off, onm_off = oracle.sparw(p.orc, oop_off, orr, ref_rgb32, ref_dz32, ot, T)
    assert onm > onm_off
    assert np.array_equal(to_np(mask), omask)
    assert int(nm.item()) == onm
    keep = omask == 0
    assert np.array_equal(to_np(rgb)[keep].astype(np.float64), orgb[keep])
    holes = np.nonzero(omask)[0]
    _, _, _, diag = oracle.render_pixels(p.orc, oop, ot, holes)
    compare(to_np(rgb)[holes], orgb[holes], margin=diag["margin"])
