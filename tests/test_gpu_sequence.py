"""GPU tests of render_sequence, the off-trajectory reference schedule
(Sec. III-C, Eq. 5-6): the overlapped two-stream schedule gives the same
bits as the serial one and as the single-frame entry points driven by hand,
and the whole sequence agrees with the oracle's schedule."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import Pair, cams, check_sparw_frame, compare, print_case, to_np
from oracle import sequence as seq

pytestmark = pytest.mark.gpu


def _trajectory(W, H, n, step_deg):
    poses = [synth.orbit_pose(k, step_deg=step_deg) for k in range(n)]
    pairs = [cams(W, H, p) for p in poses]
    return [g for g, _ in pairs], [synth.as_f32(p).reshape(3, 4) for p in poses]


def _assert_same(a, b):
    for x, y, name in zip(a[:4], b[:4], ("rgb", "depth", "mask", "n_masked")):
        assert torch.equal(torch.nan_to_num(x, posinf=-1.0), torch.nan_to_num(y, posinf=-1.0)), name
    assert a[4] == b[4]


@pytest.mark.parametrize("n,window", [(23, 5), (9, 16), (6, 1), (1, 4)])
def test_overlap_equals_serial_equals_single_calls(n, window):
    import paper_2404_11852_amd as cic
    print_case("sequence 96x96 n=%d window=%d" % (n, window))
    W = H = 96
    p = Pair(160, seed=0, mlp_seed=1, occupancy=True)
    gcams, poses = _trajectory(W, H, n, 2.0)
    opts = cic.make_opts(256, 1e-4, True)
    over = cic.render_sequence(p.gpu, opts, gcams, window, overlap=True)
    ser = cic.render_sequence(p.gpu, opts, gcams, window, overlap=False)
    part = cic.render_sequence(p.gpu, opts, gcams, window, overlap=True, target_cus_per_xcd=12)
    torch.cuda.synchronize()
    _assert_same(over, ser)
    _assert_same(part, ser)
    rgb, dz, mask, nm, refs = over
    n_win = (n - 1 + window - 1) // window
    assert len(refs) == max(n_win - 1, 0)
    # by hand: frame 0, references from the library's own pose extrapolation, sparse warps
    r0, d0, _ = cic.render_frame(p.gpu, opts, gcams[0])
    assert torch.equal(rgb[0], r0) and torch.equal(torch.nan_to_num(dz[0], posinf=-1), torch.nan_to_num(d0, posinf=-1))
    assert int(nm[0]) == W * H and int(mask[0].sum()) == W * H
    ref_cam, ref_rgb, ref_dz = gcams[0], r0, d0
    for w in range(n_win):
        s = 1 + w * window
        if w > 0:
            pose = cic.extrapolate_pose(poses[s - window - 1], poses[s - window], window / 2.0)
            assert pose == refs[w - 1]
            f, cx, cy = synth.intrinsics(W, H)
            ref_cam = cic.make_camera(W, H, f, cx, cy, pose)
            ref_rgb, ref_dz, _ = cic.render_frame(p.gpu, opts, ref_cam)
        for k in range(s, min(s + window, n)):
            T = torch.tensor(cic.relative_pose(list(ref_cam.c2w), poses[k]), dtype=torch.float32)
            r, d, m, c = cic.render_frame_sparw(p.gpu, opts, ref_cam, ref_rgb, ref_dz, gcams[k], T)
            assert torch.equal(rgb[k], r), k
            assert torch.equal(torch.nan_to_num(dz[k], posinf=-1), torch.nan_to_num(d, posinf=-1)), k
            assert torch.equal(mask[k], m) and int(nm[k]) == int(c.item()) == int(m.sum()), k


def test_sequence_matches_oracle():
    """Same trajectory through the oracle's schedule: the reference poses
    agree to float32 rounding.  Then every frame element by element: frame 0
    and the references are full renders (render tolerance, flip band
    apart); each target is checked against the oracle's warp and sparse
    render driven by the GPU's own float32 reference frame and the library's
    transform, so the hole mask and every warped pixel are bit-exact and the
    re-rendered pixels meet the render tolerance."""
    import paper_2404_11852_amd as cic
    print_case("sequence vs oracle 64x64 n=13 window=4")
    W = H = 64
    n, window = 13, 4
    p = Pair(160, seed=3, mlp_seed=4, occupancy=True)
    gcams, poses = _trajectory(W, H, n, 2.0)
    opts = cic.make_opts(256, 1e-4, True)
    rgb, dz, mask, nm, refs = cic.render_sequence(p.gpu, opts, gcams, window)
    f, cx, cy = synth.intrinsics(W, H)
    oop = oracle.opts(256, 1e-4, True)
    oposes = seq.reference_poses(poses, window)
    assert len(refs) == len(oposes) == 2
    for a, b in zip(refs, oposes):
        assert np.allclose(np.array(a), b.reshape(12), rtol=0, atol=2e-6)
    g_rgb, g_dz, g_mask = to_np(rgb), to_np(dz), to_np(mask)
    # frame 0: a full render, and reference R_0
    orgb0, _, _, diag = oracle.render_pixels(p.orc, oop, oracle.camera(W, H, f, cx, cy, poses[0].reshape(12)))
    compare(g_rgb[0], orgb0, margin=diag["margin"])
    ref_pose, ref_rgb, ref_dz = poses[0].reshape(12), g_rgb[0], g_dz[0]
    n_win = (n - 1 + window - 1) // window
    for w in range(n_win):
        if w > 0:
            ref_pose = np.array(refs[w - 1], np.float32)
            r, d, _ = cic.render_frame(p.gpu, opts, cic.make_camera(W, H, f, cx, cy, ref_pose))
            ref_rgb, ref_dz = to_np(r), to_np(d)
            orr, _, _, rdiag = oracle.render_pixels(p.orc, oop, oracle.camera(W, H, f, cx, cy, ref_pose))
            compare(ref_rgb, orr, margin=rdiag["margin"])
        ref_ocam = oracle.camera(W, H, f, cx, cy, ref_pose)
        for k in range(1 + w * window, min(1 + (w + 1) * window, n)):
            T = np.array(cic.relative_pose(list(ref_pose), poses[k]), np.float32)
            holes, _ = check_sparw_frame(g_rgb[k], g_dz[k], g_mask[k], p.orc, oop, ref_ocam, ref_rgb, ref_dz,
                                         oracle.camera(W, H, f, cx, cy, poses[k].reshape(12)), T)
            assert holes == int(nm[k]), k
            print("frame %d: %d holes, mask and warped pixels bit-exact" % (k, holes), flush=True)


def test_sequence_full_size_800():
    """800x800 frames, window 16: both schedules identical, per-frame counts
    consistent, the frame clock increasing, sampled pixels of frame 0 and of
    the first extrapolated reference R_1 against the oracle, and every target
    of window 1 (frames 17-32, warped from R_1) element by element against the
    oracle's warp driven by the GPU's R_1: hole mask and warped pixels
    bit-exact on the whole frame, 300 seeded hole pixels per target
    re-rendered by the oracle."""
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    print_case("sequence 800x800 n=34 window=16")
    W = H = 800
    n, window = 34, 16
    p = Pair(160, seed=0, mlp_seed=1, occupancy=True)
    gcams, poses = _trajectory(W, H, n, 1.0)
    opts = cic.make_opts(256, 1e-4, True)
    _lib.timing_enable(True)
    over = cic.render_sequence(p.gpu, opts, gcams, window, overlap=True)
    clock = _lib.timing_frames()
    _lib.timing_enable(False)
    ser = cic.render_sequence(p.gpu, opts, gcams, window, overlap=False)
    part = cic.render_sequence(p.gpu, opts, gcams, window, overlap=True, target_cus_per_xcd=20)
    torch.cuda.synchronize()
    _assert_same(over, ser)
    _assert_same(part, ser)
    assert len(clock) == n and all(b >= a for a, b in zip(clock, clock[1:]))
    rgb, dz, mask, nm, refs = over
    assert torch.equal(nm, mask.sum(dim=1).to(torch.int64))
    frac = (nm[1:].double() / (W * H)).cpu().numpy()
    assert 0.0 < frac.mean() < 0.5
    rng = np.random.default_rng(7)
    pix = np.sort(rng.choice(W * H, 400, replace=False))
    f, cx, cy = synth.intrinsics(W, H)
    oop = oracle.opts(256, 1e-4, True)
    orgb, _, _, diag = oracle.render_pixels(p.orc, oop, oracle.camera(W, H, f, cx, cy, poses[0].reshape(12)), pix)
    compare(to_np(rgb[0])[pix], orgb, margin=diag["margin"])
    # window 1: reference R_1 (extrapolated pose), rendered by the GPU as the sequence did
    ref_pose = np.array(refs[0], np.float32)
    r1, d1, _ = cic.render_frame(p.gpu, opts, cic.make_camera(W, H, f, cx, cy, ref_pose))
    r1, d1 = to_np(r1), to_np(d1)
    ref_ocam = oracle.camera(W, H, f, cx, cy, ref_pose)
    orr, _, _, rdiag = oracle.render_pixels(p.orc, oop, ref_ocam, pix)
    compare(r1[pix], orr, margin=rdiag["margin"])
    g_rgb, g_dz, g_mask = to_np(rgb), to_np(dz), to_np(mask)
    for k in range(1 + window, 1 + 2 * window):
        T = np.array(cic.relative_pose(list(ref_pose), poses[k]), np.float32)
        holes, checked = check_sparw_frame(g_rgb[k], g_dz[k], g_mask[k], p.orc, oop, ref_ocam, r1, d1,
                                           oracle.camera(W, H, f, cx, cy, poses[k].reshape(12)), T, sample=300,
                                           seed=k)
        assert holes == int(nm[k]) and checked > 0, k
        print("frame %d: %d holes (%d re-rendered by the oracle), mask and warped pixels bit-exact"
              % (k, holes, checked), flush=True)
