"""The allocation-free warp (warp_frame_noalloc, z-buffer in the library's
own device array) through the C ABI against warp_frame with a workspace:
the same colours, depths, masks and source indices bit for bit, on two calls
in a row with the second target smaller, and targets above the array's size
refused on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from helpers import Pair, cams, print_case

pytestmark = pytest.mark.gpu


def _frame(p, W, H, pose):
    import paper_2404_11852_amd as cic
    gc, _ = cams(W, H, pose)
    rgb, dz, _ = cic.render_frame(p.gpu, cic.make_opts(128, 1e-4, True), gc)
    return gc, rgb, dz


def _both(ref_cam, ref_rgb, ref_dz, tgt_cam, T, angle):
    """warp_frame (workspace) and warp_frame_noalloc on the same inputs."""
    from paper_2404_11852_amd import _lib
    n = tgt_cam.width * tgt_cam.height
    outs = []
    for noalloc in (False, True):
        rgb = torch.full((n, 3), -7.0, device="cuda")
        dz = torch.full((n,), -7.0, device="cuda")
        mask = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
        src = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        if noalloc:
            Tc = (C.c_float * 12)(*[float(v) for v in np.asarray(T, np.float32).reshape(12)])
            rc = _lib.lib().warp_frame_noalloc(C.byref(ref_cam), C.byref(tgt_cam), Tc, _lib._ptr(ref_rgb),
                                               _lib._ptr(ref_dz), C.c_float(angle), _lib._ptr(rgb), _lib._ptr(dz),
                                               _lib._ptr(mask), _lib._ptr(src), _lib._stream())
            assert rc == 0, _lib.last_error()
        else:
            _lib.warp_frame(ref_cam, tgt_cam, torch.from_numpy(np.asarray(T, np.float32)), ref_rgb, ref_dz, rgb, dz,
                            mask, src, angle)
        outs.append((rgb, dz, mask, src))
    torch.cuda.synchronize()
    return outs


def _same(a, b):
    for x, y, name in zip(a, b, ("rgb", "depth", "mask", "src")):
        assert torch.equal(torch.nan_to_num(x, posinf=-1.0), torch.nan_to_num(y, posinf=-1.0)), name


def test_noalloc_warp_equals_workspace_warp():
    print_case("warp_frame_noalloc 800x800 then 160x120")
    p = Pair(160, seed=0, mlp_seed=1, occupancy=True)
    # first call: 800x800, orbit frames 0 -> 9, with the angle test
    rc, rrgb, rdz = _frame(p, 800, 800, synth.orbit_pose(0))
    tc, _ = cams(800, 800, synth.orbit_pose(9))
    T = synth.relative_pose(synth.as_f32(synth.orbit_pose(0)), synth.as_f32(synth.orbit_pose(9)))
    ws, na = _both(rc, rrgb, rdz, tc, T, 6.0)
    _same(ws, na)
    assert 0 < int(na[2].sum()) < 800 * 800
    # second call, smaller: 160x120 from another reference; every pixel is
    # written again, so nothing of the first call shows through
    rc2, rrgb2, rdz2 = _frame(p, 160, 120, synth.orbit_pose(20))
    tc2, _ = cams(160, 120, synth.orbit_pose(24))
    T2 = synth.relative_pose(synth.as_f32(synth.orbit_pose(20)), synth.as_f32(synth.orbit_pose(24)))
    ws2, na2 = _both(rc2, rrgb2, rdz2, tc2, T2, 0.0)
    _same(ws2, na2)
    assert 0 < int(na2[2].sum()) < 160 * 120


def test_noalloc_warp_refuses_oversized_targets():
    import paper_2404_11852_amd as cic
    from paper_2404_11852_amd import _lib
    print_case("warp_frame_noalloc size limit")
    f, cx, cy = synth.intrinsics(2048, 1025)
    big = cic.make_camera(2048, 1025, f, cx, cy, synth.as_f32(synth.orbit_pose(0)))
    small = cic.make_camera(8, 8, f, 4.0, 4.0, synth.as_f32(synth.orbit_pose(0)))
    t = torch.zeros(4, device="cuda")
    with pytest.raises(_lib.CicError) as e:
        _lib.warp_frame_noalloc(small, big, np.eye(3, 4, dtype=np.float32), t, t, t, t, t)
    assert e.value.code == -1 and "at most 2097152" in str(e.value)
