"""C interface checks that need no GPU: the library loads, exports every
function include/cicero.h declares, and rejects bad arguments with the
documented codes before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cicero.h")


@pytest.fixture(scope="module")
def L():
    from paper_2404_11852_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2404_11852_amd import build
        build.build()
    return _lib


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("render_rays", "render_frame", "warp_frame", "render_frame_sparw", "render_backward",
              "generate_rays", "build_occupancy", "cic_workspace_bytes", "cic_last_error_message"):
        assert n in names, n


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == _declared()


def _good(L):
    g = L.Grid((C.c_int32 * 3)(32, 32, 32), 12, L.CIC_F32, (C.c_float * 3)(-1.5, -1.5, -1.5),
               (C.c_float * 3)(1.5, 1.5, 1.5), -6.9, 0x1000, 0x2000, None)
    m = L.MLP(L.CIC_F32, 39, 128, 4, 0x3000, 0x3100, 0x3200, 0x3300, 0x3400, 0x3500)
    o = L.make_opts(64)
    return g, m, o


def test_hash_grid_validation(L):
    g, m, o = _good(L)
    g.features = None
    assert _render(L, g, m, o) == -1 and "features" in L.last_error()
    g.hash_levels = 3
    assert _render(L, g, m, o) == -1 and "hash_levels" in L.last_error()
    g.hash_levels = 4
    g.hash_res = (C.c_int32 * 4)(32, 64, 128, 0)
    assert _render(L, g, m, o) == -1 and "hash_res" in L.last_error()
    g.hash_res = (C.c_int32 * 4)(32, 64, 128, 256)
    g.hash_log2_size = 30
    assert _render(L, g, m, o) == -1 and "hash_log2_size" in L.last_error()
    g.hash_log2_size = 19
    assert _render(L, g, m, o) == -1 and "hash_tables" in L.last_error()
    g.hash_tables = 0x4002   # float16 entries are read as aligned 32-bit words
    assert _render(L, g, m, o) == -1 and "4-byte aligned" in L.last_error()


def test_feature_grid_alignment(L):
    g, m, o = _good(L)
    g.features = 0x2002
    assert _render(L, g, m, o) == -1 and "features must be 4-byte aligned" in L.last_error()


def _render(L, g, m, o, n=16, ws=0x9000, ws_bytes=None):
    lib = L.lib()
    if ws_bytes is None:
        ws_bytes = L.workspace_bytes(L.OP_RENDER_RAYS, n, g, o)
    p = C.c_void_p(0x5000)
    return lib.render_rays(C.byref(g) if g is not None else None, C.byref(m) if m is not None else None,
                           C.byref(o) if o is not None else None, C.c_int64(n), p, p, p, p, p, None,
                           C.c_void_p(ws) if ws else None, C.c_size_t(ws_bytes), None)


def test_invalid_arguments_are_rejected_before_launch(L):
    g, m, o = _good(L)
    assert _render(L, None, m, o) == -1
    assert "grid" in L.last_error()
    assert _render(L, g, None, o) == -1
    assert _render(L, g, m, None) == -1
    bad = L.make_opts(0)
    assert _render(L, g, m, bad) == -1 and "n_samples" in L.last_error()
    bad = L.make_opts(2048)
    assert _render(L, g, m, bad) == -1
    bad = L.make_opts(64, use_occupancy=True)   # grid has no occupancy
    assert _render(L, g, m, bad) == -1 and "occupancy" in L.last_error()
    bad = L.make_opts(64, order=7)
    assert _render(L, g, m, bad) == -1
    bad = L.make_opts(64, et_threshold=-1.0)
    assert _render(L, g, m, bad) == -1
    g2, _, _ = _good(L)
    g2.n_feat = 8
    assert _render(L, g2, m, o) == -1 and "n_feat" in L.last_error()
    g3, _, _ = _good(L)
    g3.res[1] = 1
    assert _render(L, g3, m, o) == -1
    g4, _, _ = _good(L)
    g4.box_hi[0] = -2.0
    assert _render(L, g4, m, o) == -1
    m2 = L.MLP(L.CIC_F32, 40, 128, 4, 1, 1, 1, 1, 1, 1)
    assert _render(L, g, m2, o) == -1
    # workspace too small
    assert _render(L, g, m, o, ws_bytes=16) == -2 and "workspace" in L.last_error()
    # n = 0 is a successful no-op
    assert _render(L, g, m, o, n=0, ws=0, ws_bytes=0) == 0
    assert _render(L, g, m, o, n=-1) == -1


def test_camera_and_warp_validation(L):
    lib = L.lib()
    cam = L.make_camera(64, 64, 80.0, 32.0, 32.0, [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 4])
    bad = L.make_camera(0, 64, 80.0, 32.0, 32.0, [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 4])
    T = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    p = C.c_void_p(0x5000)
    rc = lib.warp_frame(C.byref(bad), C.byref(cam), T, p, p, C.c_float(0), p, p, p, None, p, C.c_size_t(1 << 30), None)
    assert rc == -1 and "camera" in L.last_error()
    rc = lib.warp_frame(C.byref(cam), C.byref(cam), None, p, p, C.c_float(0), p, p, p, None, p, C.c_size_t(1 << 30), None)
    assert rc == -1
    rc = lib.warp_frame(C.byref(cam), C.byref(cam), T, p, p, C.c_float(0), p, p, p, None, p, C.c_size_t(8), None)
    assert rc == -2
    Tn = (C.c_float * 12)(1, 0, 0, float("nan"), 0, 1, 0, 0, 0, 0, 1, 0)
    rc = lib.warp_frame(C.byref(cam), C.byref(cam), Tn, p, p, C.c_float(0), p, p, p, None, p, C.c_size_t(1 << 30), None)
    assert rc == -1
    rc = lib.warp_frame(C.byref(cam), C.byref(cam), T, p, p, C.c_float(-5), p, p, p, None, p, C.c_size_t(1 << 30), None)
    assert rc == -1 and "max_angle" in L.last_error()
    rc = lib.generate_rays(C.byref(cam), C.c_int64(5), None, p, p, None)
    assert rc == -1 and "width*height" in L.last_error()


def test_workspace_sizes(L):
    g, m, o = _good(L)
    a = L.workspace_bytes(L.OP_RENDER_RAYS, 1000, g, o)
    b = L.workspace_bytes(L.OP_RENDER_RAYS, 2000, g, o)
    assert 0 < a < b
    # bounded by the per-pass chunk of rays
    c = L.workspace_bytes(L.OP_RENDER_RAYS, 1 << 21, g, o)
    d = L.workspace_bytes(L.OP_RENDER_RAYS, 1 << 23, g, o)
    assert c == d
    ov = L.make_opts(64, order=L.CIC_ORDER_VOXEL)
    assert L.workspace_bytes(L.OP_RENDER_RAYS, 1000, g, ov) > a
    assert L.workspace_bytes(L.OP_WARP_FRAME, 640000) >= 8 * 640000
    assert L.workspace_bytes(L.OP_RENDER_RAYS, -1, g, o) == 0
    assert L.workspace_bytes(99, 10, g, o) == 0


def test_smaller_workspace_runs_more_passes(L):
    """render_rays takes any workspace from the one-ray size up (fewer rays
    per pass); below it the call fails before launching anything."""
    g, m, o = _good(L)
    one = L.workspace_bytes(L.OP_RENDER_RAYS, 1, g, o)
    full = L.workspace_bytes(L.OP_RENDER_RAYS, 5000, g, o)
    assert one < full
    assert _render(L, g, m, o, n=5000, ws_bytes=one - 1) == -2
    msg = L.last_error()
    assert "need at least %d bytes" % one in msg and "%d for the fewest passes" % full in msg
    # slots shared with the colours (ray order) or the sample order (voxel order)
    ov = L.make_opts(64, order=L.CIC_ORDER_VOXEL)
    per_ray = (L.workspace_bytes(L.OP_RENDER_RAYS, 4001, g, o) - L.workspace_bytes(L.OP_RENDER_RAYS, 1, g, o)) / 4000
    per_ray_v = (L.workspace_bytes(L.OP_RENDER_RAYS, 4001, g, ov) - L.workspace_bytes(L.OP_RENDER_RAYS, 1, g, ov)) / 4000
    assert abs(per_ray - (64 * 22 + 600)) < 2 and abs(per_ray_v - (64 * 32 + 600)) < 2


def test_product_has_no_cpu_fallback():
    """The package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2404_11852_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn
                assert "orc_" not in txt, fn
