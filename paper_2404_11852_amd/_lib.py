"""ctypes binding of libcicero.so (argument marshalling only).

Every function takes torch CUDA tensors, passes their device pointers and the
current HIP stream to the C entry point of the same name, and raises on a
non-zero return code.  No arithmetic of the method happens here; there is no
CPU fallback: if the library is missing or the device is not gfx950 the
calls raise.
"""
import atexit
import ctypes as C
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcicero.so")

CIC_F32, CIC_F16, CIC_BF16 = 0, 1, 2
CIC_ORDER_RAY, CIC_ORDER_VOXEL = 0, 1
(OP_RENDER_RAYS, OP_RENDER_FRAME, OP_WARP_FRAME, OP_RENDER_FRAME_SPARW, OP_RENDER_BACKWARD,
 OP_RENDER_SEQUENCE, OP_RENDER_FRAME_DS) = range(7)
CIC_SEQ_OVERLAP, CIC_SEQ_TEMPORAL = 1, 2


class CicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("cicero error %d: %s" % (code, msg))
        self.code = code


class Grid(C.Structure):
    _fields_ = [("res", C.c_int32 * 3), ("n_feat", C.c_int32), ("storage", C.c_int32),
                ("box_lo", C.c_float * 3), ("box_hi", C.c_float * 3), ("density_shift", C.c_float),
                ("density", C.c_void_p), ("features", C.c_void_p), ("occupancy", C.c_void_p),
                ("hash_levels", C.c_int32), ("hash_res", C.c_int32 * 4), ("hash_log2_size", C.c_int32),
                ("hash_tables", C.c_void_p)]


class MLP(C.Structure):
    _fields_ = [("compute", C.c_int32), ("in_dim", C.c_int32), ("hidden", C.c_int32), ("pe_freqs", C.c_int32),
                ("w0", C.c_void_p), ("b0", C.c_void_p), ("w1", C.c_void_p), ("b1", C.c_void_p),
                ("w2", C.c_void_p), ("b2", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("et_threshold", C.c_float), ("use_occupancy", C.c_int32),
                ("bg", C.c_float * 3), ("void_acc", C.c_float), ("order", C.c_int32),
                ("warp_max_angle", C.c_float)]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("f", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("c2w", C.c_float * 12)]


EXPORTS = ["cic_workspace_bytes", "cic_last_error_message", "build_occupancy", "generate_rays", "render_rays",
           "render_frame", "warp_frame", "render_frame_sparw", "render_backward", "cic_timing_enable",
           "cic_timing_read", "cic_extrapolate_pose", "cic_relative_pose", "render_sequence", "cic_timing_frames",
           "render_frame_ds", "cic_stream_create_cu_masked", "cic_stream_destroy", "warp_frame_noalloc"]
STAGES = ["march", "compact", "mlp", "reduce", "warp", "raygen", "bwd_composite", "bwd_mlp", "bwd_wgrad", "embed"]

_lib = None
_lock = threading.Lock()


def lib():
    """Load libcicero.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise CicError(-3, "libcicero.so not built (run __graft_entry__.build())")
                L = C.CDLL(LIB_PATH)
                vp, i64, f, u64 = C.c_void_p, C.c_int64, C.c_float, C.c_size_t
                L.cic_workspace_bytes.restype = u64
                L.cic_workspace_bytes.argtypes = [C.c_int, i64, vp, vp]
                L.cic_last_error_message.restype = C.c_char_p
                L.cic_last_error_message.argtypes = []
                L.build_occupancy.argtypes = [vp, f, vp, vp]
                L.generate_rays.argtypes = [vp, i64, vp, vp, vp, vp]
                L.render_rays.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, u64, vp]
                L.render_frame.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, u64, vp]
                L.warp_frame.argtypes = [vp, vp, vp, vp, vp, f, vp, vp, vp, vp, vp, u64, vp]
                L.render_frame_sparw.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, u64, vp]
                L.render_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                              vp, vp, u64, vp]
                L.cic_timing_enable.argtypes = [C.c_int]
                L.cic_timing_read.argtypes = [vp, vp, C.c_int]
                L.cic_extrapolate_pose.argtypes = [vp, vp, f, vp]
                L.cic_relative_pose.argtypes = [vp, vp, vp]
                L.render_sequence.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, f, C.c_int32, C.c_int32, vp,
                                              vp, vp, vp, vp, vp, vp, u64, vp, vp]
                L.cic_stream_create_cu_masked.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
                L.cic_stream_destroy.argtypes = [vp]
                L.warp_frame_noalloc.argtypes = [vp, vp, vp, vp, vp, f, vp, vp, vp, vp, vp]
                L.cic_timing_frames.argtypes = [vp, C.c_int]
                L.render_frame_ds.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, u64, vp]
                for name in EXPORTS[2:]:
                    getattr(L, name).restype = C.c_int
                _lib = L
                atexit.register(release)
    return _lib


def release():
    """Destroy every HIP object the binding holds for the library: the
    CU-partitioned stream pairs and the timing events.  Registered to run at
    interpreter exit, while the HIP runtime is still up; safe to call
    again."""
    if _lib is None:
        return
    with _lock:
        pairs = list(_cu_streams.items())
        _cu_streams.clear()
    for (dev, _t), (s_tgt, s_ref) in pairs:
        with torch.cuda.device(dev):
            _lib.cic_stream_destroy(s_tgt)
            _lib.cic_stream_destroy(s_ref)
    _lib.cic_timing_enable(0)


def last_error():
    return lib().cic_last_error_message().decode()


def _check(rc):
    if rc != 0:
        raise CicError(rc, last_error())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# workspace: one growing byte buffer per device, reused across calls that run
# on the same stream (calls sharing it must not overlap)
# ---------------------------------------------------------------------------
_ws = {}


def workspace(nbytes, device):
    key = torch.device(device).index or 0
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws[key] = None
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws[key] = buf
    return buf


def free_workspace():
    _ws.clear()


# Upper bound on the workspace of render_rays, render_frame and
# render_backward (None: the size for the fewest passes); the library then
# runs the rays in as many passes as the bound needs.
_ws_limit = [None]


def set_workspace_limit(nbytes=None):
    _ws_limit[0] = None if nbytes is None else int(nbytes)


def _pass_workspace(op, n, grid, opts, device):
    nb = workspace_bytes(op, n, grid, opts)
    if _ws_limit[0] is not None:
        nb = min(nb, _ws_limit[0])
    ws = workspace(nb, device)
    return ws, nb


# ---------------------------------------------------------------------------
# struct builders
# ---------------------------------------------------------------------------
def make_grid(density, features, occupancy=None, box_lo=(-1.5,) * 3, box_hi=(1.5,) * 3, density_shift=0.0,
              hash_res=None, hash_log2_size=0, hash_tables=None):
    """features: dense feature grid, or None with hash_tables [4][2^log2][3]
    (the multi-level encoding); every grid tensor float32 or every float16."""
    dense = hash_tables if features is None else features
    if density.dtype == torch.float32 and dense.dtype == torch.float32:
        storage = CIC_F32
    elif density.dtype == torch.float16 and dense.dtype == torch.float16:
        storage = CIC_F16
    else:
        raise CicError(-1, "grid tensors must all be float32 or all float16")
    if not (density.is_contiguous() and dense.is_contiguous()):
        raise CicError(-1, "grids must be contiguous")
    levels = 0 if features is not None else int(hash_tables.shape[0])
    g = Grid((C.c_int32 * 3)(*density.shape), 12 if features is None else int(features.shape[-1]), storage,
             (C.c_float * 3)(*box_lo), (C.c_float * 3)(*box_hi), float(density_shift), density.data_ptr(),
             None if features is None else features.data_ptr(),
             occupancy.data_ptr() if occupancy is not None else None,
             levels, (C.c_int32 * 4)(*(hash_res or (0, 0, 0, 0))), int(hash_log2_size),
             None if hash_tables is None else hash_tables.data_ptr())
    g._keep = (density, features, occupancy, hash_tables)
    return g


def make_mlp(w, compute=CIC_F32):
    ts = [w[k] for k in ("w0", "b0", "w1", "b1", "w2", "b2")]
    for t in ts:
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise CicError(-1, "MLP weights must be contiguous float32")
    hidden, in_dim = ts[0].shape
    m = MLP(compute, int(in_dim), int(hidden), 4, *[t.data_ptr() for t in ts])
    m._keep = ts
    return m


def make_opts(n_samples, et_threshold=0.0, use_occupancy=False, bg=(1.0, 1.0, 1.0), void_acc=1e-4,
              order=CIC_ORDER_RAY, warp_max_angle=0.0):
    return Opts(int(n_samples), float(et_threshold), int(bool(use_occupancy)), (C.c_float * 3)(*bg),
                float(void_acc), int(order), float(warp_max_angle))


def make_camera(width, height, f, cx, cy, c2w):
    vals = [float(v) for v in torch.as_tensor(c2w, dtype=torch.float32).reshape(12).tolist()]
    return Camera(int(width), int(height), float(f), float(cx), float(cy), (C.c_float * 12)(*vals))


def workspace_bytes(op, n, grid=None, opts=None):
    return int(lib().cic_workspace_bytes(op, int(n), C.byref(grid) if grid is not None else None,
                                         C.byref(opts) if opts is not None else None))


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
def build_occupancy(grid, occ_sigma, occ):
    _check(lib().build_occupancy(C.byref(grid), C.c_float(occ_sigma), _ptr(occ), _stream()))


def generate_rays(cam, pix, rays_o, rays_d):
    n = rays_o.shape[0]
    _check(lib().generate_rays(C.byref(cam), C.c_int64(n), _ptr(pix), _ptr(rays_o), _ptr(rays_d), _stream()))


def render_rays(grid, mlp, opts, rays_o, rays_d, rgb, depth_t, acc, n_eval=None):
    n = rays_o.shape[0]
    ws, nb = _pass_workspace(OP_RENDER_RAYS, n, grid, opts, rays_o.device)
    _check(lib().render_rays(C.byref(grid), C.byref(mlp), C.byref(opts), C.c_int64(n), _ptr(rays_o),
                             _ptr(rays_d), _ptr(rgb), _ptr(depth_t), _ptr(acc), _ptr(n_eval), _ptr(ws),
                             C.c_size_t(nb), _stream()))


def render_frame(grid, mlp, opts, cam, rgb, depth_z, acc=None, n_eval=None):
    ws, nb = _pass_workspace(OP_RENDER_FRAME, cam.width * cam.height, grid, opts, rgb.device)
    _check(lib().render_frame(C.byref(grid), C.byref(mlp), C.byref(opts), C.byref(cam), _ptr(rgb),
                              _ptr(depth_z), _ptr(acc), _ptr(n_eval), _ptr(ws), C.c_size_t(nb), _stream()))


def warp_frame(ref_cam, tgt_cam, T, ref_rgb, ref_depth, tgt_rgb, tgt_depth, mask, src_index=None,
               max_angle_deg=0.0):
    nb = workspace_bytes(OP_WARP_FRAME, tgt_cam.width * tgt_cam.height)
    ws = workspace(nb, ref_rgb.device)
    Tc = (C.c_float * 12)(*[float(v) for v in torch.as_tensor(T, dtype=torch.float32).reshape(12).tolist()])
    _check(lib().warp_frame(C.byref(ref_cam), C.byref(tgt_cam), Tc, _ptr(ref_rgb), _ptr(ref_depth),
                            C.c_float(max_angle_deg), _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(mask), _ptr(src_index),
                            _ptr(ws), C.c_size_t(ws.numel()), _stream()))


def warp_frame_noalloc(ref_cam, tgt_cam, T, ref_rgb, ref_depth, tgt_rgb, tgt_depth, mask, src_index=None,
                       max_angle_deg=0.0):
    """warp_frame without a workspace (the library's own z-buffer array)."""
    Tc = (C.c_float * 12)(*[float(v) for v in torch.as_tensor(T, dtype=torch.float32).reshape(12).tolist()])
    _check(lib().warp_frame_noalloc(C.byref(ref_cam), C.byref(tgt_cam), Tc, _ptr(ref_rgb), _ptr(ref_depth),
                                    C.c_float(max_angle_deg), _ptr(tgt_rgb), _ptr(tgt_depth), _ptr(mask),
                                    _ptr(src_index), _stream()))


def render_frame_sparw(grid, mlp, opts, ref_cam, ref_rgb, ref_depth, tgt_cam, T, out_rgb, out_depth, mask,
                       n_masked=None, n_eval=None):
    nb = workspace_bytes(OP_RENDER_FRAME_SPARW, tgt_cam.width * tgt_cam.height, grid, opts)
    ws = workspace(nb, ref_rgb.device)
    Tc = (C.c_float * 12)(*[float(v) for v in torch.as_tensor(T, dtype=torch.float32).reshape(12).tolist()])
    _check(lib().render_frame_sparw(C.byref(grid), C.byref(mlp), C.byref(opts), C.byref(ref_cam), _ptr(ref_rgb),
                                    _ptr(ref_depth), C.byref(tgt_cam), Tc, _ptr(out_rgb), _ptr(out_depth),
                                    _ptr(mask), _ptr(n_masked), _ptr(n_eval), _ptr(ws), C.c_size_t(ws.numel()),
                                    _stream()))


def render_backward(grid, mlp, opts, rays_o, rays_d, d_rgb, d_depth_t, d_acc, grads):
    n = rays_o.shape[0]
    ws, nb = _pass_workspace(OP_RENDER_BACKWARD, n, grid, opts, rays_o.device)
    _check(lib().render_backward(C.byref(grid), C.byref(mlp), C.byref(opts), C.c_int64(n), _ptr(rays_o),
                                 _ptr(rays_d), _ptr(d_rgb), _ptr(d_depth_t), _ptr(d_acc),
                                 _ptr(grads["density"]), _ptr(grads["features"]), _ptr(grads["w0"]),
                                 _ptr(grads["b0"]), _ptr(grads["w1"]), _ptr(grads["b1"]), _ptr(grads["w2"]),
                                 _ptr(grads["b2"]), _ptr(ws), C.c_size_t(nb), _stream()))


def timing_enable(on=True):
    _check(lib().cic_timing_enable(1 if on else 0))


def timing_read():
    """{stage: (milliseconds, launches)} since the last timing_enable."""
    n = len(STAGES)
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(lib().cic_timing_read(ms, cnt, n))
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}


def _pose12(p):
    a = (C.c_float * 12)()
    v = [float(x) for x in (p.reshape(-1).tolist() if hasattr(p, "reshape") else list(p))]
    if len(v) != 12:
        raise CicError(-1, "a pose has 12 values (row-major 3x4)")
    a[:] = v
    return a


def extrapolate_pose(c2w_prev, c2w_cur, steps):
    out = (C.c_float * 12)()
    _check(lib().cic_extrapolate_pose(_pose12(c2w_prev), _pose12(c2w_cur), C.c_float(steps), out))
    return list(out)


def relative_pose(c2w_ref, c2w_tgt):
    out = (C.c_float * 12)()
    _check(lib().cic_relative_pose(_pose12(c2w_ref), _pose12(c2w_tgt), out))
    return list(out)


# CU-partitioned stream pairs (target, reference) per (device, CUs per XCD),
# created on first use and destroyed by release(); a plain second stream for
# the shared-chip overlap is a torch stream per device.
_cu_streams = {}
_side_streams = {}


def cu_streams(target_cus_per_xcd, device=None):
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    key = (dev, int(target_cus_per_xcd))
    with _lock:
        pair = _cu_streams.get(key)
    if pair is None:
        out = []
        with torch.cuda.device(dev):
            for role in (0, 1):
                h = C.c_void_p()
                rc = lib().cic_stream_create_cu_masked(C.c_int32(target_cus_per_xcd), C.c_int32(role), C.byref(h))
                if rc != 0:
                    for s in out:
                        lib().cic_stream_destroy(s)
                    raise CicError(rc, last_error())
                out.append(h)
        pair = (out[0], out[1])
        with _lock:
            _cu_streams[key] = pair
    return pair


def side_stream(device=None):
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    with _lock:
        st = _side_streams.get(dev)
        if st is None:
            st = torch.cuda.Stream(device=dev)
            _side_streams[dev] = st
    return st


def render_sequence(grid, mlp, opts, cams, window, lead, flags, rgb, depth_z, mask, n_masked=None, n_eval=None,
                    target_cus_per_xcd=0):
    """cams: sequence of Camera structs; returns the reference poses.  With
    CIC_SEQ_OVERLAP the references run on a second stream (a torch stream, or
    with target_cus_per_xcd > 0 the CU-masked pair, targets on the first);
    the call is ordered after earlier work on the current stream and later
    work on it waits for the whole sequence."""
    n = len(cams)
    arr = (Camera * max(n, 1))(*cams)
    n_win = (n - 1 + window - 1) // window if n > 1 and window > 0 else 0
    refs = (C.c_float * (12 * max(n_win - 1, 1)))()
    npix = cams[0].width * cams[0].height if n else 0
    nb = workspace_bytes(OP_RENDER_SEQUENCE, npix, grid, opts)
    ws = workspace(nb, rgb.device)
    cur = torch.cuda.current_stream(rgb.device)
    s_tgt, s_ref = C.c_void_p(cur.cuda_stream), None
    masked = None
    if flags & CIC_SEQ_OVERLAP:
        if target_cus_per_xcd > 0:
            pair = cu_streams(target_cus_per_xcd, rgb.device)
            s_tgt, s_ref = pair
            masked = torch.cuda.ExternalStream(pair[0].value, device=rgb.device)
        else:
            s_ref = C.c_void_p(side_stream(rgb.device).cuda_stream)
    if masked is not None:
        # the target stream starts after the caller's earlier work
        masked.wait_stream(cur)
    _check(lib().render_sequence(C.byref(grid), C.byref(mlp), C.byref(opts), arr, C.c_int32(n), C.c_int32(window),
                                 C.c_float(lead), C.c_int32(flags), C.c_int32(target_cus_per_xcd), _ptr(rgb),
                                 _ptr(depth_z), _ptr(mask),
                                 _ptr(n_masked), refs, _ptr(n_eval), _ptr(ws), C.c_size_t(ws.numel()), s_tgt, s_ref))
    if masked is not None:
        # the caller's later work waits for the whole sequence
        cur.wait_stream(masked)
    return [list(refs[12 * i:12 * i + 12]) for i in range(max(n_win - 1, 0))]


def timing_frames(cap=4096):
    """Completion times (ms) of the frames of the last render_sequence call
    made while timing was on."""
    ms = (C.c_double * cap)()
    n = lib().cic_timing_frames(ms, cap)
    if n < 0:
        raise CicError(n, last_error())
    return list(ms[:min(n, cap)])


def render_frame_ds(grid, mlp, opts, cam, factor, rgb, n_eval=None):
    nb = workspace_bytes(OP_RENDER_FRAME_DS, cam.width * cam.height, grid, opts)
    ws = workspace(nb, rgb.device)
    _check(lib().render_frame_ds(C.byref(grid), C.byref(mlp), C.byref(opts), C.byref(cam), C.c_int32(factor),
                                 _ptr(rgb), _ptr(n_eval), _ptr(ws), C.c_size_t(ws.numel()), _stream()))
