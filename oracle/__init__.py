"""Python access to the plain CPU oracle (oracle/cicero_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product package.  The C file
is built with gcc (-O2 -ffp-contract=off, OpenMP) into oracle/liboracle.so.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cicero_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the oracle shared library with gcc."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-variable", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class Hash(C.Structure):
    _fields_ = [("levels", C.c_int32), ("feat_per_level", C.c_int32), ("res", C.c_int32 * 8),
                ("log2_size", C.c_int32), ("tables", C.c_void_p)]


class Grid(C.Structure):
    _fields_ = [("res", C.c_int32 * 3), ("n_feat", C.c_int32),
                ("box_lo", C.c_float * 3), ("box_hi", C.c_float * 3),
                ("density_shift", C.c_float),
                ("density", C.c_void_p), ("features", C.c_void_p), ("occ", C.c_void_p),
                ("hash", C.c_void_p)]


class MLP(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("hidden", C.c_int32), ("out_dim", C.c_int32),
                ("pe_freqs", C.c_int32),
                ("w0", C.c_void_p), ("b0", C.c_void_p), ("w1", C.c_void_p), ("b1", C.c_void_p),
                ("w2", C.c_void_p), ("b2", C.c_void_p), ("round_bf16", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("et_threshold", C.c_float),
                ("use_occupancy", C.c_int32), ("bg", C.c_float * 3), ("void_acc", C.c_float),
                ("warp_max_angle", C.c_float)]


class Cam(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("f", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("c2w", C.c_float * 12)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Model:
    """Holds contiguous arrays plus the ctypes structs that point at them."""

    def __init__(self, density, features, mlp, box_lo=(-1.5,) * 3, box_hi=(1.5,) * 3,
                 density_shift=0.0, occ=None, pe_freqs=4, round_bf16=False, hash_enc=None):
        """hash_enc: None (features from the dense grid `features`) or a dict
        with 'res' (cells per axis of each level), 'log2_size' and 'tables'
        [L][2^log2_size][F]; then `features` is ignored."""
        self.density = _f32(density)
        res = self.density.shape
        self.hash = None
        if hash_enc is not None:
            self.tables = _f32(hash_enc["tables"])
            L, T, F = self.tables.shape
            assert T == 1 << int(hash_enc["log2_size"]) and L == len(hash_enc["res"]) <= 8
            self.hash = Hash(L, F, (C.c_int32 * 8)(*hash_enc["res"]), int(hash_enc["log2_size"]),
                             _p(self.tables).value)
            self.features = np.zeros((1,), np.float32)
            n_feat = L * F
        else:
            self.features = _f32(features)
            n_feat = self.features.shape[-1]
        self.occ = None if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        self.grid = Grid((C.c_int32 * 3)(*res), n_feat, (C.c_float * 3)(*box_lo),
                         (C.c_float * 3)(*box_hi), float(np.float32(density_shift)),
                         _p(self.density).value, _p(self.features).value,
                         None if self.occ is None else _p(self.occ).value,
                         None if self.hash is None else C.addressof(self.hash))
        self.w = {k: _f32(v) for k, v in mlp.items()}
        hidden, in_dim = self.w["w0"].shape
        out_dim = self.w["w2"].shape[0]
        assert in_dim == n_feat + 3 + 6 * pe_freqs
        assert in_dim <= 256 and hidden <= 1024 and n_feat <= 64 and out_dim <= 8
        self.mlp = MLP(in_dim, hidden, out_dim, pe_freqs,
                       *[_p(self.w[k]).value for k in ("w0", "b0", "w1", "b1", "w2", "b2")],
                       int(bool(round_bf16)))

    def set_occupancy(self, occ):
        self.occ = None if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        self.grid.occ = None if self.occ is None else _p(self.occ).value


def opts(n_samples, et_threshold=0.0, use_occupancy=False, bg=(1.0, 1.0, 1.0), void_acc=1e-4,
         warp_max_angle=0.0):
    return Opts(int(n_samples), float(et_threshold), int(bool(use_occupancy)),
                (C.c_float * 3)(*bg), float(void_acc), float(warp_max_angle))


def camera(width, height, f, cx, cy, c2w):
    return Cam(int(width), int(height), float(f), float(cx), float(cy),
               (C.c_float * 12)(*[float(v) for v in np.asarray(c2w, dtype=np.float32).reshape(12)]))


def set_threads(n):
    lib().orc_set_num_threads(int(n))


def num_threads():
    return lib().orc_num_threads()


def generate_rays(cam, pix=None):
    n = cam.width * cam.height if pix is None else len(pix)
    pix = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    o = np.empty((n, 3), np.float32)
    d = np.empty((n, 3), np.float32)
    lib().orc_generate_rays(C.byref(cam), C.c_int64(n), _p(pix), _p(o), _p(d))
    return o, d


def ray_box(o, d, lo=(-1.5,) * 3, hi=(1.5,) * 3):
    o, d = _f32(o), _f32(d)
    n = o.shape[0]
    tn = np.empty(n, np.float32)
    tf = np.empty(n, np.float32)
    hit = np.empty(n, np.uint8)
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    lib().orc_ray_box(C.c_int64(n), _p(o), _p(d), _p(lo), _p(hi), _p(tn), _p(tf), _p(hit))
    return tn, tf, hit.astype(bool)


def build_occupancy(model, occ_sigma=1e-2):
    r = model.density.shape
    occ = np.empty((r[0] - 1, r[1] - 1, r[2] - 1), np.uint8)
    lib().orc_build_occupancy(C.byref(model.grid), C.c_float(occ_sigma), _p(occ))
    return occ


def trilerp(model, values, pos):
    values = _f32(values)
    n_ch = 1 if values.ndim == 3 else values.shape[-1]
    pos = _f32(pos).reshape(-1, 3)
    out = np.empty((pos.shape[0], n_ch), np.float64)
    lib().orc_trilerp(C.byref(model.grid), _p(values), C.c_int(n_ch), C.c_int64(pos.shape[0]),
                      _p(pos), _p(out))
    return out


def trilerp_scatter(model, n_ch, pos, y):
    pos = _f32(pos).reshape(-1, 3)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(pos.shape[0], n_ch)
    r = model.density.shape
    out = np.zeros(r + (n_ch,), np.float64)
    lib().orc_trilerp_scatter(C.byref(model.grid), C.c_int(n_ch), C.c_int64(pos.shape[0]),
                              _p(pos), _p(y), _p(out))
    return out


def mlp_forward(model, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty((x.shape[0], model.mlp.out_dim), np.float64)
    lib().orc_mlp_forward(C.byref(model.mlp), C.c_int64(x.shape[0]), _p(x), _p(out))
    return out


def mlp_input(model, feat, d):
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    d = _f32(d)
    n = feat.shape[0]
    x = np.empty((n, model.mlp.in_dim), np.float64)
    lib().orc_mlp_input(C.byref(model.mlp), C.c_int(feat.shape[1]), C.c_int64(n), _p(feat), _p(d), _p(x))
    return x


def render_rays(model, op, o, d, diagnostics=False, flip=False):
    """flip=True (a model in bfloat16 mode; implies diagnostics): diag['flip']
    as in render_pixels."""
    o, d = _f32(o), _f32(d)
    n = o.shape[0]
    rgb = np.empty((n, 3), np.float64)
    dep = np.empty(n, np.float64)
    acc = np.empty(n, np.float64)
    ne = np.empty(n, np.int32)
    mg = np.empty(n, np.float64)
    sig = np.empty(n, np.uint64)
    fl = np.empty(n, np.float64) if flip else None
    lib().orc_render_rays(C.byref(model.grid), C.byref(model.mlp), C.byref(op), C.c_int64(n),
                          _p(o), _p(d), _p(rgb), _p(dep), _p(acc), _p(ne), _p(mg), _p(sig), _p(fl))
    if diagnostics or flip:
        diag = {"n_eval": ne, "margin": mg, "relu_sig": sig}
        if flip:
            diag["flip"] = fl
        return rgb, dep, acc, diag
    return rgb, dep, acc


def render_pixels(model, op, cam, pix=None, flip=False):
    """diag['flip'] (with flip=True, for a model in bfloat16 mode): per pixel,
    the largest colour change one bfloat16 rounding step of one MLP input
    value could cause, weighted by its sample's compositing weight."""
    n = cam.width * cam.height if pix is None else len(pix)
    pix = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    rgb = np.empty((n, 3), np.float64)
    dz = np.empty(n, np.float64)
    acc = np.empty(n, np.float64)
    ne = np.empty(n, np.int32)
    mg = np.empty(n, np.float64)
    am = np.empty(n, np.float64)
    fl = np.empty(n, np.float64) if flip else None
    lib().orc_render_pixels(C.byref(model.grid), C.byref(model.mlp), C.byref(op), C.byref(cam),
                            C.c_int64(n), _p(pix), _p(rgb), _p(dz), _p(acc), _p(ne), _p(mg), _p(am), _p(fl))
    diag = {"n_eval": ne, "margin": mg, "acc_margin": am}
    if flip:
        diag["flip"] = fl
    return rgb, dz, acc, diag


def warp(ref_cam, tgt_cam, T, ref_rgb, ref_depth, max_angle_deg=0.0):
    ref_rgb = _f32(ref_rgb).reshape(-1, 3)
    ref_depth = _f32(ref_depth).reshape(-1)
    T = _f32(T).reshape(12)
    n = tgt_cam.width * tgt_cam.height
    rgb = np.empty((n, 3), np.float32)
    dep = np.empty(n, np.float32)
    mask = np.empty(n, np.uint8)
    src = np.empty(n, np.int32)
    lib().orc_warp_angle(C.byref(ref_cam), C.byref(tgt_cam), _p(T), _p(ref_rgb), _p(ref_depth),
                         C.c_float(max_angle_deg), _p(rgb), _p(dep), _p(mask), _p(src))
    return rgb, dep, mask, src


def sparw(model, op, ref_cam, ref_rgb, ref_depth, tgt_cam, T):
    ref_rgb = _f32(ref_rgb).reshape(-1, 3)
    ref_depth = _f32(ref_depth).reshape(-1)
    T = _f32(T).reshape(12)
    n = tgt_cam.width * tgt_cam.height
    rgb = np.empty((n, 3), np.float64)
    dep = np.empty(n, np.float64)
    mask = np.empty(n, np.uint8)
    nm = C.c_int64(0)
    lib().orc_sparw(C.byref(model.grid), C.byref(model.mlp), C.byref(op), C.byref(ref_cam),
                    _p(ref_rgb), _p(ref_depth), C.byref(tgt_cam), _p(T), _p(rgb), _p(dep),
                    _p(mask), C.byref(nm))
    return rgb, dep, mask, nm.value


def render_backward(model, op, o, d, d_rgb, d_depth_t=None, d_acc=None):
    o, d = _f32(o), _f32(d)
    n = o.shape[0]
    d_rgb = np.ascontiguousarray(d_rgb, dtype=np.float64).reshape(n, 3)
    dd = None if d_depth_t is None else np.ascontiguousarray(d_depth_t, dtype=np.float64)
    da = None if d_acc is None else np.ascontiguousarray(d_acc, dtype=np.float64)
    g = {"density": np.zeros(model.density.shape, np.float64),
         "features": np.zeros(model.features.shape, np.float64)}
    for k in ("w0", "b0", "w1", "b1", "w2", "b2"):
        g[k] = np.zeros(model.w[k].shape, np.float64)
    rgb = np.empty((n, 3), np.float64)
    dep = np.empty(n, np.float64)
    acc = np.empty(n, np.float64)
    lib().orc_render_backward(C.byref(model.grid), C.byref(model.mlp), C.byref(op), C.c_int64(n),
                              _p(o), _p(d), _p(d_rgb), _p(dd), _p(da),
                              _p(g["density"]), _p(g["features"]),
                              _p(g["w0"]), _p(g["b0"]), _p(g["w1"]), _p(g["b1"]),
                              _p(g["w2"]), _p(g["b2"]), _p(rgb), _p(dep), _p(acc))
    return g, (rgb, dep, acc)


def encode(model, pos):
    """Feature vectors [n][n_feat] (float64) of float32 positions [n][3]:
    the multi-level encoding when the model has one, else the dense grid."""
    pos = _f32(pos).reshape(-1, 3)
    out = np.empty((pos.shape[0], model.grid.n_feat), np.float64)
    lib().orc_encode(C.byref(model.grid), C.c_int64(pos.shape[0]), _p(pos), _p(out))
    return out
