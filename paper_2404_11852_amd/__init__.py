"""MI355X (gfx950) renderer for dense-grid NeRF with sparse radiance warping.

Thin Python layer over libcicero.so: tensors in, tensors out, the work is
done by the HIP kernels behind the C interface in include/cicero.h.
"""
import torch

from . import _lib
from ._lib import (CIC_F16, CIC_F32, CIC_BF16, CIC_ORDER_RAY, CIC_ORDER_VOXEL, CicError, extrapolate_pose,
                   make_camera, make_opts, relative_pose, set_workspace_limit)

__all__ = ["Model", "make_camera", "make_opts", "CicError", "render_rays", "render_frame", "warp_frame",
           "render_frame_sparw", "render_sequence", "render_temporal", "render_frame_ds", "render_backward",
           "generate_rays", "build_occupancy", "set_workspace_limit",
           "extrapolate_pose", "relative_pose", "RenderRays",
           "CIC_F32", "CIC_F16", "CIC_BF16", "CIC_ORDER_RAY", "CIC_ORDER_VOXEL"]


class Model:
    """Device copies of a dense grid (raw density + 12 feature channels) and
    the 39-128-128-3 MLP, plus the C structs that describe them."""

    def __init__(self, density, features, mlp, device="cuda", storage=torch.float32, density_shift=0.0,
                 box_lo=(-1.5,) * 3, box_hi=(1.5,) * 3, compute=CIC_F32, hash_enc=None):
        """hash_enc: None, or {'res': 4 level resolutions, 'log2_size': int,
        'tables': [4][2^log2_size][3]} for the multi-level encoding (then
        `features` is ignored)."""
        self.device = torch.device(device)
        self.density = torch.as_tensor(density, dtype=torch.float32).to(self.device).to(storage).contiguous()
        self.hash = None
        if hash_enc is not None:
            self.hash = dict(hash_enc)
            self.hash["tables"] = torch.as_tensor(hash_enc["tables"], dtype=torch.float32).to(self.device) \
                .to(storage).contiguous()
            self.features = None
        else:
            self.features = torch.as_tensor(features, dtype=torch.float32).to(self.device).to(storage).contiguous()
        self.w = {k: torch.as_tensor(v, dtype=torch.float32).to(self.device).contiguous() for k, v in mlp.items()}
        self.box_lo, self.box_hi = tuple(box_lo), tuple(box_hi)
        self.density_shift = float(density_shift)
        self.occupancy = None
        self.compute = compute
        self._rebuild()

    def _rebuild(self):
        h = self.hash or {}
        self.grid = _lib.make_grid(self.density, self.features, self.occupancy, self.box_lo, self.box_hi,
                                   self.density_shift, h.get("res"), h.get("log2_size", 0), h.get("tables"))
        self.mlp = _lib.make_mlp(self.w, self.compute)

    def build_occupancy(self, occ_sigma=1e-2):
        r = self.density.shape
        occ = torch.empty((r[0] - 1, r[1] - 1, r[2] - 1), dtype=torch.uint8, device=self.device)
        _lib.build_occupancy(self.grid, occ_sigma, occ)
        self.set_occupancy(occ)
        return occ

    def set_occupancy(self, occ):
        self.occupancy = None if occ is None else occ.to(self.device, torch.uint8).contiguous()
        self._rebuild()


def _f32(n, *shape, device):
    return torch.empty((n,) + shape, dtype=torch.float32, device=device)


def generate_rays(cam, pix=None, device="cuda"):
    n = cam.width * cam.height if pix is None else int(pix.numel())
    o = _f32(n, 3, device=device)
    d = _f32(n, 3, device=device)
    _lib.generate_rays(cam, None if pix is None else pix.to(device, torch.int64).contiguous(), o, d)
    return o, d


def build_occupancy(model, occ_sigma=1e-2):
    return model.build_occupancy(occ_sigma)


def render_rays(model, opts, rays_o, rays_d, n_eval=None):
    n = rays_o.shape[0]
    dev = rays_o.device
    rgb, dep, acc = _f32(n, 3, device=dev), _f32(n, device=dev), _f32(n, device=dev)
    _lib.render_rays(model.grid, model.mlp, opts, rays_o.contiguous(), rays_d.contiguous(), rgb, dep, acc, n_eval)
    return rgb, dep, acc


def render_frame(model, opts, cam, n_eval=None):
    n = cam.width * cam.height
    dev = model.device
    rgb, dz, acc = _f32(n, 3, device=dev), _f32(n, device=dev), _f32(n, device=dev)
    _lib.render_frame(model.grid, model.mlp, opts, cam, rgb, dz, acc, n_eval)
    return rgb, dz, acc


def warp_frame(ref_cam, tgt_cam, T, ref_rgb, ref_depth, with_src=False, max_angle_deg=0.0):
    n = tgt_cam.width * tgt_cam.height
    dev = ref_rgb.device
    rgb, dz = _f32(n, 3, device=dev), _f32(n, device=dev)
    mask = torch.empty(n, dtype=torch.uint8, device=dev)
    src = torch.empty(n, dtype=torch.int32, device=dev) if with_src else None
    _lib.warp_frame(ref_cam, tgt_cam, T, ref_rgb.contiguous(), ref_depth.contiguous(), rgb, dz, mask, src,
                    max_angle_deg)
    return (rgb, dz, mask, src) if with_src else (rgb, dz, mask)


def render_frame_sparw(model, opts, ref_cam, ref_rgb, ref_depth, tgt_cam, T, n_eval=None):
    n = tgt_cam.width * tgt_cam.height
    dev = ref_rgb.device
    rgb, dz = _f32(n, 3, device=dev), _f32(n, device=dev)
    mask = torch.empty(n, dtype=torch.uint8, device=dev)
    nm = torch.zeros(1, dtype=torch.int64, device=dev)
    _lib.render_frame_sparw(model.grid, model.mlp, opts, ref_cam, ref_rgb.contiguous(), ref_depth.contiguous(),
                            tgt_cam, T, rgb, dz, mask, nm, n_eval)
    return rgb, dz, mask, nm


def render_sequence(model, opts, cams, window, lead=-1.0, overlap=True, target_cus_per_xcd=0, n_eval=None):
    """Render a trajectory (list of cameras of one size) with off-trajectory
    references every `window` targets.  Returns rgb [F, P, 3], z-depth
    [F, P], mask [F, P], rendered-pixel counts [F] and the reference poses
    (list of 12-value rows)."""
    n = len(cams)
    npix = cams[0].width * cams[0].height
    dev = model.device
    rgb = torch.empty((n, npix, 3), dtype=torch.float32, device=dev)
    dz = torch.empty((n, npix), dtype=torch.float32, device=dev)
    mask = torch.empty((n, npix), dtype=torch.uint8, device=dev)
    nm = torch.zeros(n, dtype=torch.int64, device=dev)
    refs = _lib.render_sequence(model.grid, model.mlp, opts, cams, window, lead,
                                _lib.CIC_SEQ_OVERLAP if overlap else 0, rgb, dz, mask, nm, n_eval,
                                target_cus_per_xcd)
    return rgb, dz, mask, nm, refs


def render_temporal(model, opts, cams, window, n_eval=None):
    """Temp-N variant: full renders every `window` frames, every other frame
    warped from the previous output.  Returns rgb, z-depth, mask, counts."""
    n = len(cams)
    npix = cams[0].width * cams[0].height
    dev = model.device
    rgb = torch.empty((n, npix, 3), dtype=torch.float32, device=dev)
    dz = torch.empty((n, npix), dtype=torch.float32, device=dev)
    mask = torch.empty((n, npix), dtype=torch.uint8, device=dev)
    nm = torch.zeros(n, dtype=torch.int64, device=dev)
    _lib.render_sequence(model.grid, model.mlp, opts, cams, window, 0.0, _lib.CIC_SEQ_TEMPORAL, rgb, dz, mask, nm,
                         n_eval)
    return rgb, dz, mask, nm


def render_frame_ds(model, opts, cam, factor=2, n_eval=None):
    """DS-s variant: render at 1/factor resolution, upsample bilinearly."""
    rgb = _f32(cam.width * cam.height, 3, device=model.device)
    _lib.render_frame_ds(model.grid, model.mlp, opts, cam, factor, rgb, n_eval)
    return rgb


def render_backward(model, opts, rays_o, rays_d, d_rgb, d_depth_t=None, d_acc=None, grads=None):
    """Accumulate gradients of the rendering into `grads` (created zeroed if
    None); returns the dict.  Dense feature grids only."""
    if model.hash is not None:
        raise CicError(-1, "render_backward does not support the multi-level encoding")
    if grads is None:
        grads = {"density": torch.zeros(model.density.shape, dtype=torch.float32, device=model.device),
                 "features": torch.zeros(model.features.shape, dtype=torch.float32, device=model.device)}
        for k, v in model.w.items():
            grads[k] = torch.zeros_like(v)
    _lib.render_backward(model.grid, model.mlp, opts, rays_o.contiguous(), rays_d.contiguous(), d_rgb.contiguous(),
                         None if d_depth_t is None else d_depth_t.contiguous(),
                         None if d_acc is None else d_acc.contiguous(), grads)
    return grads


class _Bound:
    """Grid and MLP descriptors built from given tensors (the autograd
    leaves), with the occupancy, box and shift of a model."""

    def __init__(self, model, density, features, w):
        for t in (density, features, *w.values()):
            if t.device != model.density.device or t.dtype != torch.float32 or not t.is_contiguous():
                raise CicError(-1, "RenderRays takes contiguous float32 tensors on the model's device")
        if density.shape != model.density.shape or features.shape != model.features.shape:
            raise CicError(-1, "RenderRays: grid shapes differ from the model's")
        for k, v in w.items():
            if v.shape != model.w[k].shape:
                raise CicError(-1, "RenderRays: %s has shape %s, the model's %s" % (k, tuple(v.shape),
                                                                                   tuple(model.w[k].shape)))
        self.device = model.device
        self.hash = None
        self.density, self.features, self.w = density, features, w
        self.grid = _lib.make_grid(density, features, model.occupancy, model.box_lo, model.box_hi,
                                   model.density_shift)
        self.mlp = _lib.make_mlp(w, CIC_F32)


class RenderRays(torch.autograd.Function):
    """rgb, depth_t, acc = RenderRays.apply(density, features, w0, b0, w1, b1,
    w2, b2, rays_o, rays_d, model, opts).  Renders with the tensors passed
    in (float32, contiguous, on the model's device, the model's shapes); the
    model supplies the occupancy, box and density shift.  The forward keeps
    only its inputs; the backward recomputes each ray inside
    render_backward."""

    @staticmethod
    def forward(ctx, density, features, w0, b0, w1, b1, w2, b2, rays_o, rays_d, model, opts):
        if model.hash is not None:
            raise CicError(-1, "RenderRays does not support the multi-level encoding")
        bound = _Bound(model, density, features, {"w0": w0, "b0": b0, "w1": w1, "b1": b1, "w2": w2, "b2": b2})
        ctx.bound, ctx.opts = bound, opts
        ctx.save_for_backward(density, features, w0, b0, w1, b1, w2, b2, rays_o, rays_d)
        return render_rays(bound, opts, rays_o, rays_d)

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_acc):
        saved = ctx.saved_tensors   # raises if a leaf was modified in place since the forward
        rays_o, rays_d = saved[8], saved[9]
        g = render_backward(ctx.bound, ctx.opts, rays_o, rays_d, g_rgb,
                            None if g_depth is None else g_depth, None if g_acc is None else g_acc)
        return (g["density"], g["features"], g["w0"], g["b0"], g["w1"], g["b1"], g["w2"], g["b2"],
                None, None, None, None)
