"""Shared setup for the GPU parity tests: the same seeded inputs go to the
HIP library and to the oracle."""
import numpy as np
import torch

import oracle
import synth

BG = (1.0, 1.0, 1.0)
# float32 GPU vs float64 oracle: colour and distance tolerance
TOL = 1e-5
# pixels whose oracle transmittance at a termination decision lies within
# this relative band of the threshold may legitimately stop one sample
# earlier or later in float32; their bound is the size of one skipped
# sample's contribution (<= T ~ threshold) twice over
FLIP_BAND = 1e-4
FLIP_TOL = 3e-4


def print_case(msg):
    print("[case] " + msg, flush=True)


class Pair:
    """One scene on both sides."""

    def __init__(self, res, seed=0, mlp_seed=1, bias_std=0.0, occupancy=False, storage=torch.float32,
                 shift=synth.DENSITY_SHIFT, dens=None, feats=None, mlp=None):
        import paper_2404_11852_amd as cic
        if dens is None:
            dens, feats = synth.make_scene(res, seed=seed)
        if mlp is None:
            mlp = synth.make_mlp(mlp_seed, bias_std=bias_std)
        self.dens, self.feats, self.mlp = dens, feats, mlp
        self.gpu = cic.Model(dens, feats, mlp, device="cuda", storage=storage, density_shift=shift)
        if storage == torch.float16:
            # the oracle sees exactly the values the GPU reads
            dens_o = dens.astype(np.float16).astype(np.float32)
            feats_o = feats.astype(np.float16).astype(np.float32)
        else:
            dens_o, feats_o = dens, feats
        self.orc = oracle.Model(dens_o, feats_o, mlp, density_shift=shift)
        if occupancy:
            self.gpu.build_occupancy(synth.OCC_SIGMA)
            self.orc.set_occupancy(oracle.build_occupancy(self.orc, synth.OCC_SIGMA))


def cams(W, H, pose):
    import paper_2404_11852_amd as cic
    f, cx, cy = synth.intrinsics(W, H)
    c2w = synth.as_f32(pose)
    return cic.make_camera(W, H, f, cx, cy, c2w), oracle.camera(W, H, f, cx, cy, c2w)


def to_np(t):
    return t.detach().cpu().numpy()


def compare(got, want, margin=None, tol=TOL, flip_tol=FLIP_TOL, what="rgb"):
    """Element-wise |got - want| <= tol, except rows whose oracle margin is
    inside the flip band (then flip_tol).  Returns (max err clean, n flagged)."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    err = np.abs(got - want)
    if err.ndim > 1:
        err = err.max(axis=tuple(range(1, err.ndim)))
    flagged = np.zeros(err.shape, bool) if margin is None else (margin < FLIP_BAND)
    clean = err[~flagged]
    worst = float(clean.max()) if clean.size else 0.0
    assert worst <= tol, "%s: max error %.3g > %.3g at %s" % (what, worst, tol, np.argmax(np.where(flagged, 0, err)))
    if flagged.any():
        assert float(err[flagged].max()) <= flip_tol, "%s: flagged rows error %.3g" % (what, err[flagged].max())
    return worst, int(flagged.sum())


def check_sparw_frame(rgb, dz, mask, orc_model, oop, ref_ocam, ref_rgb32, ref_dz32, tgt_ocam, T, max_angle=0.0,
                      sample=None, seed=0):
    """Element-wise parity of one SpaRW target frame (GPU arrays rgb [P][3],
    z-depth [P], mask [P]) against the oracle driven by the same float32
    reference frame and transform: the hole mask, and the colour and depth
    of every warped pixel, are bit-exact; re-rendered (hole) pixels meet the
    render tolerance (flip band apart), all of them or a seeded sample of
    `sample`.  Returns (holes, holes checked)."""
    wr, wd, wm, _ = oracle.warp(ref_ocam, tgt_ocam, T, ref_rgb32, ref_dz32, max_angle)
    assert np.array_equal(mask, wm), "mask differs at %d pixels" % int((mask != wm).sum())
    keep = wm == 0
    assert np.array_equal(rgb[keep], wr[keep]), "warped colour"
    assert np.array_equal(np.nan_to_num(dz[keep], posinf=-1.0), np.nan_to_num(wd[keep], posinf=-1.0)), "warped depth"
    holes = np.nonzero(wm)[0]
    chk = holes
    if sample is not None and holes.size > sample:
        chk = np.sort(np.random.default_rng(seed).choice(holes, sample, replace=False))
    if chk.size:
        orgb, odz, oacc, diag = oracle.render_pixels(orc_model, oop, tgt_ocam, chk)
        compare(rgb[chk], orgb, margin=diag["margin"])
        am = diag["acc_margin"]
        sure = am > 1e-3
        assert np.array_equal(np.isinf(dz[chk])[sure], np.isinf(odz)[sure]), "void decision"
        fin = sure & np.isfinite(odz)
        if fin.any():
            derr = np.abs(dz[chk][fin] - odz[fin]) * oacc[fin] / (1 + np.abs(odz[fin]))
            assert derr.max() < 2e-5, derr.max()
    return int(holes.size), int(chk.size)
